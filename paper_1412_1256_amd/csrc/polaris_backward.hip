// polaris_backward.hip -- gfx950 kernels of the differentiation form: the learnable window and the
// adjoint of the path (window -> FFT -> cross power -> integration -> calibration -> Eq. 2).
//
// Notation: for a complex quantity Z, Gb(Z) = dL/dRe Z + i dL/dIm Z.  With C = Fi M Fi^H, Fi = (G J)^-1,
// M = A / (F s), s = sum w^2 and the Stokes rows of Eq. 2 (Sec. 2.1) m_P acting on [C_xx, C_xy, C_yx, C_yy]:
//   Gb(C_ij) = sum_P g_P conj(m_P,ij);  Gb(M) = Fi^H Gb(C) Fi;  Gb(Fi) = (Gb(C) + Gb(C)^H) Fi M;
//   Gb(E) = -Fi^H Gb(Fi) Fi^H for E = G J;  Gb(G) = diag(Gb(E) J^H);  Gb(J) = G^H Gb(E);
//   Gb(A) = Gb(M) / (F s), and the normaliser gives dL/dw[n] a term -2 w[n] Re tr(Gb(M)^H M) / s;
//   per frame, [X; Y] = v gives Gb(v) = 2 Gb(A) v (Gb(A) is Hermitian) and
//   dL/dw[n] += x[n] Re sum_{k<C} Gb(X_k) e^{+2 pi i n k/N} + (same for y).
// The frame transforms are recomputed instead of stored: the column pass runs again, the backward row pass
// transforms each row, applies the per-channel adjoint, and runs the inverse row transform; the backward
// column pass runs the inverse column transform and multiplies by the re-read samples.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "polaris_device.h"
#include "polaris_internal.h"

namespace ps {

#define PS_LAUNCH(kernel, grid, block, l, ...) \
  hipExtLaunchKernelGGL(kernel, grid, block, 0, (l).stream, (l).start, (l).stop, 0, __VA_ARGS__)

// ------------------------------------------------------------------------------------------------
// learnable window: taps theta_0 .. theta_{T-1} at u = n (T - 1)/(N - 1), linear in between
// ------------------------------------------------------------------------------------------------

__device__ __forceinline__ void tap_position(int64_t n, int64_t N, int T, int& j, double& t) {
  const double u = (double)n * (double)(T - 1) / (double)(N - 1);
  int jj = (int)floor(u);
  if (jj > T - 2) jj = T - 2;
  j = jj;
  t = u - (double)jj;
}

__device__ __forceinline__ double tap_window(const float* __restrict__ taps, int64_t n, int64_t N, int T) {
  int j;
  double t;
  tap_position(n, N, T, j, t);
  return (1.0 - t) * (double)taps[j] + t * (double)taps[j + 1];
}

// two points per thread: every CU takes part (16 points per thread left 16 workgroups at 2^16 points, each
// thread waiting on 16 dependent FP64 divisions)
constexpr int kWinThreads = 256, kWinPerThread = 2;

// w[n] in FP32 for the transforms, and per-block partial sums of w^2 in FP64 (fixed order)
__global__ void __launch_bounds__(kWinThreads) k_window_taps(WinArgs a) {
  __shared__ double red[kWinThreads];
  if (blockIdx.x == 0)
    for (int i = (int)threadIdx.x; i < a.n_taps; i += kWinThreads) a.taps_copy[i] = a.taps[i];
  const int64_t base = (int64_t)blockIdx.x * kWinThreads * kWinPerThread;
  double s = 0.0;
  for (int e = 0; e < kWinPerThread; ++e) {
    const int64_t n = base + (int64_t)e * kWinThreads + threadIdx.x;
    if (n < a.N) {
      const double w = tap_window(a.taps, n, a.N, a.n_taps);
      a.win[n] = (float)w;
      s += w * w;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kWinThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0];
}

// sum of the block partials: lane t adds the t-th of 64 contiguous runs in block order, then the 64 run sums
// are added by a fixed tree (the result does not depend on timing)
__global__ void __launch_bounds__(64) k_sum_partials(const double* __restrict__ partial, int n, double* out) {
  __shared__ double red[64];
  const int t = (int)threadIdx.x, run = (n + 63) / 64;
  double s = 0.0;
  for (int i = t * run; i < n && i < (t + 1) * run; ++i) s += partial[i];
  red[t] = s;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[0] = red[0];
}

// ------------------------------------------------------------------------------------------------
// per-channel adjoint of Eq. 2 and the calibration (unit-major: one thread per accumulator slot)
// ------------------------------------------------------------------------------------------------

struct cm2 {
  cd a, b, c, d;  // [[a, b], [c, d]]
};
__device__ __forceinline__ cm2 mmul(const cm2& x, const cm2& y) {
  return {cda(cdm(x.a, y.a), cdm(x.b, y.c)), cda(cdm(x.a, y.b), cdm(x.b, y.d)),
          cda(cdm(x.c, y.a), cdm(x.d, y.c)), cda(cdm(x.c, y.b), cdm(x.d, y.d))};
}
__device__ __forceinline__ cm2 madj(const cm2& x) { return {cdc(x.a), cdc(x.c), cdc(x.b), cdc(x.d)}; }
__device__ __forceinline__ cm2 madd(const cm2& x, const cm2& y) {
  return {cda(x.a, y.a), cda(x.b, y.b), cda(x.c, y.c), cda(x.d, y.d)};
}

constexpr int kBwRed = 5;  // block partials: Re/Im Gb(d_x), Re/Im Gb(d_y), Re tr(Gb(M)^H M)

// One wave per 64 channel slots of a unit (workgroups of 64 threads, so that every CU takes part: one
// workgroup per unit left half the device idle); the wave's partials are added by a fixed tree and written
// as partial (unit, quarter) of the pair: bw_parts(N1, L) = N1/2 * max(1, L/64) partials per pair.
constexpr int kBwChanThreads = 64;

template <int L>
__global__ void __launch_bounds__(kBwChanThreads) k_bw_channel(BwChanArgs a) {
  constexpr int NQ = L > kBwChanThreads ? L / kBwChanThreads : 1, TPB = L < kBwChanThreads ? L : kBwChanThreads;
  __shared__ double red[kBwRed][TPB];
  const int U = a.N1 / 2;
  const int u = (int)blockIdx.x / NQ, qq = (int)blockIdx.x % NQ, p = (int)blockIdx.y;
  const int s = qq * TPB + (int)threadIdx.x;
  const int half = s / (L / 2), k2 = s % (L / 2);
  const int row = (u == 0) ? (half ? a.N1 / 2 : 0) : (half ? a.N1 - u : u);
  const int64_t k = (int64_t)row + (int64_t)a.N1 * k2;
  const int64_t slot = ((int64_t)(p * U + u) * 4) * L + s;
  const double fs = a.n_frames * a.sumw2[0];
  // normalised coherency M (stored sums are 4 XX*, 4 YY*, 4 XY*)
  const double q = 0.25 / fs;
  // the calibration and the upstream gradient are loaded first, so their round trip overlaps the sums'
  cd gx = {1.0, 0.0}, gy = {1.0, 0.0}, dx = {0.0, 0.0}, dy = {0.0, 0.0};
  const int64_t gi = 2 * ((int64_t)p * a.C + k);
  if (a.gain_x) gx = {(double)a.gain_x[gi], (double)a.gain_x[gi + 1]};
  if (a.gain_y) gy = {(double)a.gain_y[gi], (double)a.gain_y[gi + 1]};
  if (a.dterms) {
    dx = {(double)a.dterms[4 * p + 0], (double)a.dterms[4 * p + 1]};
    dy = {(double)a.dterms[4 * p + 2], (double)a.dterms[4 * p + 3]};
  }
  const float* g = a.g_iquv + (int64_t)p * 4 * a.C + k;
  const double gI = g[0], gQ = g[a.C], gU = g[2 * a.C], gV = g[3 * a.C];
  // the slots' sums, added in slot order; the loads are issued four slots at a time (one slot at a time, each
  // add waiting for its load, the chain of round trips set the kernel's duration)
  double sum[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) sum[c] = a.acc[slot + c * L];
  int sg = 1;
  for (; sg + 4 <= a.slots; sg += 4) {
    double v[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) v[j][c] = a.acc[(int64_t)(sg + j) * a.slot_stride + slot + c * L];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) sum[c] += v[j][c];
  }
  for (; sg < a.slots; ++sg)
#pragma unroll
    for (int c = 0; c < 4; ++c) sum[c] += a.acc[(int64_t)sg * a.slot_stride + slot + c * L];
  const cd mxy = {sum[2] * q, sum[3] * q};
  const cm2 M = {{sum[0] * q, 0.0}, mxy, cdc(mxy), {sum[1] * q, 0.0}};
  const cm2 G = {gx, {0.0, 0.0}, {0.0, 0.0}, gy};
  const cm2 J = {{1.0, 0.0}, dx, dy, {1.0, 0.0}};
  const cm2 E = mmul(G, J);
  const cd det = cda(cdm(E.a, E.d), {-cdm(E.b, E.c).x, -cdm(E.b, E.c).y});
  const double inv = 1.0 / (det.x * det.x + det.y * det.y);
  const cd id = {det.x * inv, -det.y * inv};
  const cm2 Fi = {cdm(E.d, id), cdm({-E.b.x, -E.b.y}, id), cdm({-E.c.x, -E.c.y}, id), cdm(E.a, id)};
  // Gb(C) from the upstream gradient on I, Q, U, V (Eq. 2 rows; real outputs)
  const double c2 = a.cos2psi, s2 = a.sin2psi;
  const cd gc00 = {0.5 * (gI + c2 * gQ + s2 * gU), 0.0};
  const cd gc11 = {0.5 * (gI - c2 * gQ - s2 * gU), 0.0};
  const cd gc01 = {0.5 * (-s2 * gQ + c2 * gU), 0.5 * gV};   // conj of (-s2, c2, -i) / 2 rows
  const cd gc10 = {0.5 * (-s2 * gQ + c2 * gU), -0.5 * gV};  // conj of (-s2, c2, +i) / 2 rows
  const cm2 GC = {gc00, gc01, gc10, gc11};
  const cm2 GM = mmul(mmul(madj(Fi), GC), Fi);
  const cm2 GF = mmul(mmul(madd(GC, madj(GC)), Fi), M);
  cm2 GE = mmul(mmul(madj(Fi), GF), madj(Fi));
  GE = {{-GE.a.x, -GE.a.y}, {-GE.b.x, -GE.b.y}, {-GE.c.x, -GE.c.y}, {-GE.d.x, -GE.d.y}};
  const cm2 GG = mmul(GE, madj(J));
  const cm2 GJ = mmul(madj(G), GE);
  if (a.d_gain_x) {
    a.d_gain_x[gi] = (float)GG.a.x;
    a.d_gain_x[gi + 1] = (float)GG.a.y;
  }
  if (a.d_gain_y) {
    a.d_gain_y[gi] = (float)GG.d.x;
    a.d_gain_y[gi + 1] = (float)GG.d.y;
  }
  // Gb(A) = Gb(M) / (F s): Hermitian; keep its diagonal and upper entry (unit-major, coalesced)
  if (a.g_a) {
    float* ga = a.g_a + ((int64_t)(p * U + u) * 4) * L + s;
    ga[0] = (float)(GM.a.x / fs);
    ga[L] = (float)(GM.d.x / fs);
    ga[2 * L] = (float)(0.5 * (GM.b.x + GM.c.x) / fs);
    ga[3 * L] = (float)(0.5 * (GM.b.y - GM.c.y) / fs);
  }
  const double nt = GM.a.x * M.a.x + GM.a.y * M.a.y + GM.b.x * M.b.x + GM.b.y * M.b.y + GM.c.x * M.c.x +
                    GM.c.y * M.c.y + GM.d.x * M.d.x + GM.d.y * M.d.y;
  const int t = (int)threadIdx.x;
  red[0][t] = GJ.b.x;
  red[1][t] = GJ.b.y;
  red[2][t] = GJ.c.x;
  red[3][t] = GJ.c.y;
  red[4][t] = nt;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (t < h)
      for (int r = 0; r < kBwRed; ++r) red[r][t] += red[r][t + h];
    __syncthreads();
  }
  if (t < kBwRed) a.red[(((int64_t)p * U + u) * NQ + qq) * kBwRed + t] = red[t][0];
}

// per pair: leakage gradients and the normaliser term.  Lane t sums the units t, t + 64, ... (in order), then
// the 64 lanes' sums are added pairwise in a fixed tree, so the result does not depend on timing.
__global__ void __launch_bounds__(64) k_bw_reduce(BwChanArgs a) {
  __shared__ double sh[kBwRed][64];
  const int U = a.parts, p = (int)blockIdx.x, t = (int)threadIdx.x;  // U: the pair's partials
  double v[kBwRed] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int u = t; u < U; u += 64)
#pragma unroll
    for (int r = 0; r < kBwRed; ++r) v[r] += a.red[((int64_t)p * U + u) * kBwRed + r];
#pragma unroll
  for (int r = 0; r < kBwRed; ++r) sh[r][t] = v[r];
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int r = 0; r < kBwRed; ++r) sh[r][t] += sh[r][t + h];
    __syncthreads();
  }
  if (t < 4) {
    if (a.d_dterms) a.d_dterms[4 * p + t] = (float)sh[t][0];
  } else if (t == 4) {
    a.norm[p] = sh[4][0];
  }
}

// ------------------------------------------------------------------------------------------------
// backward row pass: forward row transforms of the recomputed frame, per-channel adjoint, inverse row
// transforms (by conjugation: IDFT(x) = conj(DFT(conj x))), twiddle e^{+2 pi i m1 n2 / N}, write T'
// in place of T.  The spectrum W whose inverse transform is h_x + i h_y holds, for a channel k with
// X' = Gb(A)_00 X + Gb(A)_01 Y and Y' = Gb(A)_10 X + Gb(A)_11 Y (half of Gb(X), Gb(Y)):
//   W[k] = X' + i Y',  W[N - k] = conj(X') + i conj(Y')  (0 < k < C),  W[0] = 2 Re X' + 2i Re Y',  W[C] = 0.
// ------------------------------------------------------------------------------------------------

template <int L, int UB, int FB>
__global__ void __launch_bounds__(UB * FB * L / 4) k_bw_rowpass(BwRowArgs a, int fpg) {
  // frames [blockIdx.z fpg, +fpg) of the launch: frames are independent here, so groups of them run in
  // parallel workgroups
  const int fz0 = (int)blockIdx.z * fpg;
  const int n_frames = min(fpg, a.n_frames - fz0);
  if (n_frames <= 0) return;
  constexpr int NT = UB * FB * L / 4;
  constexpr int TPS = L / 8;
  constexpr int NCH = UB * L;  // channel slots, one per owning thread
  static_assert(NCH <= NT, "one slot per thread");
  using SC = Sched<L>;
  constexpr int R0 = SC::R0;
  __shared__ __align__(16) float2 buf[UB * FB * 2 * L];
  const int tid = (int)threadIdx.x;
  const int p = (int)blockIdx.y;
  const int U = a.N1 / 2;
  const int ts = tid % TPS, q = tid / TPS;
  const int rr = q & 1, fs = (q >> 1) % FB, ub = (q >> 1) / FB;
  const int u = (int)blockIdx.x * UB + ub;
  const int row = (u == 0) ? (rr ? a.N1 / 2 : 0) : (rr ? a.N1 - u : u);
  float2* seq[1] = {buf + ((ub * FB + fs) * 2 + rr) * L};

  PassTw<L> tw;
  tw.load(a.tw_row, ts);
  // inverse four-step twiddles e^{+2 pi i row n2 / N} of this thread's outputs n2 = ts + r L/8
  float2 itw[8];
  const int mask = (1 << a.lo_bits) - 1;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int m = row * (ts + r * (L / 8));
    const float2 w = cmul(a.tw_hi[m >> a.lo_bits], a.tw_lo[m & mask]);
    itw[r] = make_float2(w.x, -w.y);
  }
  // channel slot of an owning thread and its Gb(A)
  const bool owner = tid < NCH;
  const int ubc = tid / L, sl = tid % L;
  const int uc = (int)blockIdx.x * UB + ubc;
  const int half = sl / (L / 2), k2 = sl % (L / 2);
  const int phalf = (uc == 0) ? half : 1 - half;
  const int pk2 = (uc == 0 && half == 0) ? ((L - k2) & (L - 1)) : (L - 1 - k2);
  const bool dc = (uc == 0 && half == 0 && k2 == 0);
  float g00 = 0.f, g11 = 0.f, g01r = 0.f, g01i = 0.f;
  if (owner) {
    const float* ga = a.g_a + ((int64_t)(p * U + uc) * 4) * L + sl;
    g00 = ga[0];
    g11 = ga[L];
    g01r = ga[2 * L];
    g01i = ga[3 * L];
  }
  const int oa = (ubc * FB * 2 + half) * L + swz(k2), ob = (ubc * FB * 2 + phalf) * L + swz(pk2);
  // the Nyquist bin (row 0, k2 = L/2) has no channel: the DC owner clears it
  const int onyq = (ubc * FB * 2 + 0) * L + swz(L / 2);

  const int64_t fstride = (int64_t)a.P * a.N1 * L;
  float2* const tb = a.T + (int64_t)fz0 * fstride + ((int64_t)p * a.N1 + row) * (int64_t)L;
  const float2* src = tb + ts;
  auto fetch = [&](float2 (&d)[1][8], int f0) {
    const float2* pj = src + (int64_t)min(f0 + fs, n_frames - 1) * fstride;
#pragma unroll
    for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) d[0][i * R0 + r] = pj[i * (L / 8) + r * (L / R0)];
  };
  auto batch = [&](float2 (&v)[1][8], int f0) {
    row_chain<L, 1, 0>(v, ts, tw, seq);
    __syncthreads();
    const int nf = min(FB, n_frames - f0);
    if (owner) {
      for (int g = 0; g < nf; ++g) {
        float2* fr = buf + g * 2 * L;
        const float2 A = fr[oa], B = fr[ob];
        // X = (A + conj B)/2, Y = (A - conj B)/(2i)
        const float2 X = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
        const float2 Y = make_float2(0.5f * (A.y + B.y), -0.5f * (A.x - B.x));
        const float2 Xp = make_float2(g00 * X.x + g01r * Y.x - g01i * Y.y, g00 * X.y + g01r * Y.y + g01i * Y.x);
        const float2 Yp = make_float2(g01r * X.x + g01i * X.y + g11 * Y.x, g01r * X.y - g01i * X.x + g11 * Y.y);
        if (dc) {
          fr[oa] = make_float2(2.f * Xp.x, 2.f * Yp.x);
          fr[onyq] = make_float2(0.f, 0.f);
        } else {
          fr[oa] = make_float2(Xp.x - Yp.y, Xp.y + Yp.x);   // X' + i Y'
          fr[ob] = make_float2(Xp.x + Yp.y, Yp.x - Xp.y);   // conj X' + i conj Y'
        }
      }
    }
    __syncthreads();
    // inverse row transform of this thread's sequence (frames past the end are transformed and dropped)
    float2 w[1][8];
#pragma unroll
    for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const float2 x = seq[0][swz(pin<L, R0>(ts, i, r))];
        w[0][i * R0 + r] = make_float2(x.x, -x.y);
      }
    exchange_sync<L>();
    row_chain<L, 1, 0>(w, ts, tw, seq);
    exchange_sync<L>();
    if (f0 + fs < n_frames) {
      float2* dst = tb + (int64_t)(f0 + fs) * fstride;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const float2 z = seq[0][swz(ts + r * (L / 8))];
        dst[ts + r * (L / 8)] = cmul(make_float2(z.x, -z.y), itw[r]);
      }
    }
    __syncthreads();
  };
  // unconditional prefetches (past the end they re-read the last frame): each batch waits only for its
  // own loads, as in the forward row pass
  float2 va[1][8], vb[1][8];
  fetch(va, 0);
  for (int f0 = 0; f0 < n_frames; f0 += 2 * FB) {
    fetch(vb, f0 + FB);
    batch(va, f0);
    fetch(va, f0 + 2 * FB);
    if (f0 + FB < n_frames) batch(vb, f0 + FB);
  }
}

// ------------------------------------------------------------------------------------------------
// backward column pass: inverse column transforms of T' give h_x + i h_y at n = n1 N2 + n2; multiplied by
// the re-read (unwindowed) samples they are summed per sample over the workgroup's frames in FP64 and
// added to the group's partial dL/dw (groups and frames in fixed order).
// ------------------------------------------------------------------------------------------------

template <int L, int COLS, int BITS, bool FAST>
__global__ void __launch_bounds__(L * COLS / 16) k_bw_colpass(BwColArgs a) {
  constexpr int V = 2, CPR = COLS / V;
  using SC = Sched<L>;
  constexpr int R0 = SC::R0;
  static_assert(SC::radix(SC::NPASS - 1) == 8 && SC::ns(SC::NPASS - 1) == L / 8, "last pass must be radix 8");
  constexpr int NB = (2 * L * COLS * 8 <= 128 * 1024) ? 2 : 1;
  __shared__ __align__(16) float2 tile[NB * L * COLS];

  const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cb = blk % a.col.n_colblk;
  const int rest = blk / a.col.n_colblk;
  const int p = rest % a.col.P;
  const int g = rest / a.col.P;
  const int f_begin = g * a.col.frames_per_block;
  const int f_end = min(a.col.n_frames, f_begin + a.col.frames_per_block);
  const int cv = (int)threadIdx.x % CPR, ts = (int)threadIdx.x / CPR;
  const int n2b = cb * COLS + cv * V;
  const int sx = a.col.px[p], sy = a.col.py[p];
  PassTw<L> tw;
  tw.load(a.col.tw_col, ts);

  double acc[V][8];
#pragma unroll
  for (int c = 0; c < V; ++c)
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[c][r] = 0.0;

  // The next frame's T' and samples are fetched while the current one is transformed (unconditionally: the
  // last frame fetches itself again, so every frame waits only for its own loads).
  float4 zn[8];
  ColLoader<BITS, FAST, V> ldn;
  auto fetch = [&](int f) {
    // T'[f][p][m1][n2b ..]: the inverse transform's input
    const float2* srcT = a.col.T + ((int64_t)f * a.col.P + p) * (int64_t)L * a.col.N2 + n2b;
#pragma unroll
    for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        zn[i * R0 + r] = *reinterpret_cast<const float4*>(srcT + (int64_t)pin<L, R0>(ts, i, r) * a.col.N2);
    // samples x, y at n = (ts + r L/8) N2 + n2b + c
    ldn.template fetch<L, 8>(a.col, (int64_t)f * a.col.hop, ts, n2b);
  };
  if (f_begin < f_end) fetch(f_begin);
  for (int f = f_begin; f < f_end; ++f) {
    float2 v[V][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      v[0][e] = make_float2(zn[e].x, -zn[e].y);  // conjugated
      v[1][e] = make_float2(zn[e].z, -zn[e].w);
    }
    const ColLoader<BITS, FAST, V> ld = ldn;
    fetch(min(f + 1, f_end - 1));
    col_chain<L, COLS, V, NB, 0>(v, ts, cv, tw, tile);
    if constexpr (NB == 2 && (SC::NPASS - 1) % 2 == 1) __syncthreads();
    float2 xs[V][8];
    ld.template convert<L, 8>(xs, a.col, ts, n2b, sx, sy);
#pragma unroll
    for (int c = 0; c < V; ++c)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        // h = conj of the forward result; h_x = Re h, h_y = Im h
        acc[c][r] += (double)(xs[c][r].x * v[c][r].x) - (double)(xs[c][r].y * v[c][r].y);
      }
  }
  if (f_begin >= f_end) return;
  // each (group, pair) owns its partial; pairs sum into the same window gradient
  double* dst = a.dw + (int64_t)(g * a.col.P + p) * a.col.N + n2b;
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < V; ++c) {
      double* o = dst + (int64_t)(ts + r * (L / 8)) * a.col.N2 + c;
      *o = a.first ? acc[c][r] : *o + acc[c][r];
    }
}

// ------------------------------------------------------------------------------------------------
// tap gradient: dL/dtheta_j = sum_n dw[n]/dtheta_j dL/dw[n], dL/dw[n] = sum_g partial_g[n] - 2 w[n] nt / s
// ------------------------------------------------------------------------------------------------

constexpr int kTapThreads = 256;

// the groups' partial dL/dw of each sample, added in group order into group 0's row (the order the tap
// kernel used to add them in, so the result is unchanged); one thread per sample
__global__ void __launch_bounds__(256) k_bw_dw_sum(double* __restrict__ dw, int groups, int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double s = 0.0;
#pragma unroll 8
  for (int g = 0; g < groups; ++g) s += dw[(int64_t)g * N + n];
  dw[n] = s;
}

// One pass over dL/dw in blocks of kTapThreads samples: each sample's dL/dw (the groups' partials added in
// group order, plus the normaliser term -2 w nt / s) split between the two taps around it (weights 1 - t
// and t: the window is linear between taps), summed per tap within the block by a fixed tree.  The
// dL/dw part and the window part are summed apart and combined once nt (the sum of the channel kernel's
// per-unit normaliser partials, also reduced here) is known.  Block b writes part[b][i], the sum for tap
// j_lo(b) + i (j_lo(b): the tap segment of its first sample); one extra block writes the leakage gradients.
// The host launches this form only when a block's samples touch fewer than kTapSpan taps.
constexpr int kTapSpan = 8;
constexpr int kTapRows = 2 * kTapSpan + 1;

// tap segment of sample n (as tap_position, in integer arithmetic: both give floor(n (T-1) / (N-1)))
__device__ __forceinline__ int tap_segment(int64_t n, int64_t N, int T) {
  const int64_t j = n * (int64_t)(T - 1) / (N - 1);
  return j > T - 2 ? T - 2 : (int)j;
}

template <int ROWS>
__device__ __forceinline__ void tree_sum(double (&red)[ROWS][kTapThreads], int tid) {
  __syncthreads();
  for (int h = kTapThreads / 2; h > 0; h >>= 1) {
    if (tid < h)
#pragma unroll
      for (int i = 0; i < ROWS; ++i) red[i][tid] += red[i][tid + h];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kTapThreads) k_bw_taps_block(BwTapArgs a) {
  __shared__ double red[kTapRows][kTapThreads];
  const int tid = (int)threadIdx.x, T = a.n_taps;
  if (blockIdx.x == gridDim.x - 1) {  // the extra last block: leakage gradients, per pair the unit partials 0..3
    if (!a.d_dterms) return;
    for (int p = 0; p < a.P; ++p) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        for (int u = tid; u < a.U; u += kTapThreads) s += a.red[((int64_t)p * a.U + u) * kBwRed + r];
        red[r][tid] = s;
      }
      tree_sum<kTapRows>(red, tid);
      if (tid < 4) a.d_dterms[4 * p + tid] = (float)red[tid][0];
    }
    return;
  }
  const int64_t n0 = (int64_t)blockIdx.x * kTapThreads;
  const int j_lo = tap_segment(n0, a.N, T);
#pragma unroll
  for (int i = 0; i < kTapRows; ++i) red[i][tid] = 0.0;
  double v = 0.0;  // normaliser partials: thread tid takes units tid, tid + 256, ... of every pair
  for (int p = 0; p < a.P; ++p)
    for (int u = tid; u < a.U; u += kTapThreads) v += a.red[((int64_t)p * a.U + u) * kBwRed + 4];
  red[2 * kTapSpan][tid] = v;
  const int64_t n = n0 + tid;
  if (n < a.N) {
    int jn;
    double t;
    tap_position(n, a.N, T, jn, t);
    double dw = 0.0;
#pragma unroll 8
    for (int g = 0; g < a.groups; ++g) dw += a.dw[(int64_t)g * a.N + n];
    const double w = (1.0 - t) * (double)a.taps[jn] + t * (double)a.taps[jn + 1];
    red[jn - j_lo][tid] = (1.0 - t) * dw;
    red[jn + 1 - j_lo][tid] = t * dw;
    red[kTapSpan + jn - j_lo][tid] = (1.0 - t) * w;
    red[kTapSpan + jn + 1 - j_lo][tid] = t * w;
  }
  tree_sum(red, tid);
  if (tid < kTapSpan) {
    const double coef = -2.0 * red[2 * kTapSpan][0] / a.sumw2[0];
    a.part[(int64_t)blockIdx.x * kTapSpan + tid] = red[tid][0] + coef * red[kTapSpan + tid][0];
  }
}

// tap j: the blocks whose samples can touch it (segments j - 1 and j).  One wave per tap: lane l adds the
// blocks b_lo + l, b_lo + l + 64, ... in order (their loads independent of each other: one lane walking all
// the blocks waited for each load in turn), then the 64 lane sums are added by a fixed butterfly
constexpr int kTapSumWaves = 4;

__global__ void __launch_bounds__(64 * kTapSumWaves) k_bw_taps_sum(BwTapArgs a) {
  const int lane = (int)threadIdx.x % 64;
  const int j = (int)blockIdx.x * kTapSumWaves + (int)threadIdx.x / 64, T = a.n_taps;
  if (j >= T) return;  // the same for the whole wave
  // samples of segments j - 1 and j, widened by one on each side (a block that does not touch tap j
  // holds zero in its slot for it; the last segment takes the tail)
  const double seg = (double)(a.N - 1) / (double)(T - 1);
  int64_t lo = (int64_t)floor((double)(j - 1) * seg) - 1, hi = (int64_t)ceil((double)(j + 1) * seg) + 1;
  if (j >= T - 2) hi = a.N - 1;
  if (lo < 0) lo = 0;
  if (hi > a.N - 1) hi = a.N - 1;
  double s = 0.0;
  for (int64_t b = lo / kTapThreads + lane; b <= hi / kTapThreads; b += 64) {
    int jl;
    double t;
    tap_position(b * kTapThreads, a.N, T, jl, t);  // the same segment as tap_segment (both exact floors)
    const int i = j - jl;
    if (i >= 0 && i < kTapSpan) s += a.part[b * kTapSpan + i];
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
  if (lane == 0) a.d_taps[j] = (float)s;
}

__global__ void __launch_bounds__(kTapThreads) k_bw_taps(BwTapArgs a) {
  __shared__ double red[kTapThreads];
  const int j = (int)blockIdx.x;
  const int T = a.n_taps;
  double nt = 0.0;
  for (int p = 0; p < a.P; ++p) nt += a.norm[p];
  const double coef = -2.0 * nt / a.sumw2[0];
  // samples whose window depends on tap j: u in [j - 1, j + 1)
  const double scale = (double)(a.N - 1) / (double)(T - 1);
  int64_t lo = (int64_t)floor((double)(j - 1) * scale) - 1, hi = (int64_t)ceil((double)(j + 1) * scale) + 1;
  if (j == T - 1) hi = a.N;  // the last segment is clamped onto taps T-2, T-1
  if (lo < 0) lo = 0;
  if (hi > a.N) hi = a.N;
  double s = 0.0;
  for (int64_t n = lo + threadIdx.x; n < hi; n += kTapThreads) {
    int jn;
    double t;
    tap_position(n, a.N, T, jn, t);
    double wgt = 0.0;
    if (jn == j) wgt += 1.0 - t;
    if (jn + 1 == j) wgt += t;
    if (wgt == 0.0) continue;
    double dw = 0.0;
    for (int g = 0; g < a.groups; ++g) dw += a.dw[(int64_t)g * a.N + n];
    const double w = (1.0 - t) * (double)a.taps[jn] + t * (double)a.taps[jn + 1];
    dw += coef * w;
    s += wgt * dw;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kTapThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.d_taps[j] = (float)red[0];
}

// ------------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------------

hipError_t launch_window_taps(const WinArgs& a, int n_blocks, double* sumw2, const Launch& l) {
  PS_LAUNCH(k_window_taps, dim3((unsigned)n_blocks), dim3(kWinThreads), l, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, l.stream, (const double*)a.partial, n_blocks, sumw2);
  return hipGetLastError();
}

int window_taps_blocks(int64_t N) {
  const int64_t per = (int64_t)kWinThreads * kWinPerThread;
  return (int)((N + per - 1) / per);
}

template <int L>
static hipError_t bw_channel_launch(const BwChanArgs& a, const Launch& l, bool with_reduce) {
  constexpr int NQ = L > kBwChanThreads ? L / kBwChanThreads : 1, TPB = L < kBwChanThreads ? L : kBwChanThreads;
  PS_LAUNCH((k_bw_channel<L>), dim3((unsigned)(a.N1 / 2 * NQ), (unsigned)a.P), dim3(TPB), l, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !with_reduce) return e;
  hipLaunchKernelGGL(k_bw_reduce, dim3((unsigned)a.P), dim3(64), 0, l.stream, a);
  return hipGetLastError();
}

int bw_parts(int N1, int N2) { return N1 / 2 * (N2 > kBwChanThreads ? N2 / kBwChanThreads : 1); }

hipError_t launch_bw_channel(int N2, const BwChanArgs& a, const Launch& l, bool with_reduce) {
  switch (N2) {
    case 16: return bw_channel_launch<16>(a, l, with_reduce);
    case 32: return bw_channel_launch<32>(a, l, with_reduce);
    case 64: return bw_channel_launch<64>(a, l, with_reduce);
    case 128: return bw_channel_launch<128>(a, l, with_reduce);
    case 256: return bw_channel_launch<256>(a, l, with_reduce);
    case 512: return bw_channel_launch<512>(a, l, with_reduce);
    default: return hipErrorInvalidValue;
  }
}

template <int L, int UB, int FB>
static hipError_t bw_rowpass_launch(const BwRowArgs& a, const Launch& l) {
  // enough frame groups for about 16 waves on each of the 256 CUs (four per SIMD, what the kernel's 120-odd
  // VGPRs allow): with fewer, the transforms' LDS round trips went unhidden; at N2 = 256 the workgroups hold
  // four frames (256 threads), whose barriers wait on fewer waves than those of eight-frame workgroups
  constexpr int NT = UB * FB * L / 4;
  const int units = a.N1 / 2 / UB * a.P;
  const int target = 256 * 16 * 64 / NT;
  int groups = (target + units - 1) / units;
  if (groups > a.n_frames) groups = a.n_frames > 0 ? a.n_frames : 1;
  const int fpg = (a.n_frames + groups - 1) / groups;
  groups = (a.n_frames + fpg - 1) / fpg;
  PS_LAUNCH((k_bw_rowpass<L, UB, FB>), dim3((unsigned)(a.N1 / 2 / UB), (unsigned)a.P, (unsigned)groups),
            dim3(UB * FB * L / 4), l, a, fpg);
  return hipGetLastError();
}

hipError_t launch_bw_rowpass(int N2, const BwRowArgs& a, const Launch& l) {
  switch (N2) {
    case 16: return bw_rowpass_launch<16, 8, 4>(a, l);
    case 32: return bw_rowpass_launch<32, 8, 4>(a, l);
    case 64: return bw_rowpass_launch<64, 4, 4>(a, l);
    case 128: return bw_rowpass_launch<128, 2, 4>(a, l);
    case 256: return bw_rowpass_launch<256, 1, 4>(a, l);
    case 512: return bw_rowpass_launch<512, 1, 4>(a, l);
    default: return hipErrorInvalidValue;
  }
}

template <int L>
static hipError_t bw_colpass_bits(int bits, bool fast, const BwColArgs& a, const Launch& l) {
  constexpr int COLS = 16;
  const int groups = (a.col.n_frames + a.col.frames_per_block - 1) / a.col.frames_per_block;
  const dim3 grid((unsigned)(groups * a.col.P * a.col.n_colblk)), block(L * COLS / 16);
  switch (bits) {
    case 2: PS_LAUNCH((k_bw_colpass<L, COLS, 2, false>), grid, block, l, a); break;
    case 4: PS_LAUNCH((k_bw_colpass<L, COLS, 4, false>), grid, block, l, a); break;
    case 8:
      if (fast) PS_LAUNCH((k_bw_colpass<L, COLS, 8, true>), grid, block, l, a);
      else PS_LAUNCH((k_bw_colpass<L, COLS, 8, false>), grid, block, l, a);
      break;
    case 32: PS_LAUNCH((k_bw_colpass<L, COLS, 32, false>), grid, block, l, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bw_colpass(int N1, int bits, bool fast, const BwColArgs& a, const Launch& l) {
  switch (N1) {
    case 16: return bw_colpass_bits<16>(bits, fast, a, l);
    case 32: return bw_colpass_bits<32>(bits, fast, a, l);
    case 64: return bw_colpass_bits<64>(bits, fast, a, l);
    case 128: return bw_colpass_bits<128>(bits, fast, a, l);
    case 256: return bw_colpass_bits<256>(bits, fast, a, l);
    case 512: return bw_colpass_bits<512>(bits, fast, a, l);
    default: return hipErrorInvalidValue;
  }
}

bool bw_taps_block_form(int64_t N, int n_taps) {
  // a block of kTapThreads samples spans at most ceil(255 (T - 1) / (N - 1)) + 1 segment boundaries
  return 255.0 * (double)(n_taps - 1) <= (double)(kTapSpan - 3) * (double)(N - 1);
}
int64_t bw_taps_part_doubles(int64_t N) { return ((N + kTapThreads - 1) / kTapThreads) * kTapSpan; }

hipError_t launch_bw_taps(const BwTapArgs& a, const Launch& l) {
  if (a.part && bw_taps_block_form(a.N, a.n_taps)) {
    // one block per kTapThreads samples, and one for the leakage gradients
    hipExtLaunchKernelGGL(k_bw_taps_block, dim3((unsigned)((a.N + kTapThreads - 1) / kTapThreads + 1)),
                          dim3(kTapThreads), 0, l.stream, l.start, nullptr, 0, a);
    hipExtLaunchKernelGGL(k_bw_taps_sum, dim3((unsigned)((a.n_taps + kTapSumWaves - 1) / kTapSumWaves)),
                          dim3(64 * kTapSumWaves), 0, l.stream, nullptr, l.stop, 0, a);
    return hipGetLastError();
  }
  hipExtLaunchKernelGGL(k_bw_dw_sum, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, l.stream, l.start, nullptr, 0,
                        const_cast<double*>(a.dw), a.groups, a.N);  // the plan's workspace
  BwTapArgs b = a;
  b.groups = 1;  // summed into group 0
  hipExtLaunchKernelGGL(k_bw_taps, dim3((unsigned)a.n_taps), dim3(kTapThreads), 0, l.stream, nullptr, l.stop, 0, b);
  return hipGetLastError();
}

}  // namespace ps
