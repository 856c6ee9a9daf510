// polaris_kernels.hip -- gfx950 kernels of the spectrometer path.
//
// Path (Sec. 2 and the Fig. 2 caption of Mizuno et al., arXiv 1412.1256): data translation of packed
// sampler codes, segmentation, FFT, cross products and accumulation; then Eq. 2 (Sec. 2.1) for Stokes.
//
// Design for one frame of N = N1 * N2 samples of a polarization pair (x, y):
//   * the pair is transformed as one complex sequence z = x + i*y (one length-N complex FFT gives both
//     real spectra);
//   * column pass: unpack + window straight from the packed bytes into registers, N1-point Stockham
//     radix-8 passes through LDS over a tile of adjacent columns, four-step twiddle W_N^(k1*n2), one
//     coalesced write of the FP32 intermediate;
//   * row pass: one workgroup owns the rows k1 and N1 - k1, whose bins pair up as (k, N - k); it loops
//     over every frame of the launch, runs the N2-point row transforms in LDS, splits Z into X and Y,
//     forms XX*, YY*, XY* and keeps the FP64 sums of its channels in registers across frames (frames in
//     order, so results are independent of how the frames were split over calls);
//   * the output kernels gather the unit-major accumulators through LDS into natural channel order and
//     apply the FP64 calibration and Eq. 2.
// Twiddles come from tables generated on the host in FP64 and rounded once to FP32.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <unordered_map>

#include "polaris_device.h"
#include "polaris_internal.h"

// LDS budget of a column-pass workgroup's tiles: two alternating tiles when they fit
#ifndef PS_COLPASS_LDS_MAX
#define PS_COLPASS_LDS_MAX (128 * 1024)
#endif

namespace ps {
// a kernel-invariant descriptor read through the constant address space (scalar loads into SGPRs)
template <class T>
__device__ __forceinline__ T load_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "descriptors are whole words");
  T v;
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)(p);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
  return v;
}

// Level histograms of the pair's two streams (bins in ascending level order: code c of a 2- or 4-bit
// offset-binary sample, level + 128 of an int8 one), counted in LDS and added to the device counts a.hist
// [P][2][2^BITS] at the end of the tile.  2-bit: four 8-bit counters packed per stream and thread, flushed
// every frame (at most 16 samples per stream); wider codes: LDS atomics per sample.  Element e of a column
// is counted when bit e of rows is set (overlapped frames count only their first hop samples, so that every
// sample of the stream is counted once).
template <int BITS, int NT>
struct LevelHist {
  static constexpr int NBIN = 1 << BITS;
  uint32_t packed[2];
  static __device__ __forceinline__ int bin(float level) {
    if constexpr (BITS == 8) return (int)level + 128;
    else return ((int)level + NBIN - 1) >> 1;
  }
  __device__ __forceinline__ void begin(uint32_t* hs) {
    for (int i = (int)threadIdx.x; i < 2 * NBIN; i += NT) hs[i] = 0;
    packed[0] = packed[1] = 0;
    __syncthreads();
  }
  template <int V>
  __device__ __forceinline__ void count(uint32_t* hs, const float2 (&v)[V][8], const uint32_t rows) {
#pragma unroll
    for (int c = 0; c < V; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int bx = bin(v[c][e].x), by = bin(v[c][e].y);
        const uint32_t on = (rows >> e) & 1u;
        if constexpr (BITS == 2) {
          packed[0] += on << (8 * bx);
          packed[1] += on << (8 * by);
        } else if (on) {
          atomicAdd(&hs[bx], 1u);
          atomicAdd(&hs[NBIN + by], 1u);
        }
      }
    if constexpr (BITS == 2) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t n = (packed[s] >> (8 * b)) & 0xffu;
          if (n) atomicAdd(&hs[s * 4 + b], n);
        }
        packed[s] = 0;
      }
    }
  }
  __device__ __forceinline__ void end(const uint32_t* hs, unsigned long long* out, int p) {
    __syncthreads();
    for (int i = (int)threadIdx.x; i < 2 * NBIN; i += NT)
      if (hs[i]) atomicAdd(&out[(int64_t)p * 2 * NBIN + i], (unsigned long long)hs[i]);
  }
};

// one tile of the column pass: column block, pair and frame group numbered by blk
template <int L, int COLS, int V, int BITS, int FAST, bool HIST = false>
__device__ __forceinline__ void colpass_tile(const ColArgs& a, const int blk) {
  constexpr int CPR = COLS / V;  // column groups per row
  using SC = Sched<L>;
  constexpr int R0 = SC::R0, RL = SC::radix(SC::NPASS - 1), NSL = SC::ns(SC::NPASS - 1);
  static_assert(RL == 8 && NSL == L / 8, "last pass must be radix 8");
  // two tiles when they fit beside the workgroup's other needs (one workgroup per CU)
  constexpr int NB = (2 * L * COLS * 8 <= PS_COLPASS_LDS_MAX) ? 2 : 1;
  __shared__ __align__(16) float2 tile[NB * L * COLS];

  const int cb = blk % a.n_colblk;
  const int rest = blk / a.n_colblk;
  const int p = rest % a.P;
  const int g = rest / a.P;
  const int f_begin = g * a.frames_per_block;
  const int f_end = min(a.n_frames, f_begin + a.frames_per_block);
  const int cv = (int)threadIdx.x % CPR, ts = (int)threadIdx.x / CPR;
  const int n2b = cb * COLS + cv * V;
  const int sx = a.px[p], sy = a.py[p];

  PassTw<L> tw;
  tw.load(a.tw_col, ts);
  // four-step twiddles W_N^(k1 * n2) of this thread's outputs, k1 = ts + r L/8 (the last pass's outputs)
  float2 fst[V][8];
  const int mask = (1 << a.lo_bits) - 1;
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < V; ++c) {
      const int m = (ts + r * (L / 8)) * (n2b + c);
      fst[c][r] = cmul(a.tw_hi[m >> a.lo_bits], a.tw_lo[m & mask]);
    }
  constexpr int NT = L * COLS / (8 * V);
  constexpr bool H = HIST && BITS <= 8;
  __shared__ uint32_t hs[H ? 2 << (BITS <= 8 ? BITS : 0) : 1];
  LevelHist<BITS <= 8 ? BITS : 8, NT> hist;
  uint32_t hrows = 0;  // elements of this thread's rows within the frame's first hop samples
  if constexpr (H) {
    hist.begin(hs);
#pragma unroll
    for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r)
        if (pin<L, R0>(ts, i, r) < a.hist_rows) hrows |= 1u << (i * R0 + r);
  }
  // input words are fetched one frame ahead of their use
  auto frame = [&](ColLoader<BITS, FAST, V>& ld, const int f) {
    float2 v[V][8];
    ld.template convert<L, R0>(v, a, ts, n2b, sx, sy);
    if constexpr (H) hist.count(hs, v, hrows);
    if (a.win) {  // the window is the same for every frame (and cached in L2); read before the prefetch
#pragma unroll
      for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          const int64_t n = (int64_t)pin<L, R0>(ts, i, r) * a.N2 + n2b;
#pragma unroll
          for (int c = 0; c < V; ++c) {
            const float w = a.win[n + c];
            v[c][i * R0 + r] = make_float2(v[c][i * R0 + r].x * w, v[c][i * R0 + r].y * w);
          }
        }
    }
    // The next frame's loads and this frame's stores are issued at raised wave priority, so that they reach
    // the memory system before the other waves' arithmetic (column pass 41.3 -> 40.4 us, two integrations
    // in flight 62.0 -> 61.1 us on the paper workload)
    __builtin_amdgcn_s_setprio(3);
    if (f + 1 < f_end) ld.template fetch<L, R0>(a, (int64_t)(f + 1) * a.hop, ts, n2b);
    __builtin_amdgcn_s_setprio(0);
    col_chain<L, COLS, V, NB, 0>(v, ts, cv, tw, tile);
    // with an odd number of exchanges per frame the next frame's first exchange reuses the tile the last
    // one read: wait for every reader first
    if constexpr (NB == 2 && (SC::NPASS - 1) % 2 == 1) __syncthreads();
    // write T[f][p][k1][n2b ..] for k1 = ts + r L/8 (global stores: the next kernel reads them from every XCD)
    const uint32_t voff = 8u * (uint32_t)(ts * a.N2 + n2b);
    __builtin_amdgcn_s_setprio(2);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const gbytes base = uniform_gptr(reinterpret_cast<const uint8_t*>(
          a.T + ((int64_t)f * a.P + p) * (int64_t)L * a.N2 + (int64_t)r * (L / 8) * a.N2));
      const float2 o0 = cmul(v[0][r], fst[0][r]);
      if constexpr (V == 2) {
        const float2 o1 = cmul(v[1][r], fst[1][r]);
        const f32x4 q = {o0.x, o0.y, o1.x, o1.y};
        *(__attribute__((address_space(1))) f32x4*)(base + voff) = q;
      } else {
        const f32x2 q = {o0.x, o0.y};
        *(__attribute__((address_space(1))) f32x2*)(base + voff) = q;
      }
    }
    __builtin_amdgcn_s_setprio(0);
  };
  // One loop from the first frame: the wait for a frame's input words then also waits for the previous
  // frame's stores (issued after those words).  Peeling the first frame, so that the stores stay in flight
  // into the next frame, measured 5 % slower on the paper-shaped workload (the reads of the next frame then
  // compete with a burst of writes).
  ColLoader<BITS, FAST, V> ld;
  if (f_begin < f_end) ld.template fetch<L, R0>(a, (int64_t)f_begin * a.hop, ts, n2b);
  for (int f = f_begin; f < f_end; ++f) frame(ld, f);
  if constexpr (H) hist.end(hs, a.hist, p);
}

template <int L, int COLS, int V, int BITS, int FAST>
__global__ void __launch_bounds__(L * COLS / (8 * V)) k_colpass(ColArgs a) {
  colpass_tile<L, COLS, V, BITS, FAST>(a, xcd_remap((int)blockIdx.x, (int)gridDim.x));
}

// the column pass that also counts the level histograms of its streams
template <int L, int COLS, int V, int BITS, int FAST>
__global__ void __launch_bounds__(L * COLS / (8 * V)) k_colpass_hist(ColArgs a) {
  colpass_tile<L, COLS, V, BITS, FAST, true>(a, xcd_remap((int)blockIdx.x, (int)gridDim.x));
}

// Grouped column pass over the tiles of several instances of the same shape and format: one workgroup per
// tile (a loop over tiles in each workgroup cost 10-30 registers and often a wave per SIMD).  tile_end holds
// the running tile totals; the task descriptors are read through the constant address space (scalar loads
// into SGPRs).  The grid is the tile count, renumbered as the single-instance launch does so that
// neighbouring column blocks run on one XCD.
__device__ __forceinline__ int batch_task(const int32_t* __restrict__ tile_end, int n_tasks, int tile) {
  int lo = 0, hi = n_tasks - 1;  // first task whose running total exceeds the tile
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (tile < tile_end[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

template <int L, int COLS, int V, int BITS, int FAST>
__global__ void __launch_bounds__(L * COLS / (8 * V))
    k_colpass_batch(const ColArgs* __restrict__ tasks, const int32_t* __restrict__ tile_end, int n_tasks) {
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int t = batch_task(tile_end, n_tasks, tile);
  const ColArgs a = load_const(tasks + t);
  colpass_tile<L, COLS, V, BITS, FAST>(a, tile - (t ? tile_end[t - 1] : 0));
}

// Calibrated Stokes of channel k of pair p from its accumulated products (the sums of XX*, YY*, XY*):
// normalised coherency M = A / (F sum w^2), calibration C = (G J)^-1 M (G J)^-H and Eq. 2 (or the circular
// combination), all in FP64; I, Q, U, V are written to a.iquv [P][4][C] as floats.
__device__ __forceinline__ void stokes_write(const OutArgs& a, const int p, const int64_t k, const double scale,
                                             const double axx, const double ayy, const double axr,
                                             const double axi) {
  // normalised coherency M = A / (F sum w^2); C = Fi M Fi^H with Fi = (G J)^-1 (C_yx = conj C_xy)
  const double mxx = axx * scale, myy = ayy * scale;
  const cd mxy = {axr * scale, axi * scale}, myx = cdc(mxy);
  double cxx = mxx, cyy = myy;
  cd cxy = mxy;
  if (a.gain_x || a.gain_y || a.dterms) {
    cd gx = {1.0, 0.0}, gy = {1.0, 0.0}, dx = {0.0, 0.0}, dy = {0.0, 0.0};
    const int64_t gi = 2 * ((int64_t)p * a.C + k);
    if (a.gain_x) gx = {(double)a.gain_x[gi], (double)a.gain_x[gi + 1]};
    if (a.gain_y) gy = {(double)a.gain_y[gi], (double)a.gain_y[gi + 1]};
    if (a.dterms) {
      dx = {(double)a.dterms[4 * p + 0], (double)a.dterms[4 * p + 1]};
      dy = {(double)a.dterms[4 * p + 2], (double)a.dterms[4 * p + 3]};
    }
    // E = [[gx, gx dx], [gy dy, gy]], det E = gx gy (1 - dx dy), Fi = adj(E) / det E
    const cd e01 = cdm(gx, dx), e10 = cdm(gy, dy);
    const cd dxy = cdm(dx, dy);
    const cd det = cdm(cdm(gx, gy), {1.0 - dxy.x, -dxy.y});
    const double inv = 1.0 / (det.x * det.x + det.y * det.y);
    const cd id = {det.x * inv, -det.y * inv};  // 1 / det
    const cd f00 = cdm(gy, id), f01 = cdm({-e01.x, -e01.y}, id);
    const cd f10 = cdm({-e10.x, -e10.y}, id), f11 = cdm(gx, id);
    const cd t00 = cda(cdm(f00, {mxx, 0.0}), cdm(f01, myx)), t01 = cda(cdm(f00, mxy), cdm(f01, {myy, 0.0}));
    const cd t10 = cda(cdm(f10, {mxx, 0.0}), cdm(f11, myx)), t11 = cda(cdm(f10, mxy), cdm(f11, {myy, 0.0}));
    cxx = cda(cdm(t00, cdc(f00)), cdm(t01, cdc(f01))).x;
    cxy = cda(cdm(t00, cdc(f10)), cdm(t01, cdc(f11)));
    cyy = cda(cdm(t10, cdc(f10)), cdm(t11, cdc(f11))).x;
  }
  const double c2 = a.cos2psi, s2 = a.sin2psi;
  double I, Q, Uq, V;
  if (a.circular) {
    // streams R, L: I = (C_rr + C_ll)/2, V = (C_rr - C_ll)/2, Q + iU = C_rl exp(2i psi)
    I = 0.5 * (cxx + cyy);
    V = 0.5 * (cxx - cyy);
    Q = c2 * cxy.x - s2 * cxy.y;
    Uq = s2 * cxy.x + c2 * cxy.y;
  } else {
    // Eq. 2 rows acting on [C_xx, C_xy, C_yx, C_yy] with C_yx = conj C_xy
    I = 0.5 * (cxx + cyy);
    Q = 0.5 * (c2 * (cxx - cyy) - s2 * 2.0 * cxy.x);
    Uq = 0.5 * (s2 * (cxx - cyy) + c2 * 2.0 * cxy.x);
    V = cxy.y;  // Re(-i C_xy + i C_yx) / 2
  }
  float* o = a.iquv + (int64_t)p * 4 * a.C + k;
  o[0] = (float)I;
  o[a.C] = (float)Q;
  o[2 * a.C] = (float)Uq;
  o[3 * a.C] = (float)V;
}

// one tile of the row pass: units bx*UB .. bx*UB+UB-1 of pair p, the launch's frames of accumulator slot g
// With STOKES (one accumulator slot, the integration's last launch), the owners of the channel slots also
// write the calibrated Stokes of their channels from the final sums (exactly what the output kernel
// computes from the stored accumulators).
// threads of a row-pass workgroup: UB units of two rows, FB frames, SQ sequences per thread, and L/8 threads
// per row (L/16 for the wide rows of 1024 and 2048 points)
template <int L, int UB, int FB, int SQ>
constexpr int rowpass_threads() {
  return UB * FB * 2 * (L >= 1024 ? L / 16 : L / 8) / SQ;
}

template <int L, int UB, int FB, int SQ, bool STOKES = false>
__device__ __forceinline__ void rowpass_tile(const RowArgs& a, const int bx, const int p, const int g,
                                             const OutArgs* o = nullptr) {
  constexpr bool WIDE = L >= 1024;
  static_assert(!WIDE || SQ == 1, "one wide row per thread");
  // 2048-point rows by decimation in time: wave h of a row transforms its samples 2 m + h (1024 points, 16
  // per lane, exchanges within the wave), and the channel stage forms each bin from the two halves,
  // Z[k] = E[k mod 1024] + W_2048^k O[k mod 1024]
  constexpr bool DIT = L == 2048;
  constexpr int LH = DIT ? L / 2 : L;  // points of the transform a wave group runs
  constexpr int PT = WIDE ? 16 : 8;                 // points per thread and sequence
  constexpr int NT = rowpass_threads<L, UB, FB, SQ>();
  constexpr int TPS = L / PT;                      // threads per row sequence
  constexpr int NCH = UB * L < NT ? UB * L : NT;   // threads that own channel slots
  constexpr int SPT = (UB * L) / NCH;              // channel slots per owning thread
  constexpr int FS = FB / SQ;                      // frame stride between a thread's sequences
  constexpr int SEQ = L;                           // sequence length in LDS
  using SC = Sched<L>;
  constexpr int R0 = SC::R0;
  // Long rows keep two LDS buffers, taken by the batches in turn: a batch's transform then writes the buffer
  // the previous batch's channel stage may still be reading only once every thread has passed the barrier
  // that follows the previous batch's last pass, so no barrier is needed after the channel stage.  Rows of
  // 512 points in batches of 4 frames still fit two workgroups per CU with both buffers.
  // The two buffers are interleaved by row (row q of buffer b at (2 q + b) L), so a row's place in either
  // buffer is within the reach of an LDS instruction's immediate offset from the same address register.
  constexpr bool ALT = WIDE || (L == 512 && UB * FB <= 4);
  constexpr int RS = (ALT ? 2 : 1) * SEQ;  // LDS stride between rows
  __shared__ __align__(16) float2 buf[UB * FB * 2 * RS];
  const int tid = (int)threadIdx.x;
  const int U = a.N1 / 2;
  // transform role: slot ts of row rr of frames fs + j FS (j < SQ) of unit ub
  const int ts = tid % TPS, q = tid / TPS;
  const int hw = DIT ? ts / 64 : 0, tl = DIT ? ts % 64 : ts;  // half of the row and lane within it
  const int rr = q & 1, fs = (q >> 1) % FS, ub = (q >> 1) / FS;
  const int u = bx * UB + ub;
  const int row = (u == 0) ? (rr ? a.N1 / 2 : 0) : (rr ? a.N1 - u : u);
  float2* seq[SQ];
#pragma unroll
  for (int j = 0; j < SQ; ++j) seq[j] = buf + ((ub * FB + fs + j * FS) * 2 + rr) * RS;

  using Tw = typename std::conditional<WIDE, WideTw<LH>, PassTw<L>>::type;
  Tw tw;
  if constexpr (DIT) tw.template load<2>(a.tw_row, tl);
  else tw.load(a.tw_row, ts);


  // this slot's frames of the launch: f = f_first + j G, j < n_loc (absolute frame a = F0 + f, a mod G = g)
  const int f_first = (int)(((int64_t)g - a.F0 % a.G + a.G) % a.G);
  const int n_loc = f_first < a.n_frames ? (a.n_frames - f_first + a.G - 1) / a.G : 0;
  if (n_loc == 0) return;
  const bool prior = a.F0 > g;  // the slot already holds frames of this integration
  const bool owner = tid < NCH;
  double sxx[SPT], syy[SPT], sxr[SPT], sxi[SPT];
  double* accp[SPT];
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int id = tid + k * NCH;
    const int ubc = id / L, s = id % L;
    const int uc = bx * UB + ubc;
    accp[k] = a.acc + (int64_t)g * a.slot_stride + ((int64_t)(p * U + uc) * 4) * L + s;
    sxx[k] = syy[k] = sxr[k] = sxi[k] = 0.0;
    if (owner && prior) {
      sxx[k] = accp[k][0];
      syy[k] = accp[k][L];
      sxr[k] = accp[k][2 * L];
      sxi[k] = accp[k][3 * L];
    }
  }

  // decimation in time: each slot's twiddles W_2048^k2 and, for its partner bin, +-W_2048^(pk2 mod 1024)
  float2 dwa[DIT ? SPT : 1], dwb[DIT ? SPT : 1];
  if constexpr (DIT) {
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const int id = tid + k * NCH;
      const int ubc = id / L, s = id % L;
      const int uc = bx * UB + ubc;
      const int half = s / (L / 2), k2 = s % (L / 2);
      const int pk2 = (uc == 0 && half == 0) ? ((L - k2) & (L - 1)) : (L - 1 - k2);
      dwa[k] = a.tw_row[k2];
      const float2 w = a.tw_row[pk2 & (LH - 1)];
      dwb[k] = pk2 >= LH ? make_float2(-w.x, -w.y) : w;
    }
  }

  const int64_t fstride = (int64_t)a.P * a.N1 * L;  // float2 per frame
  const float2* src = a.T + ((int64_t)p * a.N1 + row) * (int64_t)L + (DIT ? 2 * tl + hw : ts);
  // local frames past the end repeat the last one (their products are never accumulated)
  auto fetch = [&](float2 (&d)[SQ][PT], int f0) {
#pragma unroll
    for (int j = 0; j < SQ; ++j) {
      const float2* pj = src + (int64_t)(f_first + min(f0 + fs + j * FS, n_loc - 1) * a.G) * fstride;
      if constexpr (WIDE) {
#pragma unroll
        for (int k = 0; k < PT; ++k) d[j][k] = pj[k * TPS];
      } else {
#pragma unroll
        for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
          for (int r = 0; r < R0; ++r) d[j][i * R0 + r] = pj[i * (L / 8) + r * (L / R0)];
      }
    }
  };
  auto batch = [&](float2 (&v)[SQ][PT], int f0, const int par) {
    const int bo = ALT ? par * SEQ : 0;  // this batch's buffer
    float2* sq[SQ];
#pragma unroll
    for (int j = 0; j < SQ; ++j) sq[j] = seq[j] + bo;
    if constexpr (DIT) wide_chain<LH>(v[0], tl, tw, sq[0] + hw * LH);
    else if constexpr (WIDE) wide_chain<L>(v[0], ts, tw, sq[0]);
    else row_chain<L, SQ, 0>(v, ts, tw, sq);
    __syncthreads();
    if (owner) {
      const int nf = min(FB, n_loc - f0);
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        const int id = tid + k * NCH;
        const int ubc = id / L, s = id % L;
        const int uc = bx * UB + ubc;
        const int half = s / (L / 2), k2 = s % (L / 2);
        // bin (row, k2) pairs with bin N - k: rows k1 and N1 - k1 swap, k2 -> N2 - 1 - k2; row 0 -> N2 - k2
        const int phalf = (uc == 0) ? half : 1 - half;
        const int pk2 = (uc == 0 && half == 0) ? ((L - k2) & (L - 1)) : (L - 1 - k2);
        const float2* fa = buf + bo + (ubc * FB * 2 + half) * RS + swz(k2);
        const float2* fb = buf + bo + (ubc * FB * 2 + phalf) * RS + swz(DIT ? pk2 & (LH - 1) : pk2);
        for (int g = 0; g < nf; ++g) {
          float2 A, B;
          if constexpr (DIT) {  // the bins from the even-sample (E) and odd-sample (O) halves of each row
            const float2 ea = fa[g * 2 * RS], oa = fa[g * 2 * RS + LH];
            const float2 eb = fb[g * 2 * RS], ob = fb[g * 2 * RS + LH];
            const float2 ta = cmul(dwa[k], oa), tb = cmul(dwb[k], ob);
            A = make_float2(ea.x + ta.x, ea.y + ta.y);
            B = make_float2(eb.x + tb.x, eb.y + tb.y);
          } else {
            A = fa[g * 2 * RS];
            B = fb[g * 2 * RS];
          }
          const float sx_ = A.x + B.x, sy_ = A.y - B.y;   // A + conj(B) = 2 X
          const float dx_ = A.x - B.x, dy_ = A.y + B.y;   // A - conj(B) = 2i Y
          sxx[k] += (double)(sx_ * sx_ + sy_ * sy_);
          syy[k] += (double)(dx_ * dx_ + dy_ * dy_);
          sxr[k] += (double)(sx_ * dy_ - sy_ * dx_);      // Re of i (s conj d)
          sxi[k] += (double)(sx_ * dx_ + sy_ * dy_);      // Im of i (s conj d)
        }
      }
    }
    if constexpr (!ALT) __syncthreads();
    else __builtin_amdgcn_sched_barrier(0);  // keeps the next batch's transform after this channel stage
  };
  // Both prefetches are unconditional (past the end they re-read the last frame, which is never
  // accumulated): each batch then waits only for its own loads, with the next batch's still in flight.
  // A prefetch skipped on some path made every first batch of the pair wait for both.
  float2 va[SQ][PT], vb[SQ][PT];
  fetch(va, 0);
  for (int f0 = 0; f0 < n_loc; f0 += 2 * FB) {
    fetch(vb, f0 + FB);
    batch(va, f0, 0);
    fetch(va, f0 + 2 * FB);
    if (f0 + FB < n_loc) batch(vb, f0 + FB, 1);
  }
  if (owner) {
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      accp[k][0] = sxx[k];
      accp[k][L] = syy[k];
      accp[k][2 * L] = sxr[k];
      accp[k][3 * L] = sxi[k];
    }
    if constexpr (STOKES) {
      const double scale = o->sumw2_dev ? 1.0 / (o->n_frames * o->sumw2_dev[0]) : o->scale;
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        // slot s of unit uc holds bin k2 of row uc (half 0) or of its partner row (half 1): channel k2 N1 + row
        const int id = tid + k * NCH;
        const int uc = bx * UB + id / L, s = id % L;
        const int half = s / (L / 2), k2 = s % (L / 2);
        const int row = half ? (uc == 0 ? a.N1 / 2 : a.N1 - uc) : uc;
        stokes_write(*o, p, (int64_t)k2 * a.N1 + row, scale, 0.25 * sxx[k], 0.25 * syy[k], 0.25 * sxr[k],
                     0.25 * sxi[k]);
      }
    }
  }
}

template <int L, int UB, int FB, int SQ>
__global__ void __launch_bounds__((rowpass_threads<L, UB, FB, SQ>())) k_rowpass(RowArgs a) {
  rowpass_tile<L, UB, FB, SQ>(a, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z);
}

// The row pass that also writes the Stokes spectra (one slot).  A channel's four outputs are scattered
// (channel k2 N1 + row), so the units are renumbered to keep runs of consecutive rows on one XCD: the 4-byte
// writes of neighbouring rows then meet in that XCD's L2 and leave it as whole sectors.
template <int L, int UB, int FB, int SQ>
__global__ void __launch_bounds__((rowpass_threads<L, UB, FB, SQ>())) k_rowpass_stokes(RowArgs a, OutArgs o) {
  const int nbx = (int)gridDim.x;
  const int lin = xcd_remap((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
  rowpass_tile<L, UB, FB, SQ, true>(a, lin % nbx, lin / nbx, 0, &o);
}

template <int L, int UB, int FB, int SQ>
__global__ void __launch_bounds__((rowpass_threads<L, UB, FB, SQ>()))
    k_rowpass_batch(const RowArgs* __restrict__ tasks, const int32_t* __restrict__ tile_end, int n_tasks) {
  const int tile = (int)blockIdx.x;
  const int t = batch_task(tile_end, n_tasks, tile);
  const int local = tile - (t ? tile_end[t - 1] : 0);
  const RowArgs a = load_const(tasks + t);
  const int nbx = a.N1 / 2 / UB;
  rowpass_tile<L, UB, FB, SQ>(a, local % nbx, (local / nbx) % a.P, local / (nbx * a.P));
}

// ------------------------------------------------------------------------------------------------
// output: accumulators -> natural channel order (raw spectra, or calibrated Stokes by Eq. 2)
// ------------------------------------------------------------------------------------------------

constexpr int kOutThreads = 512;  // one channel of the 32 x 16 tile per thread

template <bool STOKES>
__device__ __forceinline__ void output_tile(const OutArgs& a, const int bx, const int by, const int p) {
  constexpr int RT = 32, KT = 16;
  __shared__ double t[4][RT][KT + 1];
  const int L = a.N2, U = a.N1 / 2;
  const int rt = RT < a.N1 ? RT : a.N1;
  const int kt = KT < L / 2 ? KT : L / 2;
  const int r0 = bx * rt, k20 = by * kt;
  for (int e = (int)threadIdx.x; e < rt * kt; e += kOutThreads) {
    const int rl = e / kt, kk = e % kt;
    const int r = r0 + rl, k2 = k20 + kk;
    int u, half;
    if (r == 0) { u = 0; half = 0; }
    else if (2 * r == a.N1) { u = 0; half = 1; }
    else if (2 * r < a.N1) { u = r; half = 0; }
    else { u = a.N1 - r; half = 1; }
    const double* src = a.acc + ((int64_t)(p * U + u) * 4) * L + half * (L / 2) + k2;
    // slots are added in order; their loads go out eight at a time
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = src[(int64_t)q * L];
    int g = 1;
    for (; g + 8 <= a.slots; g += 8) {
      double w[8][4];
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[j][q] = src[(int64_t)(g + j) * a.slot_stride + (int64_t)q * L];
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += w[j][q];
    }
    for (; g < a.slots; ++g)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] += src[(int64_t)g * a.slot_stride + (int64_t)q * L];
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q][rl][kk] = v[q];
  }
  __syncthreads();
  double scale = a.scale;
  if (STOKES && a.sumw2_dev) scale = 1.0 / (a.n_frames * a.sumw2_dev[0]);
  for (int e = (int)threadIdx.x; e < rt * kt; e += kOutThreads) {
    const int kk = e / rt, rl = e % rt;
    const int64_t k = (int64_t)(k20 + kk) * a.N1 + r0 + rl;
    // stored sums are 4 XX*, 4 YY*, 4 XY* (exact power-of-two scale)
    const double axx = 0.25 * t[0][rl][kk], ayy = 0.25 * t[1][rl][kk];
    const double axr = 0.25 * t[2][rl][kk], axi = 0.25 * t[3][rl][kk];
    if constexpr (!STOKES) {
      double* o = a.spectra + (int64_t)p * 4 * a.C + k;
      o[0] = axx;
      o[a.C] = ayy;
      o[2 * a.C] = axr;
      o[3 * a.C] = axi;
    } else {
      stokes_write(a, p, k, scale, axx, ayy, axr, axi);
    }
  }
}

template <bool STOKES>
__global__ void __launch_bounds__(kOutThreads) k_output(OutArgs a) {
  output_tile<STOKES>(a, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z);
}

// tiles of one instance: (N1 / rt) x (N2 / 2 / kt) x P
__host__ __device__ inline int output_tiles_x(int N1) { return N1 / (N1 < 32 ? N1 : 32); }
__host__ __device__ inline int output_tiles_y(int N2) { return N2 / 2 / (N2 / 2 < 16 ? N2 / 2 : 16); }

template <bool STOKES>
__global__ void __launch_bounds__(kOutThreads)
    k_output_batch(const OutArgs* __restrict__ tasks, const int32_t* __restrict__ tile_end, int n_tasks) {
  const int tile = (int)blockIdx.x;
  const int t = batch_task(tile_end, n_tasks, tile);
  const int local = tile - (t ? tile_end[t - 1] : 0);
  const OutArgs a = load_const(tasks + t);
  const int nx = output_tiles_x(a.N1), ny = output_tiles_y(a.N2);
  output_tile<STOKES>(a, local % nx, (local / nx) % ny, local / (nx * ny));
}

// ------------------------------------------------------------------------------------------------
// total power from level histograms: per stream, the mean square level and, for 2-bit samplers, sigma in
// units of the quantiser threshold from the fraction of samples in the two inner levels,
// P(|x| < theta) = erf(theta / (sigma sqrt 2))  ->  sigma / theta = 1 / (sqrt 2 erfinv(P))
// ------------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_hist_power(const unsigned long long* __restrict__ counts, int n_streams,
                                                   int bits, double* __restrict__ power) {
  const int s = (int)(blockIdx.x * 64 + threadIdx.x);
  if (s >= n_streams) return;
  const int nbin = 1 << bits;
  const unsigned long long* c = counts + (int64_t)s * nbin;
  double n = 0.0, m2 = 0.0;
  for (int b = 0; b < nbin; ++b) {
    const double level = bits == 8 ? (double)(b - 128) : (double)(2 * b - (nbin - 1));
    n += (double)c[b];
    m2 += level * level * (double)c[b];
  }
  power[2 * s] = n > 0.0 ? m2 / n : 0.0;
  double r = __builtin_nan("");
  if (bits == 2 && n > 0.0) {
    const double pin = ((double)c[1] + (double)c[2]) / n;
    if (pin > 0.0 && pin < 1.0) r = 1.0 / (1.4142135623730950488 * erfinv(pin));
  }
  power[2 * s + 1] = r;
}

__global__ void __launch_bounds__(256) k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0ull;
}

// ------------------------------------------------------------------------------------------------
// stand-alone data translation and a plain device copy
// ------------------------------------------------------------------------------------------------

template <int BITS>
__global__ void __launch_bounds__(256) k_unpack(const uint8_t* __restrict__ in, int S, int64_t n_time,
                                                float* __restrict__ out) {
  const int64_t n_items = n_time * S;
  for (int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x; item < n_items; item += (int64_t)gridDim.x * 256) {
    const int64_t t = item / S;
    const int s = (int)(item - t * S);
    out[(int64_t)s * n_time + t] = level_of<BITS>(in, item);
  }
}

__global__ void __launch_bounds__(256) k_copy_words(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

// ------------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------------

// Column-pass shape per N1: columns per workgroup and columns per thread (tunable at build time).
#ifndef PS_COLPASS_V
#define PS_COLPASS_V 2
#endif
#ifndef PS_ROWPASS_SQ
#define PS_ROWPASS_SQ 1
#endif

#define PS_LAUNCH(kernel, grid, block, l, ...) \
  hipExtLaunchKernelGGL(kernel, grid, block, 0, (l).stream, (l).start, (l).stop, 0, __VA_ARGS__)

// loader mode 0 (decode at use), 1 (two streams, pair (0, 1)) or 2 (four streams) of one code width
template <int L, int COLS, int V, int BITS, bool HIST>
static void colpass_mode(int mode, dim3 grid, dim3 block, const ColArgs& a, const Launch& s) {
  if constexpr (HIST) {
    if (mode == 1) PS_LAUNCH((k_colpass_hist<L, COLS, V, BITS, 1>), grid, block, s, a);
    else if (mode == 2) PS_LAUNCH((k_colpass_hist<L, COLS, V, BITS, 2>), grid, block, s, a);
    else PS_LAUNCH((k_colpass_hist<L, COLS, V, BITS, 0>), grid, block, s, a);
  } else {
    if (mode == 1) PS_LAUNCH((k_colpass<L, COLS, V, BITS, 1>), grid, block, s, a);
    else if (mode == 2) PS_LAUNCH((k_colpass<L, COLS, V, BITS, 2>), grid, block, s, a);
    else PS_LAUNCH((k_colpass<L, COLS, V, BITS, 0>), grid, block, s, a);
  }
}

template <int L, int COLS, int V>
static hipError_t colpass_bits(int bits, int mode, const ColArgs& a, const Launch& s) {
  const int groups = (a.n_frames + a.frames_per_block - 1) / a.frames_per_block;
  const dim3 grid((unsigned)(groups * a.P * a.n_colblk)), block(L * COLS / (8 * V));
  const bool hist = a.hist != nullptr;
  switch (bits) {
    case 2:
      if (hist) colpass_mode<L, COLS, V, 2, true>(mode, grid, block, a, s);
      else colpass_mode<L, COLS, V, 2, false>(mode, grid, block, a, s);
      break;
    case 4:
      if (hist) colpass_mode<L, COLS, V, 4, true>(mode, grid, block, a, s);
      else colpass_mode<L, COLS, V, 4, false>(mode, grid, block, a, s);
      break;
    case 8:
      if (hist) colpass_mode<L, COLS, V, 8, true>(mode, grid, block, a, s);
      else colpass_mode<L, COLS, V, 8, false>(mode, grid, block, a, s);
      break;
    case 32:
      if (hist) return hipErrorInvalidValue;
      PS_LAUNCH((k_colpass<L, COLS, V, 32, 0>), grid, block, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#ifndef PS_COLPASS_COLS
#define PS_COLPASS_COLS 16
#endif

int colpass_cols(int N1) { return N1 >= 2048 ? 4 : (N1 >= 1024 ? 8 : PS_COLPASS_COLS); }

// compiled (N1, columns per workgroup) pairs: the default of each N1, and 8 columns for N1 = 256 and 512
bool colpass_has(int N1, int cols) {
  if (cols == colpass_cols(N1)) return N1 >= 16 && N1 <= 2048;
  return (N1 == 256 || N1 == 512) && cols == 8;
}

hipError_t launch_colpass(int N1, int cols, int bits, int mode, const ColArgs& a, const Launch& s) {
  constexpr int V = PS_COLPASS_V;
  if (cols != colpass_cols(N1)) {
    if (N1 == 256 && cols == 8) return colpass_bits<256, 8, V>(bits, mode, a, s);
    if (N1 == 512 && cols == 8) return colpass_bits<512, 8, V>(bits, mode, a, s);
    return hipErrorInvalidValue;
  }
  switch (N1) {
    case 16: return colpass_bits<16, 16, 2>(bits, mode, a, s);
    case 32: return colpass_bits<32, 16, 2>(bits, mode, a, s);
    case 64: return colpass_bits<64, 16, 2>(bits, mode, a, s);
    case 128: return colpass_bits<128, 16, 2>(bits, mode, a, s);
    case 256: return colpass_bits<256, PS_COLPASS_COLS, V>(bits, mode, a, s);
    case 512: return colpass_bits<512, PS_COLPASS_COLS, V>(bits, mode, a, s);
    case 1024: return colpass_bits<1024, 8, 2>(bits, mode, a, s);
    case 2048: return colpass_bits<2048, 4, 2>(bits, mode, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L, int UB, int FB, int SQ>
static hipError_t rowpass_launch(const RowArgs& a, const Launch& s, const OutArgs* o) {
  const dim3 grid((unsigned)(a.N1 / 2 / UB), (unsigned)a.P, (unsigned)a.G), block(rowpass_threads<L, UB, FB, SQ>());
  if (o) {
    if (a.G != 1) return hipErrorInvalidValue;
    PS_LAUNCH((k_rowpass_stokes<L, UB, FB, SQ>), grid, block, s, a, *o);
  } else {
    PS_LAUNCH((k_rowpass<L, UB, FB, SQ>), grid, block, s, a);
  }
  return hipGetLastError();
}

// frames per row-pass workgroup batch: the default of each N2, and 4 for N2 = 256 and 512
int rowpass_frames(int N2) { return N2 >= 2048 ? 2 : (N2 >= 1024 ? 4 : 8); }
bool rowpass_has(int N2, int fb) {
  if (fb == rowpass_frames(N2)) return N2 >= 16 && N2 <= 2048;
  return (N2 == 256 || N2 == 512) && fb == 4;
}

hipError_t launch_rowpass(int N2, int fb, const RowArgs& a, const Launch& s, const OutArgs* o) {
  constexpr int SQ = PS_ROWPASS_SQ;
  if (fb != rowpass_frames(N2)) {
    if (N2 == 256 && fb == 4) return rowpass_launch<256, 1, 4, SQ>(a, s, o);
    if (N2 == 512 && fb == 4) return rowpass_launch<512, 1, 4, SQ>(a, s, o);
    return hipErrorInvalidValue;
  }
  switch (N2) {
    case 16: return rowpass_launch<16, 8, 8, 2>(a, s, o);
    case 32: return rowpass_launch<32, 8, 8, 2>(a, s, o);
    case 64: return rowpass_launch<64, 4, 8, 2>(a, s, o);
    case 128: return rowpass_launch<128, 2, 8, 2>(a, s, o);
    case 256: return rowpass_launch<256, 1, 8, SQ>(a, s, o);
    case 512: return rowpass_launch<512, 1, 8, SQ>(a, s, o);
    case 1024: return rowpass_launch<1024, 1, 4, 1>(a, s, o);
    case 2048: return rowpass_launch<2048, 1, 2, 1>(a, s, o);
    default: return hipErrorInvalidValue;
  }
}

// ---- grouped launches: one workgroup per tile of all the launch's instances

#define PS_LAUNCH_BATCH(kernel, block, total, l, ...)                                                   \
  hipExtLaunchKernelGGL(kernel, dim3((unsigned)(total)), dim3(block), 0, (l).stream, (l).start, (l).stop, 0, __VA_ARGS__)

template <int L, int COLS, int V, int BITS>
static void colpass_batch_mode(int mode, const BatchArgs& b, const Launch& s) {
  constexpr int block = L * COLS / (8 * V);
  const ColArgs* t = static_cast<const ColArgs*>(b.tasks);
  if constexpr (BITS == 32) {
    PS_LAUNCH_BATCH((k_colpass_batch<L, COLS, V, 32, 0>), block, b.total, s, t, b.tile_end, b.n_tasks);
    return;
  }
  if (mode == 1) PS_LAUNCH_BATCH((k_colpass_batch<L, COLS, V, BITS, 1>), block, b.total, s, t, b.tile_end, b.n_tasks);
  else if (mode == 2) PS_LAUNCH_BATCH((k_colpass_batch<L, COLS, V, BITS, 2>), block, b.total, s, t, b.tile_end, b.n_tasks);
  else PS_LAUNCH_BATCH((k_colpass_batch<L, COLS, V, BITS, 0>), block, b.total, s, t, b.tile_end, b.n_tasks);
}

template <int L, int COLS, int V>
static hipError_t colpass_batch_bits(int bits, int mode, const BatchArgs& b, const Launch& s) {
  switch (bits) {
    case 2: colpass_batch_mode<L, COLS, V, 2>(mode, b, s); break;
    case 4: colpass_batch_mode<L, COLS, V, 4>(mode, b, s); break;
    case 8: colpass_batch_mode<L, COLS, V, 8>(mode, b, s); break;
    case 32: colpass_batch_mode<L, COLS, V, 32>(0, b, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_colpass_batch(int N1, int cols, int bits, int mode, const BatchArgs& b, const Launch& s) {
  constexpr int V = PS_COLPASS_V;
  if (cols != colpass_cols(N1)) {
    if (N1 == 256 && cols == 8) return colpass_batch_bits<256, 8, V>(bits, mode, b, s);
    if (N1 == 512 && cols == 8) return colpass_batch_bits<512, 8, V>(bits, mode, b, s);
    return hipErrorInvalidValue;
  }
  switch (N1) {
    case 16: return colpass_batch_bits<16, 16, 2>(bits, mode, b, s);
    case 32: return colpass_batch_bits<32, 16, 2>(bits, mode, b, s);
    case 64: return colpass_batch_bits<64, 16, 2>(bits, mode, b, s);
    case 128: return colpass_batch_bits<128, 16, 2>(bits, mode, b, s);
    case 256: return colpass_batch_bits<256, PS_COLPASS_COLS, V>(bits, mode, b, s);
    case 512: return colpass_batch_bits<512, PS_COLPASS_COLS, V>(bits, mode, b, s);
    case 1024: return colpass_batch_bits<1024, 8, 2>(bits, mode, b, s);
    case 2048: return colpass_batch_bits<2048, 4, 2>(bits, mode, b, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L, int UB, int FB, int SQ>
static hipError_t rowpass_batch_launch(const BatchArgs& b, const Launch& s) {
  constexpr int block = rowpass_threads<L, UB, FB, SQ>();
  PS_LAUNCH_BATCH((k_rowpass_batch<L, UB, FB, SQ>), block, b.total, s,
                  static_cast<const RowArgs*>(b.tasks), b.tile_end, b.n_tasks);
  return hipGetLastError();
}

hipError_t launch_rowpass_batch(int N2, int fb, const BatchArgs& b, const Launch& s) {
  constexpr int SQ = PS_ROWPASS_SQ;
  if (fb != rowpass_frames(N2)) {
    if (N2 == 256 && fb == 4) return rowpass_batch_launch<256, 1, 4, SQ>(b, s);
    if (N2 == 512 && fb == 4) return rowpass_batch_launch<512, 1, 4, SQ>(b, s);
    return hipErrorInvalidValue;
  }
  switch (N2) {
    case 16: return rowpass_batch_launch<16, 8, 8, 2>(b, s);
    case 32: return rowpass_batch_launch<32, 8, 8, 2>(b, s);
    case 64: return rowpass_batch_launch<64, 4, 8, 2>(b, s);
    case 128: return rowpass_batch_launch<128, 2, 8, 2>(b, s);
    case 256: return rowpass_batch_launch<256, 1, 8, SQ>(b, s);
    case 512: return rowpass_batch_launch<512, 1, 8, SQ>(b, s);
    case 1024: return rowpass_batch_launch<1024, 1, 4, 1>(b, s);
    case 2048: return rowpass_batch_launch<2048, 1, 2, 1>(b, s);
    default: return hipErrorInvalidValue;
  }
}

int rowpass_units_per_tile(int N2) { return N2 >= 256 ? 1 : (N2 == 128 ? 2 : (N2 == 64 ? 4 : 8)); }

int output_tiles(int N1, int N2, int P) { return output_tiles_x(N1) * output_tiles_y(N2) * P; }

hipError_t launch_output_batch(bool stokes, const BatchArgs& b, const Launch& s) {
  const OutArgs* t = static_cast<const OutArgs*>(b.tasks);
  if (stokes) PS_LAUNCH_BATCH((k_output_batch<true>), kOutThreads, b.total, s, t, b.tile_end, b.n_tasks);
  else PS_LAUNCH_BATCH((k_output_batch<false>), kOutThreads, b.total, s, t, b.tile_end, b.n_tasks);
  return hipGetLastError();
}

static dim3 output_grid(const OutArgs& a) {
  const int rt = a.N1 < 32 ? a.N1 : 32;
  const int kt = a.N2 / 2 < 16 ? a.N2 / 2 : 16;
  return dim3((unsigned)(a.N1 / rt), (unsigned)(a.N2 / 2 / kt), (unsigned)a.P);
}

hipError_t launch_stokes(const OutArgs& a, const Launch& s) {
  PS_LAUNCH((k_output<true>), output_grid(a), dim3(kOutThreads), s, a);
  return hipGetLastError();
}

hipError_t launch_spectra(const OutArgs& a, const Launch& s) {
  PS_LAUNCH((k_output<false>), output_grid(a), dim3(kOutThreads), s, a);
  return hipGetLastError();
}

hipError_t launch_unpack(const void* packed, int bits, int S, int64_t n_time, float* out, hipStream_t s) {
  const int64_t items = n_time * S;
  int64_t blocks = (items + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  const uint8_t* in = static_cast<const uint8_t*>(packed);
  switch (bits) {
    case 2: hipLaunchKernelGGL(k_unpack<2>, dim3((unsigned)blocks), dim3(256), 0, s, in, S, n_time, out); break;
    case 4: hipLaunchKernelGGL(k_unpack<4>, dim3((unsigned)blocks), dim3(256), 0, s, in, S, n_time, out); break;
    case 8: hipLaunchKernelGGL(k_unpack<8>, dim3((unsigned)blocks), dim3(256), 0, s, in, S, n_time, out); break;
    case 32: hipLaunchKernelGGL(k_unpack<32>, dim3((unsigned)blocks), dim3(256), 0, s, in, S, n_time, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hist_power(const unsigned long long* counts, int n_streams, int bits, double* power,
                             const Launch& l) {
  PS_LAUNCH(k_hist_power, dim3((unsigned)((n_streams + 63) / 64)), dim3(64), l, counts, n_streams, bits, power);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy_words, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint32_t*>(src),
                     static_cast<uint32_t*>(dst), n);
  return hipGetLastError();
}

}  // namespace ps
