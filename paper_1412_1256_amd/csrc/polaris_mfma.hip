// polaris_mfma.hip -- precision form of the spectrometer path: the FFT passes in FP16 or BF16 as blocked
// DFT matrix products on the gfx950 matrix cores (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulate), the
// integration of the products in FP64 or in compensated (Kahan) FP32.
//
// The frame transform keeps the four-step structure of the plain path (Sec. 2: segmentation, FFT, cross
// products, accumulation; N = N1 * N2, pair z = x + i*y).  Each N1- or N2-point DFT is itself split as
// 16 x R: n = R*a + b, k = kappa + 16*kb,
//   stage A: Y[kappa][b] = sum_a W16^(a*kappa) z[R*a + b]          (16 vectors b per matrix product)
//   twiddle: Y *= W_L^(b*kappa) / 16                                 (FP32, then rounded to 16 bits)
//   stage B: Z[kappa + 16*kb] = sum_b WR^(b*kb) Y[kappa][b] / R      (16 vectors of 16 columns or kappas)
//
// A DFT of radix r applied to 16 vectors is one r x r complex matrix product.  With the complex values as
// (re, im) pairs it is a 2r x 2r real product, which maps onto 16x16x32 matrix instructions: the vectors
// are the 16 columns of the B operand, each lane holding 4 consecutive complex points (8 halves) of one
// vector, and the outputs come back 4 complex points per lane in the same arrangement.  The DFT matrix is
// given as hi + lo parts in the 16-bit format (two products), so its own rounding error is of order
// 2^-22 (FP16) or 2^-16 (BF16); the remaining error is the rounding of the data between stages.
//
// Lane layouts of v_mfma_f32_16x16x32 (lane l, g = l / 16, n = l % 16):
//   A (16 x 32): row n, columns 8g .. 8g+7;  B (32 x 16): rows 8g .. 8g+7, column n;
//   C (16 x 16): rows 4g .. 4g+3, column n.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "polaris.h"
#include "polaris_device.h"
#include "polaris_internal.h"

namespace ps {
namespace {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t w4v __attribute__((ext_vector_type(4)));

// (re, im) rounded to nearest even in the 16-bit format, re in the low half
template <int PREC>
__device__ __forceinline__ uint32_t pk(float re, float im) {
  if constexpr (PREC == PS_PREC_FP16) {
    const _Float16 a = (_Float16)re, b = (_Float16)im;
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  } else {
    const __bf16 a = (__bf16)re, b = (__bf16)im;
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
}

template <int PREC>
__device__ __forceinline__ f4v mma(w4v a, w4v b, f4v c) {
  if constexpr (PREC == PS_PREC_FP16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a), __builtin_bit_cast(h8v, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v, a), __builtin_bit_cast(b8v, b), c, 0,
                                                   0, 0);
}

// DFT matrix of radix r in A-operand lane layout: [hi, lo][tile t = 2*qb + part][K-step s][lane][4 words].
// Tile (qb, part) gives the real (part 0) or imaginary (part 1) parts of outputs 16*qb .. 16*qb+15; K-step s
// takes input points 16*s .. 16*s+15.
template <int r>
struct Mat {
  static constexpr int NT = 2 * r / 16, NS = r / 16;
  w4v hi[NT][NS], lo[NT][NS];
  __device__ __forceinline__ void load(const uint32_t* __restrict__ m, int lane) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        hi[t][s] = *reinterpret_cast<const w4v*>(m + (((0 * NT + t) * NS + s) * 64 + lane) * 4);
        lo[t][s] = *reinterpret_cast<const w4v*>(m + (((1 * NT + t) * NS + s) * 64 + lane) * 4);
      }
  }
  // o[t] = tile t of the product with the vectors x[s] (FP32)
  template <int PREC>
  __device__ __forceinline__ void apply(const w4v (&x)[NS], f4v (&o)[NT]) const {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      f4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = mma<PREC>(hi[t][s], x[s], acc);
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = mma<PREC>(lo[t][s], x[s], acc);
      o[t] = acc;
    }
  }
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Input samples of the pair (x, y) at time t of the launch.  MODE 1: int8, two streams, pair (0, 1): one
// 16-bit word.  MODE 2: int8, four streams: one 32-bit word holding every stream.  MODE 0: any format,
// decoded item by item.
template <int BITS, int MODE>
struct MxIn {
  uint32_t raw;
  // fb: wave-uniform base of the frame's samples (bytes); off: this sample's time index within the frame
  __device__ __forceinline__ void fetch(gbytes fb, uint32_t off) {
    if constexpr (MODE == 1) raw = *(const __attribute__((address_space(1))) uint16_t*)(fb + 2u * off);
    else if constexpr (MODE == 2) raw = *(const __attribute__((address_space(1))) uint32_t*)(fb + 4u * off);
    else raw = 0;
  }
  __device__ __forceinline__ float2 level(const ColArgs& c, int64_t t, int sx, int sy) const {
    if constexpr (MODE == 1) {
      return make_float2((float)(int)(int8_t)(raw & 0xffu), (float)(int)(int8_t)(raw >> 8));
    } else if constexpr (MODE == 2) {
      return make_float2((float)(int)(int8_t)(raw >> (8 * sx)), (float)(int)(int8_t)(raw >> (8 * sy)));
    } else {
      return make_float2(level_of<BITS>(c.in, t * c.S + sx), level_of<BITS>(c.in, t * c.S + sy));
    }
  }
};

// ------------------------------------------------------------------------------------------------
// column pass: a workgroup of 4 waves transforms 16 adjacent columns (all N1 rows) of a frame, for a
// group of frames.  Stage A: wave w handles b = 4q + j for the quads q = w + 4t; the results go to LDS as
// [kappa][column][b].  Stage B: wave w handles kappa = w + 4t, then the four-step twiddle W_N^(k1*n2) / R,
// and the packed 16-bit result is written to T[f][p][k1][n2].
// ------------------------------------------------------------------------------------------------
template <int R, int PREC, int BITS, int MODE>
__global__ void __launch_bounds__(256) k_colpass_mx(MxColArgs a) {
  constexpr int N1 = 16 * R;
  constexpr int NQ = R / 16;  // b-quads per wave
  constexpr int XS = R + 4;   // words per (kappa, column) row of the exchange, 16-byte aligned rows
  __shared__ __align__(16) uint32_t X[16 * 16 * XS];
  __shared__ float2 tws[N1];
  const ColArgs& c = a.col;
  const int tid = (int)threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, n = lane & 15;
  const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int cb = blk % c.n_colblk;
  const int rest = blk / c.n_colblk;
  const int p = rest % c.P;
  const int grp = rest / c.P;
  const int f_begin = grp * c.frames_per_block;
  const int f_end = min(c.n_frames, f_begin + c.frames_per_block);
  const int n2 = cb * 16 + n;
  const int sx = c.px[p], sy = c.py[p];

  for (int i = tid; i < N1; i += 256) tws[i] = a.m.tws[i];
  const gbytes win = c.win ? uniform_gptr(reinterpret_cast<const uint8_t*>(c.win)) : nullptr;
  Mat<16> A16;
  Mat<R> AR;
  A16.load(a.m.a16, lane);
  AR.load(a.m.aR, lane);
  // four-step twiddles W_N^(k1 * n2), k1 = kappa + 16 kb: t1 for this wave's kappas, t2 for this lane's kb
  const int mask = (1 << c.lo_bits) - 1;
  float2 t1[4], t2[NQ][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int m = (w + 4 * t) * n2;
    t1[t] = cmul(c.tw_hi[m >> c.lo_bits], c.tw_lo[m & mask]);
  }
#pragma unroll
  for (int qb = 0; qb < NQ; ++qb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * (16 * qb + 4 * g + i) * n2;
      const float2 v = cmul(c.tw_hi[m >> c.lo_bits], c.tw_lo[m & mask]);
      t2[qb][i] = make_float2(v.x * (1.0f / R), v.y * (1.0f / R));
    }
  __syncthreads();

  MxIn<BITS, MODE> in[NQ][4][4];  // [quad][j][point a = 4g + jj]
  constexpr int BPT = MODE == 1 ? 2 : 4;  // bytes per time step on the word paths
  auto fetch = [&](int f) {
    if constexpr (MODE != 0) {
      const gbytes fb = uniform_gptr(c.in + (int64_t)f * c.N * BPT);
#pragma unroll
      for (int t = 0; t < NQ; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int b = 4 * (w + 4 * t) + j;
            const int n1 = R * (4 * g + jj) + b;
            in[t][j][jj].fetch(fb, (uint32_t)(n1 * c.N2 + n2));
          }
    }
  };
  if (f_begin < f_end) fetch(f_begin);
  for (int f = f_begin; f < f_end; ++f) {
    // ---- stage A
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int q = w + 4 * t;
      uint32_t Y[4][4];  // [i][j]
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = 4 * q + j;
        w4v xb[1];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int n1 = R * (4 * g + jj) + b;
          const int64_t tt = (int64_t)f * c.N + (int64_t)n1 * c.N2 + n2;
          float2 v = in[t][j][jj].level(c, tt, sx, sy);
          if (win) {
            const float wv = *(const __attribute__((address_space(1))) float*)(win + 4u * (uint32_t)(n1 * c.N2 + n2));
            v = make_float2(v.x * wv, v.y * wv);
          }
          xb[0][jj] = pk<PREC>(v.x, v.y);
        }
        f4v o[2];
        A16.template apply<PREC>(xb, o);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float2 tw = tws[(b * (4 * g + i)) & (N1 - 1)];
          Y[i][j] = pk<PREC>(o[0][i] * tw.x - o[1][i] * tw.y, o[0][i] * tw.y + o[1][i] * tw.x);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const w4v v = {Y[i][0], Y[i][1], Y[i][2], Y[i][3]};
        *reinterpret_cast<w4v*>(&X[((4 * g + i) * 16 + n) * XS + 4 * q]) = v;
      }
    }
    if (f + 1 < f_end) fetch(f + 1);
    __syncthreads();
    // ---- stage B and the four-step twiddle
    const gbytes Tf = uniform_gptr(reinterpret_cast<const uint8_t*>(a.T + ((int64_t)f * c.P + p) * (int64_t)N1 * c.N2));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int kap = w + 4 * t;
      w4v xs[NQ];
#pragma unroll
      for (int s = 0; s < NQ; ++s) xs[s] = *reinterpret_cast<const w4v*>(&X[(kap * 16 + n) * XS + 16 * s + 4 * g]);
      f4v o[2 * NQ];
      AR.template apply<PREC>(xs, o);
#pragma unroll
      for (int qb = 0; qb < NQ; ++qb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k1 = kap + 16 * (16 * qb + 4 * g + i);
          const float2 tw = cmul(t1[t], t2[qb][i]);
          const float2 z = make_float2(o[2 * qb][i], o[2 * qb + 1][i]);
          const float2 v = cmul(z, tw);
          *(__attribute__((address_space(1))) uint32_t*)(Tf + 4u * (uint32_t)(k1 * c.N2 + n2)) = pk<PREC>(v.x, v.y);
        }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------------
// row pass: a workgroup owns one unit (rows k1 and N1 - k1, or 0 and N1/2) of one pair; wave w takes the
// frames f = w, w + 4, ...  For each row, stage A (vectors b = 16h + n) goes through a wave-private LDS
// exchange to stage B (vectors kappa); the spectra of both rows go to LDS, and each lane forms XX*, YY*,
// XY* of its channel slots and integrates them in registers.  At the end the four waves' sums are added in
// wave order, unscaled (an exact power of two) and stored into the FP64 accumulators.
// ------------------------------------------------------------------------------------------------
template <int R, int PREC, bool KAHAN>
__global__ void __launch_bounds__(256, 2) k_rowpass_mx(MxRowArgs a) {
  constexpr int N2 = 16 * R;
  constexpr int NQ = R / 16;
  constexpr int NW = 4;
  constexpr int XS = R + 4;
  constexpr int SPL = N2 / 64;          // channel slots per lane
  constexpr int SP = N2 + N2 / 16;      // padded spectrum row
  constexpr int WAVE_BYTES = 16 * XS * 4 + 2 * SP * 8;
  constexpr int LOOP_BYTES = NW * WAVE_BYTES;
  constexpr int SUM_BYTES = (NW - 1) * 64 * SPL * 4 * 8;
  __shared__ __align__(16) unsigned char lds[LOOP_BYTES > SUM_BYTES ? LOOP_BYTES : SUM_BYTES];
  const int tid = (int)threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, n = lane & 15;
  const int u = (int)blockIdx.x, p = (int)blockIdx.y;
  const int N1 = a.N1, U = N1 / 2;
  const int rows[2] = {u == 0 ? 0 : u, u == 0 ? N1 / 2 : N1 - u};
  uint32_t* X = reinterpret_cast<uint32_t*>(lds + w * WAVE_BYTES);
  float2* spec = reinterpret_cast<float2*>(lds + w * WAVE_BYTES + 16 * XS * 4);

  Mat<16> A16;
  Mat<R> AR;
  A16.load(a.m.a16, lane);
  AR.load(a.m.aR, lane);
  float2 tw[NQ][4];  // W_N2^(b * kappa) / 16 for b = 16h + n, kappa = 4g + i
#pragma unroll
  for (int h = 0; h < NQ; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) tw[h][i] = a.m.tws[((16 * h + n) * (4 * g + i)) & (N2 - 1)];

  using acc_t = typename std::conditional<KAHAN, float, double>::type;
  acc_t sum[SPL][4], cmp[SPL][4];
#pragma unroll
  for (int m = 0; m < SPL; ++m)
#pragma unroll
    for (int k = 0; k < 4; ++k) sum[m][k] = cmp[m][k] = 0;

  uint32_t raw[2][NQ][4];
  auto fetch = [&](int f) {
    const gbytes fb = uniform_gptr(reinterpret_cast<const uint8_t*>(a.T + ((int64_t)f * a.P + p) * N1 * N2));
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int h = 0; h < NQ; ++h)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          raw[r][h][jj] = *(const __attribute__((address_space(1))) uint32_t*)(
              fb + 4u * (uint32_t)(rows[r] * N2 + R * (4 * g + jj) + 16 * h + n));
  };
  if (w < a.n_frames) fetch(w);
  for (int f = w; f < a.n_frames; f += NW) {
    uint32_t cur[2][NQ][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int h = 0; h < NQ; ++h)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) cur[r][h][jj] = raw[r][h][jj];
    if (f + NW < a.n_frames) fetch(f + NW);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int h = 0; h < NQ; ++h) {
        w4v xb[1] = {{cur[r][h][0], cur[r][h][1], cur[r][h][2], cur[r][h][3]}};
        f4v o[2];
        A16.template apply<PREC>(xb, o);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float2 t = tw[h][i];
          X[(4 * g + i) * XS + 16 * h + n] = pk<PREC>(o[0][i] * t.x - o[1][i] * t.y, o[0][i] * t.y + o[1][i] * t.x);
        }
      }
      wave_sync();
      w4v xs[NQ];
#pragma unroll
      for (int s = 0; s < NQ; ++s) xs[s] = *reinterpret_cast<const w4v*>(&X[n * XS + 16 * s + 4 * g]);
      f4v o[2 * NQ];
      AR.template apply<PREC>(xs, o);
#pragma unroll
      for (int qb = 0; qb < NQ; ++qb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k2 = n + 16 * (16 * qb + 4 * g + i);
          spec[r * SP + k2 + (k2 >> 4)] = make_float2(o[2 * qb][i], o[2 * qb + 1][i]);
        }
      wave_sync();
    }
#pragma unroll
    for (int m = 0; m < SPL; ++m) {
      const int s = lane + 64 * m;
      const int half = s / (N2 / 2), k2 = s % (N2 / 2);
      // bin (row, k2) pairs with bin N - k: rows k1 and N1 - k1 swap and k2 -> N2 - 1 - k2; row 0 -> N2 - k2
      const int phalf = (u == 0) ? half : 1 - half;
      const int pk2 = (u == 0 && half == 0) ? ((N2 - k2) & (N2 - 1)) : (N2 - 1 - k2);
      const float2 A = spec[half * SP + k2 + (k2 >> 4)];
      const float2 B = spec[phalf * SP + pk2 + (pk2 >> 4)];
      const float sx_ = A.x + B.x, sy_ = A.y - B.y;  // A + conj(B) = 2 X
      const float dx_ = A.x - B.x, dy_ = A.y + B.y;  // A - conj(B) = 2i Y
      const float v[4] = {sx_ * sx_ + sy_ * sy_, dx_ * dx_ + dy_ * dy_, sx_ * dy_ - sy_ * dx_,
                          sx_ * dx_ + sy_ * dy_};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if constexpr (KAHAN) {
          const float y = v[k] - cmp[m][k];
          const float t = sum[m][k] + y;
          cmp[m][k] = (t - sum[m][k]) - y;
          sum[m][k] = t;
        } else {
          sum[m][k] += (double)v[k];
        }
      }
    }
    wave_sync();
  }
  // ---- combine the waves' sums in wave order
  __syncthreads();
  double* part = reinterpret_cast<double*>(lds);
  if (w > 0) {
#pragma unroll
    for (int m = 0; m < SPL; ++m)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        part[(((w - 1) * SPL + m) * 4 + k) * 64 + lane] = (double)sum[m][k] - (double)cmp[m][k];
  }
  __syncthreads();
  if (w == 0) {
    double* acc = a.acc + (int64_t)(p * U + u) * 4 * N2;
#pragma unroll
    for (int m = 0; m < SPL; ++m) {
      const int s = lane + 64 * m;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double t = (double)sum[m][k] - (double)cmp[m][k];
#pragma unroll
        for (int v = 0; v < NW - 1; ++v) t += part[((v * SPL + m) * 4 + k) * 64 + lane];
        t *= a.unscale;
        acc[k * N2 + s] = a.first ? t : acc[k * N2 + s] + t;
      }
    }
  }
}

#define PS_LAUNCH(kernel, grid, block, l, ...) \
  hipExtLaunchKernelGGL(kernel, grid, block, 0, (l).stream, (l).start, (l).stop, 0, __VA_ARGS__)

template <int R, int PREC>
hipError_t colpass_mx_bits(int bits, const MxColArgs& a, int n_blocks, const Launch& l) {
  const dim3 grid((unsigned)n_blocks), block(256);
  switch (a.mode) {
    case 1: PS_LAUNCH((k_colpass_mx<R, PREC, 8, 1>), grid, block, l, a); break;
    case 2: PS_LAUNCH((k_colpass_mx<R, PREC, 8, 2>), grid, block, l, a); break;
    default:
      switch (bits) {
        case 2: PS_LAUNCH((k_colpass_mx<R, PREC, 2, 0>), grid, block, l, a); break;
        case 4: PS_LAUNCH((k_colpass_mx<R, PREC, 4, 0>), grid, block, l, a); break;
        case 8: PS_LAUNCH((k_colpass_mx<R, PREC, 8, 0>), grid, block, l, a); break;
        case 32: PS_LAUNCH((k_colpass_mx<R, PREC, 32, 0>), grid, block, l, a); break;
        default: return hipErrorInvalidValue;
      }
  }
  return hipGetLastError();
}

template <int R>
hipError_t rowpass_mx_r(int prec, int accum, const MxRowArgs& a, const Launch& l) {
  const dim3 grid((unsigned)(a.N1 / 2), (unsigned)a.P), block(256);
  const bool kahan = accum == PS_ACC_KAHAN32;
  if (prec == PS_PREC_FP16) {
    if (kahan) PS_LAUNCH((k_rowpass_mx<R, PS_PREC_FP16, true>), grid, block, l, a);
    else PS_LAUNCH((k_rowpass_mx<R, PS_PREC_FP16, false>), grid, block, l, a);
  } else if (prec == PS_PREC_BF16) {
    if (kahan) PS_LAUNCH((k_rowpass_mx<R, PS_PREC_BF16, true>), grid, block, l, a);
    else PS_LAUNCH((k_rowpass_mx<R, PS_PREC_BF16, false>), grid, block, l, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_colpass_mx(int N1, int prec, int bits, const MxColArgs& a, int n_blocks, const Launch& l) {
  if (prec == PS_PREC_FP16) {
    if (N1 == 256) return colpass_mx_bits<16, PS_PREC_FP16>(bits, a, n_blocks, l);
    if (N1 == 512) return colpass_mx_bits<32, PS_PREC_FP16>(bits, a, n_blocks, l);
  } else if (prec == PS_PREC_BF16) {
    if (N1 == 256) return colpass_mx_bits<16, PS_PREC_BF16>(bits, a, n_blocks, l);
    if (N1 == 512) return colpass_mx_bits<32, PS_PREC_BF16>(bits, a, n_blocks, l);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rowpass_mx(int N2, int prec, int accum, const MxRowArgs& a, const Launch& l) {
  if (N2 == 256) return rowpass_mx_r<16>(prec, accum, a, l);
  if (N2 == 512) return rowpass_mx_r<32>(prec, accum, a, l);
  return hipErrorInvalidValue;
}

}  // namespace ps
