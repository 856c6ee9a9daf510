// polaris_mfma.hip -- precision form of the spectrometer path: the FFT passes in FP16 or BF16 as blocked
// DFT matrix products on the gfx950 matrix cores (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulate), the
// integration of the products in FP64 or in compensated (Kahan) FP32.
//
// The frame transform keeps the four-step structure of the plain path (Sec. 2: segmentation, FFT, cross
// products, accumulation; N = N1 * N2, pair z = x + i*y).  Each N1- or N2-point DFT is itself split as
// 16 x R: n = R*a + b, k = kappa + 16*kb,
//   stage A: Y[kappa][b] = sum_a W16^(a*kappa) z[R*a + b]          (16 vectors b per matrix product)
//   twiddle: Y *= W_L^(b*kappa) / 16                                 (FP32, then rounded to 16 bits)
//   stage B: Z[kappa + 16*kb] = sum_b WR^(b*kb) Y[kappa][b] / R      (16 vectors of 16 columns or kappas;
//            for R = 32 a radix-2 butterfly in FP32 and two radix-16 products)
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

typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));

// (re, im) rounded to nearest even in the 16-bit format, re in the low half (one packed conversion on
// gfx950: v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32)
template <int PREC>
__device__ __forceinline__ uint32_t pk(float re, float im) {
  const f2v v = {re, im};
  if constexpr (PREC == PS_PREC_FP16) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, h2v));
  else return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2v));
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
// 16-bit word.  MODE 2: int8, four streams: one 32-bit word holding every stream.  MODE 3: as MODE 2 with
// the pairs (0, 2) and (1, 3), both transformed by the workgroup that reads the word.  MODE 0: any format,
// decoded item by item.
template <int BITS, int MODE>
struct MxIn {
  uint32_t raw;
  // buffer load of the launch's input: voff the lane's byte offset, soff the wave-uniform byte offset
  __device__ __forceinline__ void fetch(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
    if constexpr (MODE == 1) raw = __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0);
    else if constexpr (MODE >= 2) raw = __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0);
    else raw = 0;
  }
  __device__ __forceinline__ float2 level(const ColArgs& c, int64_t t, int sx, int sy) const {
    if constexpr (MODE == 1) {
      return make_float2((float)(int)(int8_t)(raw & 0xffu), (float)(int)(int8_t)(raw >> 8));
    } else if constexpr (MODE >= 2) {  // (MODE 3: sx, sy are constants after unrolling, so byte selects)
      return make_float2((float)(int)(int8_t)(raw >> (8 * sx)), (float)(int)(int8_t)(raw >> (8 * sy)));
    } else {
      return make_float2(level_of<BITS>(c.in, t * c.S + sx), level_of<BITS>(c.in, t * c.S + sy));
    }
  }
};

// ------------------------------------------------------------------------------------------------
// Radix-32 stage B as a radix-2 butterfly and two radix-16 products.  With b = b_lo + 16 b_hi and the stage A
// outputs Y (twiddle not yet applied),
//   Z[2m]   = sum_blo W16^(blo m) W_L^(blo kappa) (Y[blo] + W32^kappa Y[blo + 16]) / 16
//   Z[2m+1] = sum_blo W16^(blo m) W_L^(blo (kappa + 16)) (Y[blo] - W32^kappa Y[blo + 16]) / 16
// (W_L^(16 kappa) = W32^kappa for L = 512), so one radix-16 matrix serves every stage and the butterfly runs
// in FP32 before the rounding to 16 bits.  H = R / 16 is the number of such halves (1 for R = 16).
// ------------------------------------------------------------------------------------------------

// column pass: a workgroup of 4 waves transforms 16 adjacent columns (all N1 rows) of a frame, for a group
// of frames.  Stage A: wave w handles b_lo = 4w + j (and b_lo + 16); the results go to LDS as
// [half][kappa][column][b_lo].  Stage B: wave w handles kappa = w + 4t, then the four-step twiddle
// W_N^(k1*n2) / R, and the packed 16-bit result is written to T[f][p][k1][n2].
template <int R, int N2, int PREC, int BITS, int MODE, bool WIN>
__global__ void __launch_bounds__(256, 2) k_colpass_mx(MxColArgs a) {
  constexpr int N1 = 16 * R;
  constexpr int H = R / 16;
  constexpr int XS = 20;  // words per (half, kappa, column) row: 16 points + 4 of padding (16-byte aligned)
  __shared__ __align__(16) uint32_t X[H * 16 * 16 * XS];
  __shared__ float2 tws[N1];
  const ColArgs& c = a.col;
  const int tid = (int)threadIdx.x, lane = tid & 63, g = lane >> 4, n = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
  const int blk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  constexpr int NPP = MODE == 3 ? 2 : 1;  // pairs transformed by the workgroup
  const int cb = blk % c.n_colblk;
  const int rest = blk / c.n_colblk;
  const int p0 = NPP == 2 ? 0 : rest % c.P;
  const int grp = NPP == 2 ? rest : rest / c.P;
  const int f_begin = grp * c.frames_per_block;
  const int f_end = min(c.n_frames, f_begin + c.frames_per_block);
  const int n2 = cb * 16 + n;
  // Addresses: a wave-uniform base (SGPRs) per element, which changes with the frame, plus one per-lane
  // offset shared by every element, so no per-element offsets stay live across the frame loop.
  const uint32_t lane_t = (uint32_t)(4 * R * g * N2 + n2);                // time index, lane part
  const uint32_t lane_o = (uint32_t)(16 * H * 4 * g * N2 + n2) * 4u;     // output byte offset, lane part

  for (int i = tid; i < N1; i += 256) tws[i] = a.m.tws[i];
  Mat<16> A16;
  A16.load(a.m.a16, lane);
  // four-step twiddles W_N^(k1 * n2) / R of this lane's outputs k1 = kappa + 16 kb, kappa = w + 4t,
  // kb = H (4g + i) + half, as the product t1[t] * t2[half][i] = W_N^(kappa n2) * W_N^(16 kb n2) / R
  const int mask = (1 << c.lo_bits) - 1;
  float2 t1[4], t2[H][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int m = (w + 4 * t) * n2;
    t1[t] = cmul(c.tw_hi[m >> c.lo_bits], c.tw_lo[m & mask]);
  }
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * (H * (4 * g + i) + h) * n2;
      const float2 v = cmul(c.tw_hi[m >> c.lo_bits], c.tw_lo[m & mask]);
      t2[h][i] = make_float2(v.x * (1.0f / R), v.y * (1.0f / R));
    }
  __syncthreads();
  // W32^kappa for kappa = 4g + i (the stage twiddle table holds W_N1^m / 16)
  float2 w32[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float2 v = tws[(16 * (4 * g + i)) & (N1 - 1)];
    w32[i] = make_float2(16.0f * v.x, 16.0f * v.y);
  }

  MxIn<BITS, MODE> in[4][H][4];  // [j][b_hi][point a = 4g + jj]
  constexpr int BPT = MODE == 1 ? 2 : 4;  // bytes per time step on the word paths
  // time index of element (j, h, jj) within the frame: lane_t + (R jj + 4w + j + 16h) N2
  // the word paths read through a buffer resource over the launch's input (fewer than 2^31 bytes): the
  // frame and element offsets are wave-uniform (scalar registers), the lane's offset one 32-bit register
  const __amdgpu_buffer_rsrc_t rin = buffer_rsrc(c.in, c.in_bytes);
  auto fetch = [&](int f) {
    if constexpr (MODE != 0) {
      const uint32_t fo = ((uint32_t)__builtin_amdgcn_readfirstlane(f) * (uint32_t)c.hop + 4u * w * N2) * BPT;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            in[j][h][jj].fetch(rin, lane_t * BPT, fo + (uint32_t)((R * jj + j + 16 * h) * N2 * BPT));
    }
  };
  if (f_begin < f_end) fetch(f_begin);
  for (int f = f_begin; f < f_end; ++f) {
#pragma unroll
    for (int pp = 0; pp < NPP; ++pp) {
      const int p = p0 + pp;
      const int sx = NPP == 2 ? pp : c.px[p], sy = NPP == 2 ? pp + 2 : c.py[p];
      // the stage twiddles are read from LDS in every frame: an opaque zero keeps the compiler from holding
      // all of them in registers across the frame loop
      int z0;
      asm volatile("v_mov_b32 %0, 0" : "=v"(z0));
      // ---- stage A (and the radix-2 butterfly of a radix-32 stage B)
      uint32_t Y[H][4][4];  // [half][i][j]
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = 4 * w + j;
        f4v o[H][2];
#pragma unroll
        for (int h = 0; h < H; ++h) {
          w4v xb[1];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int64_t tt = (int64_t)f * c.hop + (int64_t)(R * jj + b + 16 * h) * N2 + lane_t;
            float2 v = in[j][h][jj].level(c, tt, sx, sy);
            if constexpr (WIN) {
              const gbytes wb = uniform_gptr(reinterpret_cast<const uint8_t*>(c.win + (R * jj + b + 16 * h) * N2));
              const float wv = *(const __attribute__((address_space(1))) float*)(wb + 4u * lane_t);
              v = make_float2(v.x * wv, v.y * wv);
            }
            xb[0][jj] = pk<PREC>(v.x, v.y);
          }
          A16.template apply<PREC>(xb, o[h]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int kap = 4 * g + i;
          const float2 y0 = make_float2(o[0][0][i], o[0][1][i]);
          if constexpr (H == 1) {
            const float2 t = tws[((b * kap) & (N1 - 1)) + z0];
            Y[0][i][j] = pk<PREC>(y0.x * t.x - y0.y * t.y, y0.x * t.y + y0.y * t.x);
          } else {
            const float2 v = cmul(w32[i], make_float2(o[1][0][i], o[1][1][i]));
            const float2 s0 = cadd(y0, v), d0 = csub(y0, v);
            const float2 ta = tws[((b * kap) & (N1 - 1)) + z0];
            const float2 tb = tws[((b * (kap + 16)) & (N1 - 1)) + z0];
            Y[0][i][j] = pk<PREC>(s0.x * ta.x - s0.y * ta.y, s0.x * ta.y + s0.y * ta.x);
            Y[1][i][j] = pk<PREC>(d0.x * tb.x - d0.y * tb.y, d0.x * tb.y + d0.y * tb.x);
          }
        }
      }
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const w4v v = {Y[h][i][0], Y[h][i][1], Y[h][i][2], Y[h][i][3]};
          *reinterpret_cast<w4v*>(&X[((h * 16 + 4 * g + i) * 16 + n) * XS + 4 * w]) = v;
        }
      // the next frame's words, once the last pair's stage A has used this frame's: issued here, not earlier,
      // so they do not hold registers through stage A; unconditional (the last frame fetches itself again),
      // see the row pass
      if (pp == NPP - 1) {
        __builtin_amdgcn_sched_barrier(0);
        fetch(min(f + 1, f_end - 1));
      }
      __syncthreads();
      // ---- stage B and the four-step twiddle
      const uint32_t* Tf = a.T + ((int64_t)__builtin_amdgcn_readfirstlane(f) * c.P + p) * (int64_t)N1 * N2;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kap = w + 4 * t;
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const w4v xs[1] = {*reinterpret_cast<const w4v*>(&X[((h * 16 + kap) * 16 + n) * XS + 4 * g])};
          f4v o[2];
          A16.template apply<PREC>(xs, o);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            // k1 = kap + 16 (H (4g + i) + h): lane part 16 H 4g, uniform part kap + 16 (H i + h)
            const float2 v = cmul(make_float2(o[0][i], o[1][i]), cmul(t1[t], t2[h][i]));
            // global stores (the next kernel reads the buffer from every XCD), frame base and row offset in
            // scalar registers, the lane's offset one 32-bit register
            const gbytes ob = uniform_gptr(reinterpret_cast<const uint8_t*>(Tf + (kap + 16 * (H * i + h)) * N2));
            *(__attribute__((address_space(1))) uint32_t*)(ob + lane_o) = pk<PREC>(v.x, v.y);
          }
        }
      }
      __syncthreads();
    }
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
  constexpr int H = R / 16;
  constexpr int NW = 4;
  constexpr int XS = 20;
  constexpr int SPL = N2 / 64;          // channel slots per lane
  constexpr int SP = N2 + N2 / 16;      // padded spectrum row
  constexpr int WAVE_BYTES = H * 16 * XS * 4 + 2 * SP * 8;
  constexpr int LOOP_BYTES = NW * WAVE_BYTES;
  constexpr int SUM_BYTES = (NW - 1) * 64 * SPL * 4 * 8;
  __shared__ __align__(16) unsigned char lds[LOOP_BYTES > SUM_BYTES ? LOOP_BYTES : SUM_BYTES];
  const int tid = (int)threadIdx.x, lane = tid & 63, g = lane >> 4, n = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
  const int u = (int)blockIdx.x, p = (int)blockIdx.y;
  const int N1 = a.N1, U = N1 / 2;
  const int rows[2] = {u == 0 ? 0 : u, u == 0 ? N1 / 2 : N1 - u};
  uint32_t* X = reinterpret_cast<uint32_t*>(lds + w * WAVE_BYTES);
  float2* spec = reinterpret_cast<float2*>(lds + w * WAVE_BYTES + H * 16 * XS * 4);

  Mat<16> A16;
  A16.load(a.m.a16, lane);
  // stage twiddles (W_N2^m / 16 in the table) for b_lo = n, kappa = 4g + i; W32^kappa unscaled
  float2 ta[4], tb[4], w32[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int kap = 4 * g + i;
    ta[i] = a.m.tws[(n * kap) & (N2 - 1)];
    tb[i] = a.m.tws[(n * (kap + 16)) & (N2 - 1)];
    const float2 v = a.m.tws[(16 * kap) & (N2 - 1)];
    w32[i] = make_float2(16.0f * v.x, 16.0f * v.y);
  }

  using acc_t = typename std::conditional<KAHAN, float, double>::type;
  acc_t sum[SPL][4], cmp[SPL][4];
#pragma unroll
  for (int m = 0; m < SPL; ++m)
#pragma unroll
    for (int k = 0; k < 4; ++k) sum[m][k] = cmp[m][k] = 0;

  uint32_t raw[2][H][4];
  // buffer loads over one frame of the pair: the row and element offsets are wave-uniform, the lane's
  // offset (column R (4g) + n) one 32-bit register
  const uint32_t lane_c = (uint32_t)(R * 4 * g + n) * 4u;
  auto fetch = [&](int f) {
    const uint32_t* Tf = a.T + ((int64_t)__builtin_amdgcn_readfirstlane(f) * a.P + p) * N1 * N2;
    const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(Tf, (uint32_t)(N1 * N2 * 4));
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          raw[r][h][jj] = __builtin_amdgcn_raw_buffer_load_b32(rs, lane_c, (uint32_t)(rows[r] * N2 + R * jj + 16 * h) * 4u, 0);
  };
  // prefetches are unconditional (past the end a wave fetches its last frame again), so each frame waits
  // only for its own loads and the next frame's stay in flight
  if (w < a.n_frames) fetch(w);
  for (int f = w; f < a.n_frames; f += NW) {
    uint32_t cur[2][H][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) cur[r][h][jj] = raw[r][h][jj];
    fetch(f + NW < a.n_frames ? f + NW : f);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      f4v o[H][2];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const w4v xb[1] = {{cur[r][h][0], cur[r][h][1], cur[r][h][2], cur[r][h][3]}};
        A16.template apply<PREC>(xb, o[h]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 y0 = make_float2(o[0][0][i], o[0][1][i]);
        if constexpr (H == 1) {
          X[(4 * g + i) * XS + n] = pk<PREC>(y0.x * ta[i].x - y0.y * ta[i].y, y0.x * ta[i].y + y0.y * ta[i].x);
        } else {
          const float2 v = cmul(w32[i], make_float2(o[1][0][i], o[1][1][i]));
          const float2 s0 = cadd(y0, v), d0 = csub(y0, v);
          X[(4 * g + i) * XS + n] = pk<PREC>(s0.x * ta[i].x - s0.y * ta[i].y, s0.x * ta[i].y + s0.y * ta[i].x);
          X[(16 + 4 * g + i) * XS + n] =
              pk<PREC>(d0.x * tb[i].x - d0.y * tb[i].y, d0.x * tb[i].y + d0.y * tb[i].x);
        }
      }
      wave_sync();
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const w4v xs[1] = {*reinterpret_cast<const w4v*>(&X[(h * 16 + n) * XS + 4 * g])};
        f4v z[2];
        A16.template apply<PREC>(xs, z);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k2 = n + 16 * (H * (4 * g + i) + h);
          spec[r * SP + k2 + (k2 >> 4)] = make_float2(z[0][i], z[1][i]);
        }
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

// int8 word paths (no window), or item-by-item decoding of any format with or without a window
template <int R, int N2, int PREC, bool WIN>
hipError_t colpass_mx_generic(int bits, const MxColArgs& a, const dim3& grid, const Launch& l) {
  const dim3 block(256);
  switch (bits) {
    case 2: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 2, 0, WIN>), grid, block, l, a); break;
    case 4: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 4, 0, WIN>), grid, block, l, a); break;
    case 8: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 8, 0, WIN>), grid, block, l, a); break;
    case 32: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 32, 0, WIN>), grid, block, l, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int R, int N2, int PREC>
hipError_t colpass_mx_bits(int bits, const MxColArgs& a, int n_blocks, const Launch& l) {
  const dim3 grid((unsigned)n_blocks), block(256);
  if (a.col.win) return colpass_mx_generic<R, N2, PREC, true>(bits, a, grid, l);
  switch (a.mode) {
    case 1: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 8, 1, false>), grid, block, l, a); break;
    case 2: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 8, 2, false>), grid, block, l, a); break;
    case 3: PS_LAUNCH((k_colpass_mx<R, N2, PREC, 8, 3, false>), grid, block, l, a); break;
    default: return colpass_mx_generic<R, N2, PREC, false>(bits, a, grid, l);
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t colpass_mx_prec(int N1, int N2, int bits, const MxColArgs& a, int n_blocks, const Launch& l) {
  if (N1 == 256 && N2 == 256) return colpass_mx_bits<16, 256, PREC>(bits, a, n_blocks, l);
  if (N1 == 256 && N2 == 512) return colpass_mx_bits<16, 512, PREC>(bits, a, n_blocks, l);
  if (N1 == 512 && N2 == 512) return colpass_mx_bits<32, 512, PREC>(bits, a, n_blocks, l);
  return hipErrorInvalidValue;
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
  if (prec == PS_PREC_FP16) return colpass_mx_prec<PS_PREC_FP16>(N1, a.col.N2, bits, a, n_blocks, l);
  if (prec == PS_PREC_BF16) return colpass_mx_prec<PS_PREC_BF16>(N1, a.col.N2, bits, a, n_blocks, l);
  return hipErrorInvalidValue;
}

hipError_t launch_rowpass_mx(int N2, int prec, int accum, const MxRowArgs& a, const Launch& l) {
  if (N2 == 256) return rowpass_mx_r<16>(prec, accum, a, l);
  if (N2 == 512) return rowpass_mx_r<32>(prec, accum, a, l);
  return hipErrorInvalidValue;
}

}  // namespace ps
