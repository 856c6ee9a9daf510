// polaris_device.h -- device building blocks shared by the gfx950 kernels of the spectrometer path:
// complex helpers and small DFTs, the Stockham schedule and its register-held twiddles, LDS exchanges of
// the column and row transforms, and the decoding of packed sampler codes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "polaris_internal.h"

namespace ps {

// ------------------------------------------------------------------------------------------------
// complex helpers and small DFTs (forward, exp(-2 pi i n k / R))
// ------------------------------------------------------------------------------------------------

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// (x + i y) * (-i) = y - i x
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

template <int R>
struct Dft;

template <>
struct Dft<2> {
  static __device__ __forceinline__ void run(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  static __device__ __forceinline__ void run(float2* v) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]), t3 = cmul_mi(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <>
struct Dft<8> {
  // even/odd split into two 4-point DFTs, odd half rotated by W_8^k
  static __device__ __forceinline__ void run(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4>::run(e);
    Dft<4>::run(o);
    const float h = 0.70710678118654752440f;  // 1/sqrt(2)
    const float2 o1 = make_float2((o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h);    // * (1 - i)/sqrt2
    const float2 o2 = cmul_mi(o[2]);                                                // * (-i)
    const float2 o3 = make_float2((o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h);  // * (-1 - i)/sqrt2
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// 16-point DFT: even/odd split into two 8-point DFTs, the odd half rotated by W_16^k (W_32^k =
// exp(-2 pi i k / 32) rounded to FP32, W_16^k = W_32^(2k); the table serves a 32-point split as well).
struct W32 {
  static constexpr float c[16] = {1.0f,           9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f,
                                  7.071067812e-01f, 5.555702330e-01f, 3.826834324e-01f, 1.950903220e-01f,
                                  0.0f,           -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
                                  -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f};
  static constexpr float s[16] = {0.0f,           -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
                                  -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f,
                                  -1.0f,          -9.807852804e-01f, -9.238795325e-01f, -8.314696123e-01f,
                                  -7.071067812e-01f, -5.555702330e-01f, -3.826834324e-01f, -1.950903220e-01f};
};

// a * W_R^k for R = 16 or 32 (k < R/2, a compile-time constant after unrolling)
template <int R>
__device__ __forceinline__ float2 rot_w(float2 a, int k) {
  if (k == 0) return a;
  if (4 * k == R) return cmul_mi(a);
  const int e = k * (32 / R);
  return make_float2(a.x * W32::c[e] - a.y * W32::s[e], a.x * W32::s[e] + a.y * W32::c[e]);
}

template <int R>
struct DftSplit {
  static __device__ __forceinline__ void run(float2* v) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int m = 0; m < R / 2; ++m) {
      e[m] = v[2 * m];
      o[m] = v[2 * m + 1];
    }
    Dft<R / 2>::run(e);
    Dft<R / 2>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float2 t = rot_w<R>(o[k], k);
      v[k] = cadd(e[k], t);
      v[k + R / 2] = csub(e[k], t);
    }
  }
};
template <>
struct Dft<16> : DftSplit<16> {};

// ------------------------------------------------------------------------------------------------
// Stockham schedule for a length-L sequence held as 8 points per thread (L/8 threads per sequence).
// Pass p has radix R_p (first 2, 4 or 8, then 8) and sub-transform length NS_p = prod_{q<p} R_q.
// Task j of a radix-R pass reads points j + r*L/R, rotates them by W_(NS*R)^(r*(j mod NS)), applies the
// R-point DFT and writes them to (j / NS)*NS*R + (j mod NS) + r*NS; after the last pass the sequence is
// in natural order.  A thread with slot ts runs tasks j = ts + i*L/8, i < 8/R.
// ------------------------------------------------------------------------------------------------

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

template <int L>
struct Sched {
  static constexpr int M = ilog2c(L);
  static constexpr int R0 = (M % 3 == 0) ? 8 : ((M % 3 == 1) ? 2 : 4);
  static constexpr int NPASS = 1 + (M - ilog2c(R0)) / 3;
  static constexpr int radix(int p) { return p == 0 ? R0 : 8; }
  static constexpr int ns(int p) { return p == 0 ? 1 : R0 << (3 * (p - 1)); }
};

template <int L, int R>
__device__ __forceinline__ int pin(int ts, int i, int r) {
  return ts + i * (L / 8) + r * (L / R);
}

template <int L, int R, int NS>
__device__ __forceinline__ int pout(int ts, int i, int r) {
  const int j = ts + i * (L / 8);
  return (j / NS) * NS * R + (j & (NS - 1)) + r * NS;
}

// ------------------------------------------------------------------------------------------------
// launch helpers
// ------------------------------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Renumber them so that
// logically adjacent workgroups (which read neighbouring bytes of the same cache lines) share an XCD.
// The map is a bijection of [0, G) whatever the dispatch order.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  constexpr int X = 8;
  const int q = G / X, r = G % X, x = b % X, i = b / X;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Raw buffer resources: a wave-uniform base in SGPRs, 32-bit per-lane offsets and SGPR offsets for the
// parts that are the same across the wave, so loads and stores need no 64-bit address arithmetic.
// Accesses past num_records return zero / are dropped by the hardware.
constexpr int kBufferFlags = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferFlags);
}

// A pointer that is the same in every lane of the wave, made visibly uniform so the compiler keeps it in
// SGPRs and addresses with the scalar-base form of global loads.
typedef const __attribute__((address_space(1))) uint8_t* gbytes;

__device__ __forceinline__ gbytes uniform_gptr(const uint8_t* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gbytes)(((uint64_t)hi << 32) | lo);
}

// ------------------------------------------------------------------------------------------------
// data translation: level of one packed item (offset-binary 2/4-bit, int8, float32)
// ------------------------------------------------------------------------------------------------

template <int BITS>
__device__ __forceinline__ float level_of(const uint8_t* __restrict__ in, int64_t item) {
  if constexpr (BITS == 8) {
    return (float)(int)(int8_t)in[item];
  } else if constexpr (BITS == 32) {
    return reinterpret_cast<const float*>(in)[item];
  } else {
    const int64_t bit = item * BITS;
    const unsigned code = ((unsigned)in[bit >> 3] >> (unsigned)(bit & 7)) & ((1u << BITS) - 1u);
    return (float)(2 * (int)code - ((1 << BITS) - 1));
  }
}

// ------------------------------------------------------------------------------------------------
// per-thread pass twiddles.  A thread keeps the same slot ts for every frame it transforms, so the
// twiddles of its passes are loaded once into registers: pass p >= 1 is radix 8 with one task per thread,
// rotating point r by W_L^(r * step), step = (L / (NS * 8)) * (ts mod NS).
// ------------------------------------------------------------------------------------------------

template <int L>
struct PassTw {
  static constexpr int NP = Sched<L>::NPASS;
  float2 w[NP > 1 ? NP - 1 : 1][7];
  __device__ __forceinline__ void load(const float2* __restrict__ table, int ts) {
#pragma unroll
    for (int p = 1; p < NP; ++p) {
      const int ns = Sched<L>::ns(p);
      const int step = (L / (ns * 8)) * (ts & (ns - 1));
#pragma unroll
      for (int r = 1; r < 8; ++r) w[p - 1][r - 1] = table[r * step];
    }
  }
};

template <int L, int P>
__device__ __forceinline__ void pass_compute_reg(float2 (&v)[8], const PassTw<L>& tw) {
  constexpr int R = Sched<L>::radix(P);
  if constexpr (P > 0) {
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tw.w[P - 1][r - 1]);
  }
#pragma unroll
  for (int i = 0; i < 8 / R; ++i) Dft<R>::run(v + i * R);
}

// LDS index of element e of a row sequence.  The low five bits of e are XORed with bits 4..7 so that the
// stride-8 and stride-64 write patterns of the radix-8 passes, their unit-stride reads and the channel
// stage's forward and reversed reads all fall on distinct banks; the map stays inside each aligned block
// of 32 elements, so a sequence needs no padding.
__device__ __forceinline__ int swz(int e) {
  return e ^ (((e >> 4) & 7) | (((e >> 6) & 1) << 3) | (((e >> 7) & 1) << 4));
}

// ------------------------------------------------------------------------------------------------
// column pass: a workgroup owns COLS adjacent columns of one pair and loops over a group of frames,
// reusing its registers' pass and four-step twiddles; the next frame's input is fetched while the
// current one is transformed.  Each thread owns V adjacent columns (8 points of each).
// ------------------------------------------------------------------------------------------------

// Input of 8 rows x V adjacent columns of one thread.  Loader modes: 0 decodes every code at use; 1 (two
// streams, pair (0, 1)) and 2 (four streams) fetch the next frame's raw words ahead of use.
template <int BITS, int FAST, int V>
struct ColLoader {
  int64_t fbase;
  template <int L, int R0>
  __device__ __forceinline__ void fetch(const ColArgs&, int64_t fb, int, int) { fbase = fb; }
  template <int L, int R0>
  __device__ __forceinline__ void convert(float2 (&v)[V][8], const ColArgs& a, int ts, int n2b, int sx,
                                          int sy) const {
#pragma unroll
    for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int64_t t = fbase + (int64_t)pin<L, R0>(ts, i, r) * a.N2 + n2b;
#pragma unroll
        for (int c = 0; c < V; ++c) {
          const int64_t it = (t + c) * a.S;
          v[c][i * R0 + r] = make_float2(level_of<BITS>(a.in, it + sx), level_of<BITS>(a.in, it + sy));
        }
      }
  }
};

// NS = 2 or 4 interleaved streams of 2-, 4- or 8-bit codes: time sample t is the NS*BITS-bit field at bit
// offset NS*BITS*t, so the V adjacent columns (t a multiple of V) of a row are one word of V*NS*BITS bits
// (8 to 64), fetched ahead of use.  Two streams form the pair (0, 1); of four, the pair's streams sx, sy are
// picked from the word by shifts.
// Input words are read once: with column blocks of at least 16 columns (N1 <= 512) they are streamed past
// the caches (keeps the last-level cache for the intermediate buffer; about 4 % faster at 2^18 with input
// streamed from HBM).  Longer columns come in blocks of 8 or fewer columns, whose row segments are a
// fraction of a cache line: those loads go through L2, where the neighbouring blocks (same XCD) find the
// rest of each line.
#ifndef PS_INPUT_NONTEMPORAL
#define PS_INPUT_NONTEMPORAL 1
#endif

template <int BITS, int V, int NS>
struct ColLoaderWords {
  static_assert(BITS == 2 || BITS == 4 || BITS == 8, "word loader formats");
  static_assert(NS == 2 || NS == 4, "two or four streams");
  static constexpr int WBITS = V * NS * BITS;  // bits of one row's word
  static_assert(WBITS >= 8 && WBITS <= 64, "one load per row");
  using word = typename std::conditional<(WBITS > 32), uint64_t, uint32_t>::type;
  word raw[8];  // the row's V x NS codes
  template <class T, bool NT>
  static __device__ __forceinline__ word load(gbytes p) {
    if constexpr (NT && PS_INPUT_NONTEMPORAL)  // read once: streamed past the caches
      return (word)__builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
    else
      return (word)*(const __attribute__((address_space(1))) T*)p;
  }
  template <int L, int R0>
  __device__ __forceinline__ void fetch(const ColArgs& a, int64_t fb, int ts, int n2b) {
    // row n1 = ts + i L/8 + r L/R0 of frame fb / N: a wave-uniform 64-bit base per (frame, i, r) plus a
    // 32-bit per-lane offset (the global_load scalar-base form); byte offset of sample t: t NS BITS / 8
    const uint32_t voff = (uint32_t)(ts * a.N2 + n2b) * (NS * BITS) / 8u;
#pragma unroll
    for (int i = 0; i < 8 / R0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int64_t t0 = fb + (int64_t)a.N2 * (i * (L / 8) + r * (L / R0));
        const gbytes p = uniform_gptr(a.in + t0 * (NS * BITS) / 8) + voff;
        constexpr bool NT = L <= 512;
        if constexpr (WBITS == 64) raw[i * R0 + r] = load<uint64_t, NT>(p);
        else if constexpr (WBITS == 32) raw[i * R0 + r] = load<uint32_t, NT>(p);
        else if constexpr (WBITS == 16) raw[i * R0 + r] = load<uint16_t, NT>(p);
        else raw[i * R0 + r] = load<uint8_t, NT>(p);
      }
  }
  static __device__ __forceinline__ float lvl(word w, int field) {
    const uint32_t c = (uint32_t)(w >> (BITS * field)) & ((1u << BITS) - 1u);
    if constexpr (BITS == 8) return (float)(int)(int8_t)c;
    else return (float)(2 * (int)c - ((1 << BITS) - 1));  // offset binary
  }
  template <int L, int R0>
  __device__ __forceinline__ void convert(float2 (&v)[V][8], const ColArgs&, int, int, int sx, int sy) const {
    const int fx = NS == 2 ? 0 : sx, fy = NS == 2 ? 1 : sy;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const word w = raw[e];
#pragma unroll
      for (int c = 0; c < V; ++c) v[c][e] = make_float2(lvl(w, c * NS + fx), lvl(w, c * NS + fy));
    }
  }
};

template <int V>
struct ColLoader<8, 1, V> : ColLoaderWords<8, V, 2> {};
template <int V>
struct ColLoader<4, 1, V> : ColLoaderWords<4, V, 2> {};
template <int V>
struct ColLoader<2, 1, V> : ColLoaderWords<2, V, 2> {};
template <int V>
struct ColLoader<8, 2, V> : ColLoaderWords<8, V, 4> {};
template <int V>
struct ColLoader<4, 2, V> : ColLoaderWords<4, V, 4> {};
template <int V>
struct ColLoader<2, 2, V> : ColLoaderWords<2, V, 4> {};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// LDS tile [L][COLS]: element l of column cv*V + c at l*COLS + cv*V + c
template <int V>
__device__ __forceinline__ void tile_store(float2* __restrict__ tile, int idx, const float2 (&w)[V]) {
  if constexpr (V == 2)
    *reinterpret_cast<float4*>(tile + idx) = make_float4(w[0].x, w[0].y, w[1].x, w[1].y);
  else
    tile[idx] = w[0];
}

template <int V>
__device__ __forceinline__ void tile_load(const float2* __restrict__ tile, int idx, float2 (&w)[V]) {
  if constexpr (V == 2) {
    const float4 q = *reinterpret_cast<const float4*>(tile + idx);
    w[0] = make_float2(q.x, q.y);
    w[1] = make_float2(q.z, q.w);
  } else {
    w[0] = tile[idx];
  }
}

// Exchanges alternate between NB tiles: with two tiles a pass writes the tile the previous exchange did not
// read, so one barrier per exchange suffices (every reader of that tile has passed the previous barrier).
template <int L, int COLS, int V, int NB, int P>
__device__ __forceinline__ void col_chain(float2 (&v)[V][8], int ts, int cv, const PassTw<L>& tw,
                                          float2* __restrict__ tiles) {
  using SC = Sched<L>;
  constexpr int R = SC::radix(P), NS = SC::ns(P);
  float2* __restrict__ tile = tiles + (P % NB) * (L * COLS);
#pragma unroll
  for (int c = 0; c < V; ++c) pass_compute_reg<L, P>(v[c], tw);
  if constexpr (P + 1 < SC::NPASS) {
#pragma unroll
    for (int i = 0; i < 8 / R; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 w[V];
#pragma unroll
        for (int c = 0; c < V; ++c) w[c] = v[c][i * R + r];
        tile_store<V>(tile, pout<L, R, NS>(ts, i, r) * COLS + cv * V, w);
      }
    __syncthreads();
    constexpr int R2 = SC::radix(P + 1);
    if constexpr (V == 2) {
      // 16-byte reads of both columns; each kept whole (the empty asm takes the vector as one operand), as the
      // compiler otherwise splits some into 8-byte pairs whose lane pattern conflicts on the LDS banks
      f32x4 q[8];
#pragma unroll
      for (int i = 0; i < 8 / R2; ++i)
#pragma unroll
        for (int r = 0; r < R2; ++r)
          q[i * R2 + r] = *reinterpret_cast<const f32x4*>(tile + pin<L, R2>(ts, i, r) * COLS + cv * V);
      __builtin_amdgcn_sched_barrier(0);  // all eight reads issued before the first is waited for
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        asm("" : "+v"(q[e]));
        v[0][e] = make_float2(q[e].x, q[e].y);
        v[1][e] = make_float2(q[e].z, q[e].w);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 8 / R2; ++i)
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          float2 w[V];
          tile_load<V>(tile, pin<L, R2>(ts, i, r) * COLS + cv * V, w);
#pragma unroll
          for (int c = 0; c < V; ++c) v[c][i * R2 + r] = w[c];
        }
    }
    if constexpr (NB == 1) __syncthreads();
    col_chain<L, COLS, V, NB, P + 1>(v, ts, cv, tw, tiles);
  }
}

// ------------------------------------------------------------------------------------------------
// row pass + two-for-one split + cross power + FP64 accumulation
// UB units (row pairs) per workgroup, FB frames per batch; each thread transforms SQ row sequences (frames
// fs + j FB/SQ of a batch, same row and slot) and the first UB*L threads own one channel slot each for
// the whole launch (SPT slots each when there are fewer threads than slots).  The next batch's input is
// fetched while the current one is transformed.
// Accumulated per channel and frame, unscaled: |A + B*|^2, |A - B*|^2 and i (A + B*) conj(A - B*)
// with A = Z[k], B = Z[N - k]; the factor 1/4 that turns them into XX*, YY*, XY* is applied on output.
// ------------------------------------------------------------------------------------------------

// Exchange barrier between passes.  When a wave holds whole sequences (L/8 <= 64 threads per sequence)
// every exchange stays inside the wave: LDS operations of one wave complete in order, so ordering the
// wave's LDS writes before its reads is enough and no workgroup barrier is needed.
template <int L>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (L / 8 <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int L, int SQ, int P>
__device__ __forceinline__ void row_chain(float2 (&v)[SQ][8], int ts, const PassTw<L>& tw,
                                          float2* const (&seq)[SQ]) {
  using SC = Sched<L>;
  constexpr int R = SC::radix(P), NS = SC::ns(P);
#pragma unroll
  for (int j = 0; j < SQ; ++j) pass_compute_reg<L, P>(v[j], tw);
#pragma unroll
  for (int i = 0; i < 8 / R; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int o = swz(pout<L, R, NS>(ts, i, r));
#pragma unroll
      for (int j = 0; j < SQ; ++j) seq[j][o] = v[j][i * R + r];
    }
  if constexpr (P + 1 < SC::NPASS) {
    exchange_sync<L>();
    constexpr int R2 = SC::radix(P + 1);
#pragma unroll
    for (int i = 0; i < 8 / R2; ++i)
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int o = swz(pin<L, R2>(ts, i, r));
#pragma unroll
        for (int j = 0; j < SQ; ++j) v[j][i * R2 + r] = seq[j][o];
      }
    exchange_sync<L>();
    row_chain<L, SQ, P + 1>(v, ts, tw, seq);
  }
}

// Wide rows (L = 1024, 2048): a row held as 16 points per thread (T = L/16 threads: one wave for 1024
// points, two for 2048), with three passes of radix 8, R1 = L/128 and 16 (two exchanges, where 8 points per
// thread need four passes and three exchanges).  The thread's points are ts + k T (k < 16); task
// j = ts + i T (i < 16/R) of a radix-R pass takes registers i + r 16/R (points j + r L/R), rotates input r by
// W_(NS R)^(r (j mod NS)), applies the R-point DFT and writes output r to (j / NS) NS R + (j mod NS) + r NS.
// NS (1, 8, 8 R1) divides T, so j mod NS = ts mod NS for every task of the thread, and its pass twiddles are
// loaded once.  After the last pass the row is in natural order.
template <int L>
struct WideTw {
  static constexpr int T = L / 16, R1 = L / 128;
  float2 w1[R1 - 1], w2[15];
  // table: W_(L ST)^m, m < L ST (ST = 2: the table of a transform twice as long)
  template <int ST = 1>
  __device__ __forceinline__ void load(const float2* __restrict__ table, int ts) {
    const int m1 = ts & 7, m2 = ts & (8 * R1 - 1);
#pragma unroll
    for (int r = 1; r < R1; ++r) w1[r - 1] = table[r * m1 * 16 * ST];  // W_(8 R1)^(r m1)
#pragma unroll
    for (int r = 1; r < 16; ++r) w2[r - 1] = table[r * m2 * ST];       // W_L^(r m2)
  }
};

template <int L, int P>
__device__ __forceinline__ void wide_pass(float2 (&v)[16], const WideTw<L>& tw, int ts, float2* __restrict__ seq) {
  constexpr int T = L / 16, R1 = L / 128;
  constexpr int R = P == 0 ? 8 : (P == 1 ? R1 : 16), NT = 16 / R, NS = P == 0 ? 1 : (P == 1 ? 8 : 8 * R1);
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    float2 t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = v[i + r * NT];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      if constexpr (P == 1) t[r] = cmul(t[r], tw.w1[r - 1]);
      if constexpr (P == 2) t[r] = cmul(t[r], tw.w2[r - 1]);
    }
    Dft<R>::run(t);
    const int j = ts + i * T;
#pragma unroll
    for (int r = 0; r < R; ++r) seq[swz((j / NS) * NS * R + (j % NS) + r * NS)] = t[r];
  }
}

template <int L>
__device__ __forceinline__ void wide_chain(float2 (&v)[16], int ts, const WideTw<L>& tw, float2* __restrict__ seq) {
  constexpr int T = L / 16;
  wide_pass<L, 0>(v, tw, ts, seq);
  exchange_sync<8 * T>();  // within the wave for one-wave rows, else a workgroup barrier
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = seq[swz(ts + k * T)];
  exchange_sync<8 * T>();
  wide_pass<L, 1>(v, tw, ts, seq);
  exchange_sync<8 * T>();
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = seq[swz(ts + k * T)];
  exchange_sync<8 * T>();
  wide_pass<L, 2>(v, tw, ts, seq);
}

// FP64 complex arithmetic
struct cd {
  double x, y;
};
__device__ __forceinline__ cd cdm(cd a, cd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cd cda(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd cdc(cd a) { return {a.x, -a.y}; }

}  // namespace ps
