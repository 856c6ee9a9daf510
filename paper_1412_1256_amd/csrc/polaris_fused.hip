// Single-pass transform of short frames (N = 2^8 .. 2^12): the whole frame of a pair, z = x + i y, lives in
// LDS (at most 36 KB with padding, beside a copy of the twiddle table), is transformed in place by radix-8 Stockham passes
// (N/8 threads, one radix-8 task per thread and pass), and the cross-power products of
// its channels are added to FP64 registers; only the packed input is read from HBM.  A workgroup is one
// accumulator slot of one pair: absolute frame a of the integration belongs to slot a mod G, and the
// workgroup adds its frames in order, then writes the slot in the layout of the four-step row pass, so
// Stokes, spectra, state export and the backward read it unchanged.
#include <hip/hip_ext.h>

#include "polaris_fused.h"
#include "polaris_device.h"

namespace ps {

namespace {

__host__ __device__ constexpr int fused_nt(int N) { return N / 8; }

// LDS positions: one pad point per 8 frame points and per 32 twiddles, so that the stride-8 and
// stride-64 writes of the first passes and the twiddle reads fall on distinct banks
__device__ __forceinline__ int zp(int i) { return i + (i >> 3); }
__device__ __forceinline__ int tp(int i) { return i + (i >> 5); }

// raw word holding item `item` of a frame whose first item is at the wave-uniform base (32-bit lane
// offsets): the byte of a 2-, 4- or 8-bit code, or the bits of a float
template <int BITS>
__device__ __forceinline__ uint32_t frame_raw(gbytes base, uint32_t item) {
  if constexpr (BITS == 32) return *(const __attribute__((address_space(1))) uint32_t*)(base + 4u * item);
  else return (uint32_t)*(base + ((item * BITS) >> 3));
}

template <int BITS>
__device__ __forceinline__ float raw_level(uint32_t raw, uint32_t item) {
  if constexpr (BITS == 8) {
    return (float)(int)(int8_t)(uint8_t)raw;
  } else if constexpr (BITS == 32) {
    return __uint_as_float(raw);
  } else {
    const unsigned code = (raw >> ((item * BITS) & 7u)) & ((1u << BITS) - 1u);
    return (float)(2 * (int)code - ((1 << BITS) - 1));
  }
}

// One Stockham pass of radix R over the N points in LDS: task j reads points j + r N/R, rotates them by
// W_(NS R)^(r (j mod NS)) (twiddle W_N^(r (j mod NS) N/(NS R)) from the table), applies the R-point DFT and
// writes them to (j / NS) NS R + (j mod NS) + r NS.  Reads and writes are separated by barriers, so the
// pass runs in place.
template <int N, int NT, int R, int NS>
__device__ __forceinline__ void fused_pass(float2* __restrict__ z, const float2* __restrict__ tw, const int t) {
  constexpr int TPT = N / R / NT;  // tasks per thread
  static_assert(TPT >= 1 && TPT * NT * R == N, "tasks cover the frame");
  float2 v[TPT][R];
#pragma unroll
  for (int i = 0; i < TPT; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r) v[i][r] = z[zp(t + i * NT + r * (N / R))];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    const int j = t + i * NT;
    const int jm = j & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[tp(r * jm * (N / (NS * R)))]);
    }
    Dft<R>::run(v[i]);
    const int base = (j - jm) * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) z[zp(base + r * NS)] = v[i][r];
  }
  __syncthreads();
}

// passes P .. of the schedule: first radix R0 (sub-length 1), then radix 8
template <int N, int NT, int R0, int P, int NS>
__device__ __forceinline__ void fused_passes(float2* z, const float2* tw, const int t) {
  if constexpr (NS < N) {
    constexpr int R = P == 0 ? R0 : 8;
    fused_pass<N, NT, R, NS>(z, tw, t);
    fused_passes<N, NT, R0, P + 1, NS * R>(z, tw, t);
  }
}

template <int N, int BITS>
__global__ void __launch_bounds__(fused_nt(N)) k_fused(FusedArgs a) {
  constexpr int NT = fused_nt(N);
  constexpr int M = ilog2c(N);
  constexpr int R0 = (M % 3 == 0) ? 8 : ((M % 3 == 1) ? 2 : 4);
  constexpr int EPT = N / NT;        // points loaded per thread
  constexpr int CPT = N / 2 / NT;    // channels owned per thread
  __shared__ __align__(16) float2 z[N + N / 8];
  __shared__ __align__(16) float2 twl[N + N / 32];  // W_N^m, copied once per workgroup
  const int t = (int)threadIdx.x;
  const int g = (int)blockIdx.x, p = (int)blockIdx.y;
  const int sx = a.px[p], sy = a.py[p];
  // this slot's frames of the launch: f = f_first + j G (absolute frame F0 + f = g mod G)
  const int f_first = (int)(((int64_t)g - a.F0 % a.G + a.G) % a.G);
  if (f_first >= a.n_frames) return;
  const int n_loc = (a.n_frames - f_first + a.G - 1) / a.G;
  const bool prior = a.F0 > g;  // the slot already holds frames of this integration
  const int U = a.N1 / 2, L = a.N2;

  // channel k = k1 + N1 k2 (k1 < N1, k2 < N2/2) sits in unit u of row half `half` (the row pass's layout)
  double* slot = a.acc + (int64_t)g * a.slot_stride;
  int at[CPT];
  double sxx[CPT], syy[CPT], sxr[CPT], sxi[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int k = t + c * NT;
    const int k1 = k & (a.N1 - 1), k2 = k / a.N1;
    int u, half;
    if (k1 == 0) { u = 0; half = 0; }
    else if (2 * k1 == a.N1) { u = 0; half = 1; }
    else if (2 * k1 < a.N1) { u = k1; half = 0; }
    else { u = a.N1 - k1; half = 1; }
    at[c] = (p * U + u) * 4 * L + half * (L / 2) + k2;
    sxx[c] = syy[c] = sxr[c] = sxi[c] = 0.0;
    if (prior) {
      sxx[c] = slot[at[c]];
      syy[c] = slot[at[c] + L];
      sxr[c] = slot[at[c] + 2 * L];
      sxi[c] = slot[at[c] + 3 * L];
    }
  }

  for (int i = t; i < N; i += NT) twl[tp(i)] = a.tw[i];
  // raw codes of the next frame, fetched while the current one is transformed
  uint32_t rx[EPT], ry[EPT];
  auto fetch = [&](int jf) {
    const int64_t t0 = (int64_t)(f_first + jf * a.G) * a.hop;
    const gbytes fb = uniform_gptr(a.in + t0 * a.S * BITS / 8);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const uint32_t it = (uint32_t)((t + e * NT) * a.S);
      rx[e] = frame_raw<BITS>(fb, it + sx);
      ry[e] = frame_raw<BITS>(fb, it + sy);
    }
  };
  fetch(0);
  for (int jf = 0; jf < n_loc; ++jf) {
    // the window is re-read (from cache) every frame: an opaque zero in its index keeps the compiler from
    // holding it in registers across the frame loop
    int z0;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z0));
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int n = t + e * NT;
      const uint32_t it = (uint32_t)(n * a.S);
      const float w = a.win[n + z0];
      z[zp(n)] = make_float2(raw_level<BITS>(rx[e], it + sx) * w, raw_level<BITS>(ry[e], it + sy) * w);
    }
    __syncthreads();
    if (jf + 1 < n_loc) fetch(jf + 1);
    fused_passes<N, NT, R0, 0, 1>(z, twl, t);
    // Z[k] and Z[N - k]: A + conj B = 2 X, A - conj B = 2i Y; 4 XX*, 4 YY*, 4 XY* (as the row pass)
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int k = t + c * NT;
      const float2 A = z[zp(k)], B = z[zp((N - k) & (N - 1))];
      const float sx_ = A.x + B.x, sy_ = A.y - B.y;
      const float dx_ = A.x - B.x, dy_ = A.y + B.y;
      sxx[c] += (double)(sx_ * sx_ + sy_ * sy_);
      syy[c] += (double)(dx_ * dx_ + dy_ * dy_);
      sxr[c] += (double)(sx_ * dy_ - sy_ * dx_);
      sxi[c] += (double)(sx_ * dx_ + sy_ * dy_);
    }
    __syncthreads();  // the next frame overwrites z
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    slot[at[c]] = sxx[c];
    slot[at[c] + L] = syy[c];
    slot[at[c] + 2 * L] = sxr[c];
    slot[at[c] + 3 * L] = sxi[c];
  }
}

template <int N>
hipError_t fused_bits(int bits, const FusedArgs& a, const Launch& l) {
  const dim3 grid((unsigned)a.G, (unsigned)a.P), block(fused_nt(N));
  switch (bits) {
    case 2: hipExtLaunchKernelGGL((k_fused<N, 2>), grid, block, 0, l.stream, l.start, l.stop, 0, a); break;
    case 4: hipExtLaunchKernelGGL((k_fused<N, 4>), grid, block, 0, l.stream, l.start, l.stop, 0, a); break;
    case 8: hipExtLaunchKernelGGL((k_fused<N, 8>), grid, block, 0, l.stream, l.start, l.stop, 0, a); break;
    case 32: hipExtLaunchKernelGGL((k_fused<N, 32>), grid, block, 0, l.stream, l.start, l.stop, 0, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// stage 1: part[c][e] = sum of slots c*kReduceChunk .. in order; stage 2: out[e] = sum of part[c][e] in order
__global__ void __launch_bounds__(256) k_slot_chunks(const double* __restrict__ acc, int64_t elems, int slots,
                                                     int64_t slot_stride, double* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = (int)blockIdx.y;
  if (e >= elems) return;
  const int g1 = min(slots, (c + 1) * kReduceChunk);
  double s = 0.0;
#pragma unroll 8
  for (int g = c * kReduceChunk; g < g1; ++g) s += acc[(int64_t)g * slot_stride + e];  // loads issue 8 at a time
  part[(int64_t)c * elems + e] = s;
}

__global__ void __launch_bounds__(256) k_slot_total(const double* __restrict__ part, int64_t elems, int chunks,
                                                    double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= elems) return;
  double s = 0.0;
#pragma unroll 8
  for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * elems + e];
  out[e] = s;
}

}  // namespace

int fused_threads(int N) { return fused_nt(N); }

hipError_t launch_slot_reduce(const double* acc, int64_t elems, int slots, int64_t slot_stride, double* part,
                              double* out, const Launch& l) {
  const int chunks = (int)slot_reduce_chunks(slots);
  const unsigned gx = (unsigned)((elems + 255) / 256);
  hipExtLaunchKernelGGL(k_slot_chunks, dim3(gx, (unsigned)chunks), dim3(256), 0, l.stream, l.start, nullptr, 0, acc,
                        elems, slots, slot_stride, part);
  hipExtLaunchKernelGGL(k_slot_total, dim3(gx), dim3(256), 0, l.stream, nullptr, l.stop, 0, part, elems, chunks, out);
  return hipGetLastError();
}

hipError_t launch_fused(int N, int bits, const FusedArgs& a, const Launch& l) {
  switch (N) {
    case 1 << 8: return fused_bits<1 << 8>(bits, a, l);
    case 1 << 9: return fused_bits<1 << 9>(bits, a, l);
    case 1 << 10: return fused_bits<1 << 10>(bits, a, l);
    case 1 << 11: return fused_bits<1 << 11>(bits, a, l);
    case 1 << 12: return fused_bits<1 << 12>(bits, a, l);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ps
