// Post-integration reductions on integrated spectra: channel averaging with flags (Sec. 4), the smoothed
// bandpass and the bandpass variation (Sec. 3.3.2), band moments and the Allan variances of Eq. 3 / Eq. 4
// (Sec. 3.3.1, 3.3.3).  These run once per integration or per series on data of a few MB, so they are
// latency-bound; sums are FP64 in a fixed order (run-to-run identical results).
#include "polaris_post.h"

#include <math.h>

#include <mutex>

namespace ps {

namespace {

constexpr int kNT = 256;  // threads per workgroup

// Sum of v over the workgroup in a fixed order: wave butterflies, then wave partials in order.  Every thread
// gets the result.  sh: kNT / 64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();  // earlier readers of sh are done
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kNT / 64; ++w) r += sh[w];
  return r;
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

// ------------------------------------------------------------------------------------------------
// channel averaging: bins of `factor` channels, flagged and non-finite channels left out

// factor <= kSpan: a workgroup stages the span of nb = kSpan / factor whole bins of one spectrum in LDS
// (coalesced loads).  Bins of fewer than 64 channels are then summed by one thread each, in channel order;
// a bin of 64 or more by a wave: lane j adds the channels j, j + 64, ... in order and the 64 lane sums are
// added by a fixed butterfly (one thread per bin had the lanes of a wave a whole bin apart in LDS, on the
// same banks, each waiting on a chain of factor reads: 16.4 -> 9.7 us for 30 spectra at factor 256; at
// factor 32 the wave form was slower, 9.3 against 5.7 us).
constexpr int kSpan = 2048;

__global__ void __launch_bounds__(kNT) k_chan_avg_span(ChanAvgArgs a) {
  __shared__ float v[kSpan];
  __shared__ uint8_t ok[kSpan];
  const int64_t s = blockIdx.y;
  const int F = a.factor;
  const int nb = kSpan / F;
  const int64_t n_bins = a.n_chan / F;
  const int64_t b0 = (int64_t)blockIdx.x * nb;
  const int nbl = (int)((n_bins - b0) < nb ? (n_bins - b0) : nb);
  const int span = nbl * F;
  const float* row = a.in + s * a.n_chan + b0 * F;
  for (int i = (int)threadIdx.x; i < span; i += kNT) {
    const float x = row[i];
    const bool use = isfinite(x) && !(a.flags && a.flags[b0 * F + i]);
    v[i] = use ? x : 0.0f;
    ok[i] = use ? 1 : 0;
  }
  __syncthreads();
  if (F < 64) {
    for (int b = (int)threadIdx.x; b < nbl; b += kNT) {
      double sum = 0.0;
      int n = 0;
      for (int i = 0; i < F; ++i) {
        sum += (double)v[b * F + i];
        n += ok[b * F + i];
      }
      const int64_t o = s * n_bins + b0 + b;
      a.out[o] = n ? (float)(sum / n) : NAN;
      if (a.counts) a.counts[o] = n;
    }
    return;
  }
  const int lane = (int)threadIdx.x % 64;
  for (int b = (int)threadIdx.x / 64; b < nbl; b += kNT / 64) {  // the same rounds for a whole wave
    double sum = 0.0;
    int n = 0;
    for (int i = lane; i < F; i += 64) {
      sum += (double)v[b * F + i];
      n += ok[b * F + i];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sum += __shfl_xor(sum, o, 64);
      n += __shfl_xor(n, o, 64);
    }
    if (lane == 0) {
      const int64_t o = s * n_bins + b0 + b;
      a.out[o] = n ? (float)(sum / n) : NAN;
      if (a.counts) a.counts[o] = n;
    }
  }
}

// factor > kSpan: one workgroup per (spectrum, bin)
__global__ void __launch_bounds__(kNT) k_chan_avg_wide(ChanAvgArgs a) {
  __shared__ double sh[kNT / 64];
  const int64_t s = blockIdx.y, b = blockIdx.x;
  const int64_t n_bins = a.n_chan / a.factor;
  const int64_t c0 = b * a.factor;
  double sum = 0.0, n = 0.0;
  for (int64_t i = threadIdx.x; i < a.factor; i += kNT) {
    const float x = a.in[s * a.n_chan + c0 + i];
    if (isfinite(x) && !(a.flags && a.flags[c0 + i])) {
      sum += (double)x;
      n += 1.0;
    }
  }
  sum = block_sum(sum, sh);
  n = block_sum(n, sh);
  if (threadIdx.x == 0) {
    a.out[s * n_bins + b] = n > 0.0 ? (float)(sum / n) : NAN;
    if (a.counts) a.counts[s * n_bins + b] = (int32_t)n;
  }
}

// ------------------------------------------------------------------------------------------------
// smoothed bandpass: least-squares cubic spline, uniform knots every K channels from c0

// the four uniform cubic B-spline pieces at local position u of an interval
__device__ __forceinline__ void bspline4(double u, double (&b)[4]) {
  const double u2 = u * u, u3 = u2 * u, v = 1.0 - u;
  b[0] = v * v * v / 6.0;
  b[1] = (3.0 * u3 - 6.0 * u2 + 4.0) / 6.0;
  b[2] = (-3.0 * u3 + 3.0 * u2 + 3.0 * u + 1.0) / 6.0;
  b[3] = u3 / 6.0;
}

// one workgroup per knot interval j: the interval's contributions to the normal equations, Gram entries
// G[q][p] (q <= p, ten of them) of basis functions j + q, j + p and right-hand sides r[q]
__global__ void __launch_bounds__(kNT) k_spline_gram(SplineArgs a) {
  __shared__ double sh[kNT / 64];
  const int64_t j = blockIdx.x;
  const int64_t lo = a.c0 + j * a.K;
  const int64_t hi = (lo + a.K) < a.c1 ? (lo + a.K) : a.c1;
  double g[14];
#pragma unroll
  for (int q = 0; q < 14; ++q) g[q] = 0.0;
  for (int64_t c = lo + threadIdx.x; c < hi; c += kNT) {
    double b[4];
    bspline4((double)(c - lo) / (double)a.K, b);
    const double h = (double)a.h[c];
    int k = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int p = q; p < 4; ++p) g[k++] += b[q] * b[p];
#pragma unroll
    for (int q = 0; q < 4; ++q) g[10 + q] += b[q] * h;
  }
#pragma unroll
  for (int q = 0; q < 14; ++q) {
    const double t = block_sum(g[q], sh);
    if (threadIdx.x == 0) a.partial[j * 14 + q] = t;
  }
}

// index of G[q][p] (q <= p) in an interval's ten Gram entries
__device__ __forceinline__ int gidx(int q, int p) {
  constexpr int start[4] = {0, 4, 7, 9};
  return start[q] + (p - q);
}

// One workgroup: the threads assemble the banded normal matrix (row i: A[i][i-3 .. i]) and the right-hand
// side in LDS from the interval partials; one thread then factors A = L L^T (banded Cholesky, keeping the
// last three rows of L in registers and each finished row of L in place of A's, the diagonal as its
// reciprocal so that the recurrence has one division and one square root per row), solves L y = r on the
// way, and solves L^T a = y backwards from LDS.
__global__ void __launch_bounds__(kNT) k_spline_solve(SplineArgs a) {
  __shared__ double lds[5 * kMaxSplineCoef];
  double* A = lds;                  // [n_coef][4], A[i][3 - d] = A(i, i - d)
  double* r = lds + 4 * a.n_coef;   // [n_coef]
  const int64_t n = a.n_coef;
  for (int64_t i = threadIdx.x; i < n; i += kNT) {
    double row[4] = {0.0, 0.0, 0.0, 0.0}, rhs = 0.0;
    // intervals j = i - 3 .. i touch basis function i (as j + q, q = i - j)
    for (int q = 0; q < 4; ++q) {
      const int64_t j = i - q;
      if (j < 0 || j >= a.n_int) continue;
      const double* G = a.partial + j * 14;
      rhs += G[10 + q];
      for (int p = 0; p <= q; ++p) row[3 - (q - p)] += G[gidx(p, q)];  // A(i, j + p), j + p = i - (q - p)
    }
    for (int d = 0; d < 4; ++d) A[i * 4 + d] = row[d];
    r[i] = rhs;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  // L rows i-3, i-2, i-1 (each as L(k, k-3 .. k-1) and 1 / L(k, k)) and y
  double Lm[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};  // Lm[0] = row i-1, Lm[1] = i-2, Lm[2] = i-3
  double ym[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    double Li[4];
    // L(i, i-d) for d = 3, 2, 1, then the diagonal
    for (int d = 3; d >= 1; --d) {
      if (i - d < 0) {
        Li[3 - d] = 0.0;
        continue;
      }
      // sum over k = i-3 .. i-d-1 of L(i, k) L(i-d, k); row i-d is Lm[d-1], its entry L(i-d, k) at 3-(i-d-k)
      double s = A[i * 4 + 3 - d];
      for (int e = 3; e > d; --e) {  // k = i - e
        const double lik = Li[3 - e];
        const double ldk = Lm[d - 1][3 - (e - d)];
        s -= lik * ldk;
      }
      Li[3 - d] = s * Lm[d - 1][3];
    }
    double dg = A[i * 4 + 3];
    for (int e = 1; e <= 3; ++e) dg -= Li[3 - e] * Li[3 - e];
    Li[3] = 1.0 / sqrt(dg);
    double y = r[i];
    for (int e = 1; e <= 3; ++e) y -= Li[3 - e] * ym[e - 1];
    y *= Li[3];
    for (int q = 0; q < 4; ++q) A[i * 4 + q] = Li[q];  // row i of A is no longer needed
    r[i] = y;
    for (int q = 0; q < 4; ++q) {
      Lm[2][q] = Lm[1][q];
      Lm[1][q] = Lm[0][q];
      Lm[0][q] = Li[q];
    }
    ym[2] = ym[1];
    ym[1] = ym[0];
    ym[0] = y;
  }
  // L^T a = y: a_i = (y_i - sum_{e=1..3} L(i+e, i) a_{i+e}) / L(i, i)  (A[i][3] holds 1 / L(i, i))
  double am[3] = {0, 0, 0};  // a_{i+1}, a_{i+2}, a_{i+3}
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = r[i];
    for (int e = 1; e <= 3; ++e)
      if (i + e < n) s -= A[(i + e) * 4 + 3 - e] * am[e - 1];
    const double ai = s * A[i * 4 + 3];
    a.coef[i] = ai;
    am[2] = am[1];
    am[1] = am[0];
    am[0] = ai;
  }
}

__global__ void __launch_bounds__(kNT) k_spline_eval(SplineArgs a) {
  const int64_t c = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (c >= a.n_chan) return;
  if (c < a.c0 || c >= a.c1) {
    a.smooth[c] = NAN;
    return;
  }
  const int64_t j = (c - a.c0) / a.K;
  double b[4];
  bspline4((double)(c - a.c0 - j * a.K) / (double)a.K, b);
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) v += a.coef[j + q] * b[q];
  a.smooth[c] = (float)v;
}

// ------------------------------------------------------------------------------------------------

__global__ void __launch_bounds__(kNT) k_bandpass_correct(const float* __restrict__ hk, int64_t n_chan,
                                                          const float* __restrict__ smooth,
                                                          const double* __restrict__ gain,
                                                          float* __restrict__ out) {
  const int64_t s = blockIdx.y;
  const int64_t c = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (c >= n_chan) return;
  const double g = gain ? gain[s] : 1.0;
  out[s * n_chan + c] = (float)((double)hk[s * n_chan + c] / (g * (double)smooth[c]));
}

// one workgroup per spectrum: mean of the finite channels, then the root mean square deviation from it
__global__ void __launch_bounds__(kNT) k_band_stats(const float* __restrict__ x, int64_t n_chan,
                                                    double* __restrict__ mean_sd) {
  __shared__ double sh[kNT / 64];
  const float* row = x + (int64_t)blockIdx.x * n_chan;
  double s = 0.0, n = 0.0;
  for (int64_t c = threadIdx.x; c < n_chan; c += kNT) {
    const float v = row[c];
    if (isfinite(v)) {
      s += (double)v;
      n += 1.0;
    }
  }
  s = block_sum(s, sh);
  n = block_sum(n, sh);
  const double m = n > 0.0 ? s / n : NAN;
  double q = 0.0;
  for (int64_t c = threadIdx.x; c < n_chan; c += kNT) {
    const float v = row[c];
    if (isfinite(v)) q += ((double)v - m) * ((double)v - m);
  }
  q = block_sum(q, sh);
  if (threadIdx.x == 0) {
    mean_sd[2 * blockIdx.x] = m;
    mean_sd[2 * blockIdx.x + 1] = n > 0.0 ? sqrt(q / n) : NAN;
  }
}

// Eq. 3 / Eq. 4, block form: workgroup (chunk c, series s) covers the points t of chunk c and writes, per lag
// L, the sum of squared second differences (x[t+L] - 2 x[t] + x[t-L])^2 over its t with all three samples
// finite and their count, and (normalised) the sum and count of its finite points; a second kernel adds
// the chunks of each series in order.
__global__ void __launch_bounds__(kNT) k_allan_part(AllanArgs a, int64_t chunks) {
  __shared__ double sh[kNT / 64];
  const int64_t s_ = blockIdx.x, c = blockIdx.y;
  const float* x = a.x + s_ * a.series_stride;
  const int64_t P = a.n_points, st = a.point_stride;
  const int64_t t0 = c * kAllanChunk, t1 = (t0 + kAllanChunk) < P ? (t0 + kAllanChunk) : P;
  double* out = a.part + (s_ * chunks + c) * (a.n_lags + 1) * 2;
  if (a.normalize) {
    double s = 0.0, n = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kNT) {
      const float v = x[t * st];
      if (isfinite(v)) {
        s += (double)v;
        n += 1.0;
      }
    }
    s = block_sum(s, sh);
    n = block_sum(n, sh);
    if (threadIdx.x == 0) {
      out[2 * a.n_lags] = s;
      out[2 * a.n_lags + 1] = n;
    }
  }
  for (int l = 0; l < a.n_lags; ++l) {
    const int64_t L = a.lags[l];
    double s = 0.0, n = 0.0;
    const int64_t lo = t0 > L ? t0 : L, hi = t1 < P - L ? t1 : P - L;
    for (int64_t t = lo + threadIdx.x; t < hi; t += kNT) {
      const double d = (double)x[(t + L) * st] - 2.0 * (double)x[t * st] + (double)x[(t - L) * st];
      if (finite(d)) {
        s += d * d;
        n += 1.0;
      }
    }
    s = block_sum(s, sh);
    n = block_sum(n, sh);
    if (threadIdx.x == 0) {
      out[2 * l] = s;
      out[2 * l + 1] = n;
    }
  }
}

__global__ void __launch_bounds__(kNT) k_allan_total(AllanArgs a, int64_t chunks) {
  const int64_t s_ = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (s_ >= a.n_series) return;
  const double* part = a.part + s_ * chunks * (a.n_lags + 1) * 2;
  // the chunks' (sum, count) pairs of field f added in chunk order, their loads issued eight chunks at a time
  // (one chunk at a time, each add waited for its own load)
  auto chunk_sum = [&](int f, double& s, double& n) {
    const int64_t rec = (int64_t)(a.n_lags + 1) * 2;
    const double* q = part + 2 * f;
    int64_t c = 0;
    for (; c + 8 <= chunks; c += 8) {
      double v[8][2];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        v[j][0] = q[(c + j) * rec];
        v[j][1] = q[(c + j) * rec + 1];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        s += v[j][0];
        n += v[j][1];
      }
    }
    for (; c < chunks; ++c) {
      s += q[c * rec];
      n += q[c * rec + 1];
    }
  };
  double mean2 = 1.0;
  if (a.normalize) {
    double s = 0.0, n = 0.0;
    chunk_sum(a.n_lags, s, n);
    const double m = s / n;
    mean2 = m * m;
  }
  for (int l = 0; l < a.n_lags; ++l) {
    double s = 0.0, n = 0.0;
    chunk_sum(l, s, n);
    const double tau = (double)a.lags[l] * a.spacing;
    a.out[s_ * a.n_lags + l] = n > 0.0 ? s / n / (2.0 * tau * tau) / mean2 : NAN;
  }
}

// The same for series stored side by side (series_stride 1, e.g. one series per channel of a run of
// integrations [t][channel]): a wave holds 64 consecutive series, so its loads are consecutive addresses, and
// the t range of each series is cut into kColsSlices slices handled by the workgroup's waves (one thread per
// series and slice: a single thread sweeping all t paid one memory round trip per step).  One sweep serves
// up to 8 lags (their sums in registers), so the rows t - L, t, t + L of nearby lags are reused from cache;
// each slice adds its terms in t order and the slices' sums are added in slice order (a fixed order).
constexpr int kColsSeries = 64, kColsSlices = 4;

__global__ void __launch_bounds__(kColsSeries * kColsSlices) k_allan_cols(AllanArgs a) {
  constexpr int LG = 8;
  __shared__ double red[kColsSlices][LG][2][kColsSeries];
  __shared__ double msum[kColsSlices][2][kColsSeries];
  const int lane = (int)threadIdx.x % kColsSeries, slice = (int)threadIdx.x / kColsSeries;
  const int64_t s = (int64_t)blockIdx.x * kColsSeries + lane;
  const bool valid = s < a.n_series;  // every thread still takes part in the barriers
  const float* x = a.x + (valid ? s : 0);
  const int64_t P = a.n_points, st = a.point_stride;
  const int64_t t0 = P * slice / kColsSlices, t1 = P * (slice + 1) / kColsSlices;
  double mean2 = 1.0;
  if (a.normalize) {
    double sum = 0.0, n = 0.0;
    if (valid)
      for (int64_t t = t0; t < t1; ++t) {
        const float v = x[t * st];
        if (isfinite(v)) {
          sum += (double)v;
          n += 1.0;
        }
      }
    msum[slice][0][lane] = sum;
    msum[slice][1][lane] = n;
    __syncthreads();
    double S = 0.0, N = 0.0;
#pragma unroll
    for (int k = 0; k < kColsSlices; ++k) {
      S += msum[k][0][lane];
      N += msum[k][1][lane];
    }
    const double m = S / N;
    mean2 = m * m;
  }
  for (int l0 = 0; l0 < a.n_lags; l0 += LG) {
    int64_t L[LG];
    double sum[LG], n[LG];
#pragma unroll
    for (int l = 0; l < LG; ++l) {
      L[l] = l0 + l < a.n_lags ? a.lags[l0 + l] : 0;  // 0: not a lag of this group
      sum[l] = n[l] = 0.0;
    }
    if (valid)
      for (int64_t t = t0; t < t1; ++t) {
        const double xt = (double)x[t * st];
#pragma unroll
        for (int l = 0; l < LG; ++l) {
          if (L[l] >= 1 && t >= L[l] && t < P - L[l]) {  // the same for every lane
            const double d = (double)x[(t + L[l]) * st] - 2.0 * xt + (double)x[(t - L[l]) * st];
            if (isfinite(d)) {
              sum[l] += d * d;
              n[l] += 1.0;
            }
          }
        }
      }
#pragma unroll
    for (int l = 0; l < LG; ++l) {
      red[slice][l][0][lane] = sum[l];
      red[slice][l][1][lane] = n[l];
    }
    __syncthreads();
    if (slice == 0 && valid) {
#pragma unroll
      for (int l = 0; l < LG; ++l) {
        if (l0 + l >= a.n_lags) break;
        double S = 0.0, N = 0.0;
#pragma unroll
        for (int k = 0; k < kColsSlices; ++k) {
          S += red[k][l][0][lane];
          N += red[k][l][1][lane];
        }
        const double tau = (double)L[l] * a.spacing;
        a.out[s * a.n_lags + l0 + l] = N > 0.0 && L[l] >= 1 && 2 * L[l] < P ? S / N / (2.0 * tau * tau) / mean2 : NAN;
      }
    }
    __syncthreads();  // the next lag group reuses red
  }
}

// The same for side-by-side series whose lags are at most kWinMaxLag, through a window of the series held in
// LDS.  A workgroup owns 32 neighbouring series (128-byte rows of the [t][series] array) and walks t in steps
// of 64 rows; every row is read from memory once and then serves all its second differences from LDS.  The
// window is a ring of kWinRing rows (the rows t - 2 Lmax .. t + 63 of a step) whose first 64 slots are
// repeated after its end, so a run of 64 consecutive rows never wraps.  Thread (group g, phase q, half h)
// holds the four series 4g .. 4g+3 (16-byte LDS reads) and takes the point t = r0 - Lmax + q of every step
// r0 (the point whose t + Lmax has just arrived) for lags 4h .. 4h+3 of a group of up to eight.  A term is
// added without a finiteness test: a series with a non-finite sample ends with a non-finite sum, and only
// then is that (series, lag) summed again term by term, leaving out non-finite triples.  The 64 phases'
// sums are added in phase order.  Needs rows that are 8-byte aligned and a row stride of whole float pairs.
constexpr int kWinSeries = 32, kWinStep = 64, kWinGroups = kWinSeries / 4, kWinLags = 8, kWinAhead = 2;
constexpr int kWinHalfLags = kWinLags / 2;
constexpr int kWinRing = 2 * kWinMaxLag + 2 * kWinStep;
constexpr int kWinThreads = kWinGroups * kWinStep * 2;

__global__ void __launch_bounds__(kWinThreads) k_allan_window(AllanArgs a) {
  __shared__ __align__(16) float buf[(kWinRing + kWinStep) * kWinSeries];
  double* red = reinterpret_cast<double*>(buf);  // [lag][phase][series] phase sums, after a sweep
  __shared__ double meanv[kWinSeries];            // squared series means (normalisation)
  static_assert(kWinLags * kWinStep * kWinSeries * 8 <= (kWinRing + kWinStep) * kWinSeries * 4,
                "the phase sums fit in the ring");
  const int tid = (int)threadIdx.x;
  const int g = tid % kWinGroups, q = (tid / kWinGroups) % kWinStep;
  // the half is the same for a whole wave (512-thread halves): made visibly uniform, so the lag and ring-slot
  // arithmetic below runs on the scalar unit
  const int h = __builtin_amdgcn_readfirstlane(tid / (kWinGroups * kWinStep));
  const int64_t sb = (int64_t)blockIdx.x * kWinSeries;  // first series of the workgroup
  const int P = (int)a.n_points;                          // < 2^31 (checked by the launcher)
  const int64_t st = a.point_stride;
  // loads: row r0 + q, the two series 4g + 2h, 4g + 2h + 1 (a wave reads whole 128-byte rows).  The series
  // count is even, so a pair is wholly in or out; every load is issued (past the end: from row P - 1 or the
  // first pair, a valid address) and replaced by zeros, so no load sits behind a branch.
  const int ls = 4 * g + 2 * h;
  const bool pin = sb + ls < a.n_series;
  const float* xl = a.x + (pin ? sb + ls : 0);
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  // (the zeros are substituted when the pair enters the ring, so the load is not waited for until then)
  auto fetch = [&](f2& d, int r) { d = *reinterpret_cast<const f2*>(xl + (int64_t)(r < P ? r : P - 1) * st); };
  auto wrap = [](int k) { return k >= kWinRing ? k - kWinRing : k; };
  // ring slot X + q of this lane: a per-lane byte offset plus the wave-uniform X times the row bytes (one
  // vector add per read)
  const uint32_t lane_b = (uint32_t)(q * kWinSeries + 4 * g) * 4u;
  auto rdq = [&](int x) {
    const uint32_t off = lane_b + (uint32_t)__builtin_amdgcn_readfirstlane(x) * (kWinSeries * 4u);
    return *reinterpret_cast<const f4*>(reinterpret_cast<const char*>(buf) + off);
  };
  double xs[2] = {0, 0}, xn[2] = {0, 0};  // finite samples of the loaded series (normalisation), first sweep
  for (int l0 = 0; l0 < a.n_lags; l0 += kWinLags) {
    int L[kWinLags];
    int lmax = 1;
#pragma unroll
    for (int l = 0; l < kWinLags; ++l) {
      L[l] = l0 + l < a.n_lags ? a.lags[l0 + l] : 0;  // 0: not a lag of this group
      lmax = L[l] > lmax ? L[l] : lmax;
    }
    int Lh[kWinHalfLags];
#pragma unroll
    for (int l = 0; l < kWinHalfLags; ++l) Lh[l] = h ? L[kWinHalfLags + l] : L[l];
    double S[kWinHalfLags][4];
#pragma unroll
    for (int l = 0; l < kWinHalfLags; ++l)
#pragma unroll
      for (int c = 0; c < 4; ++c) S[l][c] = 0.0;
    f2 pre[kWinAhead];
    // issued in step order (the loop then finds the same order each time round: a step waits only for the
    // loads issued before its own)
#pragma unroll
    for (int u = 0; u < kWinAhead; ++u) {
      fetch(pre[u], u * kWinStep + q);
      __builtin_amdgcn_sched_barrier(0);
    }
    int k0 = 0;                // slot of row r0
    int bt = kWinRing - lmax;  // slot of row r0 - lmax (lmax <= kWinMaxLag < kWinRing)
    // the point t = r0 - lmax + q of step r0 counts for lag L when L <= t < P - L: every point of the step
    // counts for every lag of this half (the same for every lane) in a contiguous middle range of steps
    auto step_all = [&](const int r0) {
      bool all = true;
#pragma unroll
      for (int l = 0; l < kWinHalfLags; ++l)
        all = all && Lh[l] >= 1 && r0 - lmax >= Lh[l] && r0 - lmax + kWinStep - 1 < P - Lh[l];
      return all;
    };
    auto step = [&](const int r0, f2& d, auto masked) {
      __syncthreads();  // every thread is done with the previous step's rows
      {
        if (!(pin && r0 + q < P)) d = f2{0.f, 0.f};
        const int k = wrap(k0 + q);
        *reinterpret_cast<f2*>(&buf[k * kWinSeries + ls]) = d;
        if (k < kWinStep) *reinterpret_cast<f2*>(&buf[(k + kWinRing) * kWinSeries + ls]) = d;
        if (l0 == 0 && a.normalize && r0 + q < P) {
          if (isfinite(d.x)) {
            xs[0] += (double)d.x;
            xn[0] += 1.0;
          }
          if (isfinite(d.y)) {
            xs[1] += (double)d.y;
            xn[1] += 1.0;
          }
        }
      }
      fetch(d, r0 + kWinAhead * kWinStep + q);
      __syncthreads();
      const int t = r0 - lmax + q;
      const f4 b = rdq(bt);
      const double xb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int l = 0; l < kWinHalfLags; ++l) {
        const f4 ua = rdq(wrap(bt + Lh[l]));
        const f4 dc = rdq(bt >= Lh[l] ? bt - Lh[l] : bt - Lh[l] + kWinRing);
        const double xa[4] = {ua.x, ua.y, ua.z, ua.w}, xc[4] = {dc.x, dc.y, dc.z, dc.w};
        const bool use = !decltype(masked)::value || (Lh[l] >= 1 && t >= Lh[l] && t < P - Lh[l]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double dd = xa[c] - 2.0 * xb[c] + xc[c];
          const double e = use ? dd : 0.0;  // an exact zero term outside the lag's range
          S[l][c] = fma(e, e, S[l][c]);
        }
      }
      k0 = wrap(k0 + kWinStep);
      bt = wrap(bt + kWinStep);
    };
    // Every step of an unrolled group runs: a step past the last point writes zero rows and adds exact
    // zeros (its points are out of every lag's range), and no load then sits behind a branch, so each step
    // waits only for its own rows while the later steps' loads stay in flight.
    // Three loops over the step groups: those before the middle range, the middle range (no range test), and
    // those after it; each loop then has one definition of the sums (a test inside one loop had the compiler
    // copy all sixteen FP64 sums on every step).
    constexpr int GS = kWinAhead * kWinStep;  // rows per step group
    auto group_all = [&](const int r0) {
      bool all = true;
#pragma unroll
      for (int u = 0; u < kWinAhead; ++u) all = all && step_all(r0 + u * kWinStep);
      return all;
    };
    int r0 = 0;
    for (; r0 < P + lmax && !group_all(r0); r0 += GS) {
#pragma unroll
      for (int u = 0; u < kWinAhead; ++u) step(r0 + u * kWinStep, pre[u], std::true_type{});
    }
    for (; r0 < P + lmax && group_all(r0); r0 += GS) {
#pragma unroll
      for (int u = 0; u < kWinAhead; ++u) step(r0 + u * kWinStep, pre[u], std::false_type{});
    }
    for (; r0 < P + lmax; r0 += GS) {
#pragma unroll
      for (int u = 0; u < kWinAhead; ++u) step(r0 + u * kWinStep, pre[u], std::true_type{});
    }
    __syncthreads();  // the ring is free: it holds the phase sums from here on
    if (l0 == 0 && a.normalize) {  // series means: [2][phase][series] sums, added in phase order
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        red[q * kWinSeries + ls + c] = xs[c];
        red[(kWinStep + q) * kWinSeries + ls + c] = xn[c];
      }
      __syncthreads();
      if (tid < kWinSeries) {
        double sx = 0.0, sn = 0.0;
        for (int p = 0; p < kWinStep; ++p) {
          sx += red[p * kWinSeries + tid];
          sn += red[(kWinStep + p) * kWinSeries + tid];
        }
        meanv[tid] = (sx / sn) * (sx / sn);
      }
      __syncthreads();
    }
#pragma unroll
    for (int l = 0; l < kWinHalfLags; ++l)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[((h * kWinHalfLags + l) * kWinStep + q) * kWinSeries + 4 * g + c] = S[l][c];
    __syncthreads();
    // writers: one thread per (series, lag) of the group
    if (tid < kWinSeries * kWinLags) {
      const int c = tid % kWinSeries, l = tid / kWinSeries;
      const int64_t sr = sb + c;
      if (sr < a.n_series && l0 + l < a.n_lags) {
        const double mean2 = a.normalize ? meanv[c] : 1.0;
        double sum = 0.0;
        for (int p = 0; p < kWinStep; ++p) sum += red[(l * kWinStep + p) * kWinSeries + c];
        const int64_t Ll = L[l];
        double n = (double)(P - 2 * Ll > 0 ? P - 2 * Ll : 0);  // every term counts (finite sum)
        if (!isfinite(sum)) {
          // a non-finite sample in the series: the terms again, in t order, without the non-finite ones
          const float* xc = a.x + sr;
          sum = 0.0;
          n = 0.0;
          for (int64_t t = Ll; t < P - Ll; ++t) {
            const double dd = (double)xc[(t + Ll) * st] - 2.0 * (double)xc[t * st] + (double)xc[(t - Ll) * st];
            if (isfinite(dd)) {
              sum += dd * dd;
              n += 1.0;
            }
          }
        }
        const double tau = (double)Ll * a.spacing;
        a.out[sr * a.n_lags + l0 + l] = n > 0.0 && Ll >= 1 && 2 * Ll < P ? sum / n / (2.0 * tau * tau) / mean2 : NAN;
      }
    }
    __syncthreads();  // the next lag group refills the ring
  }
}

}  // namespace

hipError_t launch_channel_average(const ChanAvgArgs& a, hipStream_t s) {
  const int64_t n_bins = a.n_chan / a.factor;
  if (a.factor <= kSpan) {
    const int nb = kSpan / a.factor;
    const dim3 grid((unsigned)((n_bins + nb - 1) / nb), (unsigned)a.n_spec);
    hipLaunchKernelGGL(k_chan_avg_span, grid, dim3(kNT), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_chan_avg_wide, dim3((unsigned)n_bins, (unsigned)a.n_spec), dim3(kNT), 0, s, a);
  }
  return hipGetLastError();
}

// ---- scratch of the allocation-free bandpass fit: a file-scope device array, one copy per GPU, found once
// per device with hipGetSymbolAddress (host code may use only that address, never the array's name)
static __device__ __align__(256) unsigned char scratch[kBandpassScratchBytes];

hipError_t bandpass_scratch(hipStream_t stream, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int cur = -1;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_bandpass_fit(const SplineArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_spline_gram, dim3((unsigned)a.n_int), dim3(kNT), 0, s, a);
  hipLaunchKernelGGL(k_spline_solve, dim3(1), dim3(kNT), 0, s, a);
  hipLaunchKernelGGL(k_spline_eval, dim3((unsigned)((a.n_chan + kNT - 1) / kNT)), dim3(kNT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bandpass_correct(const float* hk, int64_t n_spec, int64_t n_chan, const float* smooth,
                                   const double* gain, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bandpass_correct, dim3((unsigned)((n_chan + kNT - 1) / kNT), (unsigned)n_spec), dim3(kNT), 0,
                     s, hk, n_chan, smooth, gain, out);
  return hipGetLastError();
}

hipError_t launch_band_stats(const float* x, int64_t n_spec, int64_t n_chan, double* mean_sd, hipStream_t s) {
  hipLaunchKernelGGL(k_band_stats, dim3((unsigned)n_spec), dim3(kNT), 0, s, x, n_chan, mean_sd);
  return hipGetLastError();
}

static bool allan_cols(int64_t n_series, int64_t point_stride, int64_t series_stride) {
  return series_stride == 1 && point_stride >= n_series && n_series >= 64;
}

int64_t allan_part_doubles(int64_t n_points, int64_t n_series, int64_t point_stride, int64_t series_stride,
                           int n_lags) {
  if (allan_cols(n_series, point_stride, series_stride)) return 0;
  const int64_t chunks = n_points > 0 ? (n_points + kAllanChunk - 1) / kAllanChunk : 1;
  return n_series * chunks * (n_lags + 1) * 2;
}

hipError_t launch_allan(const AllanArgs& a, hipStream_t s) {
  int lmax = 0;
  for (int l = 0; l < a.n_lags; ++l) lmax = a.lags[l] > lmax ? a.lags[l] : lmax;
  const bool rows16 = reinterpret_cast<uintptr_t>(a.x) % 8 == 0 && a.point_stride % 2 == 0 && a.n_series % 2 == 0;
  if (allan_cols(a.n_series, a.point_stride, a.series_stride) && lmax <= kWinMaxLag && rows16 &&
      a.n_points >= 1 && a.n_points < (int64_t(1) << 31)) {  // (no rows: the column form writes NaN)
    hipLaunchKernelGGL(k_allan_window, dim3((unsigned)((a.n_series + kWinSeries - 1) / kWinSeries)),
                       dim3(kWinThreads), 0, s, a);
  } else if (allan_cols(a.n_series, a.point_stride, a.series_stride)) {
    hipLaunchKernelGGL(k_allan_cols, dim3((unsigned)((a.n_series + kColsSeries - 1) / kColsSeries)),
                       dim3(kColsSeries * kColsSlices), 0, s, a);
  } else {
    const int64_t chunks = a.n_points > 0 ? (a.n_points + kAllanChunk - 1) / kAllanChunk : 1;
    hipLaunchKernelGGL(k_allan_part, dim3((unsigned)a.n_series, (unsigned)chunks), dim3(kNT), 0, s, a, chunks);
    hipLaunchKernelGGL(k_allan_total, dim3((unsigned)((a.n_series + kNT - 1) / kNT)), dim3(kNT), 0, s, a, chunks);
  }
  return hipGetLastError();
}

}  // namespace ps
