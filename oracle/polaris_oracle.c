/*
 * polaris_oracle.c -- plain, slow FP64 reference of the PolariS spectrometer path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load this file; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * What it computes (Mizuno et al., "Software Polarization Spectrometer PolariS", arXiv 1412.1256):
 *   - Sec. 2 and the Fig. 2 caption: the processor translates 4- or 8-bit integer samples to floats,
 *     segments the streams, Fourier transforms each segment, multiplies the spectra into auto- and
 *     cross-power products (Table 1: <XX*>, <YY*>, <XY*>) and accumulates them over the integration;
 *   - Sec. 2 (statement of the spectrometer's four functions): accept two orthogonal polarizations,
 *     FFT, multiply spectra into power and cross-power spectra, integrate;
 *   - Sec. 3.1: the segment window is rectangular (apodisation is an offline option);
 *   - Sec. 2.1, Eq. 2: full Stokes I, Q, U, V from the four correlation products divided by the
 *     voltage-domain gain products, rotated by twice the parallactic angle.
 *
 * Readings where the paper is silent (each one is listed with its reason in the design notes):
 *   - codes: b-bit offset-binary codes map to the odd levels 2c - (2^b - 1) for b = 2, 4; b = 8 is
 *     two's-complement int8; b = 32 is IEEE float32.  Item t*S + s of a time-major, stream-interleaved
 *     buffer sits at bit offset (t*S + s)*b, least significant bits first;
 *   - channels: frame length N gives channels k = 0 .. N/2 - 1 (DC kept, Nyquist dropped);
 *   - transform: X[k] = sum_n w[n] x[n] exp(-2 pi i n k / N), unnormalised; cross product X * conj(Y);
 *   - normalised products M = A / (F * sum w^2);
 *   - leakage (Sec. 2.1 defers its model): observed voltages v' = G J v with G = diag(g_x, g_y) and
 *     J = [[1, d_x], [d_y, 1]], so the calibrated coherency is C = (G J)^-1 M (G J)^-H; with d = 0 this is
 *     exactly Eq. 2's division by G_X G_X*, G_X G_Y*, G_Y G_X*, G_Y G_Y*;
 *   - learnable window: 64 control points theta_j at u = n (n_taps - 1)/(N - 1), linear in between.
 *
 * Arithmetic: FP64 everywhere, compiled with -ffp-contract=off.  The FFT is an iterative radix-2
 * decimation-in-time transform whose twiddles are cos/sin(2 pi j / N) evaluated directly (no recurrence);
 * a brute-force DFT with exactly reduced angles is provided for small N.  Frames are summed in fixed
 * blocks of 8 consecutive frames, blocks in order, so the result does not depend on the thread count.
 */
#include "polaris_oracle.h"

#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define OR_FRAME_BLOCK 8
static const double OR_TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------------------------------ */
/* unpack: one item of the packed buffer -> its level                                                */
/* ------------------------------------------------------------------------------------------------ */

static double or_level(const uint8_t* packed, int bits, int n_streams, int64_t t, int s) {
  int64_t item = t * (int64_t)n_streams + s;
  if (bits == 32) {
    float v;
    memcpy(&v, packed + 4 * item, sizeof v);
    return (double)v;
  }
  if (bits == 8) return (double)(int8_t)packed[item];
  int64_t bit = item * bits;
  unsigned byte = packed[bit >> 3];
  unsigned code = (byte >> (bit & 7)) & ((1u << bits) - 1u);
  return 2.0 * (double)code - (double)((1 << bits) - 1);
}

static int or_bits_ok(int bits) { return bits == 2 || bits == 4 || bits == 8 || bits == 32; }

int or_unpack(const uint8_t* packed, int bits, int n_streams, int64_t n_time, double* out) {
  if (!packed || !out || !or_bits_ok(bits) || n_streams <= 0 || n_time < 0) return OR_ERR_ARG;
  for (int s = 0; s < n_streams; ++s)
    for (int64_t t = 0; t < n_time; ++t) out[(int64_t)s * n_time + t] = or_level(packed, bits, n_streams, t, s);
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* window                                                                                            */
/* ------------------------------------------------------------------------------------------------ */

int or_window(int kind, int64_t n, const double* taps, int n_taps, double* w, double* sumsq) {
  if (!w || n <= 1) return OR_ERR_ARG;
  for (int64_t i = 0; i < n; ++i) {
    double v;
    if (kind == OR_WIN_RECT) {
      v = 1.0;
    } else if (kind == OR_WIN_HANN) { /* periodic (DFT-even) Hann */
      v = 0.5 - 0.5 * cos(OR_TWO_PI * (double)i / (double)n);
    } else if (kind == OR_WIN_HAMMING) { /* periodic Hamming, coefficients 0.54 and 0.46 */
      v = 0.54 - 0.46 * cos(OR_TWO_PI * (double)i / (double)n);
    } else if (kind == OR_WIN_BLACKMAN) { /* periodic Blackman, coefficients 0.42, 0.5 and 0.08 */
      v = 0.42 - 0.5 * cos(OR_TWO_PI * (double)i / (double)n) + 0.08 * cos(2.0 * OR_TWO_PI * (double)i / (double)n);
    } else if (kind == OR_WIN_TAPS) {
      if (!taps || n_taps < 2) return OR_ERR_ARG;
      double u = (double)i * (double)(n_taps - 1) / (double)(n - 1);
      int j = (int)floor(u);
      if (j > n_taps - 2) j = n_taps - 2;
      double t = u - (double)j;
      v = (1.0 - t) * taps[j] + t * taps[j + 1];
    } else {
      return OR_ERR_ARG;
    }
    w[i] = v;
  }
  if (sumsq) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += w[i] * w[i];
    *sumsq = s;
  }
  return OR_OK;
}

/* d w[n] / d theta_j of the piecewise-linear window, folded against a gradient on w */
static void or_taps_adjoint(int64_t n, int n_taps, const double* d_w, double* d_taps) {
  for (int j = 0; j < n_taps; ++j) d_taps[j] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double u = (double)i * (double)(n_taps - 1) / (double)(n - 1);
    int j = (int)floor(u);
    if (j > n_taps - 2) j = n_taps - 2;
    double t = u - (double)j;
    d_taps[j] += (1.0 - t) * d_w[i];
    d_taps[j + 1] += t * d_w[i];
  }
}

/* ------------------------------------------------------------------------------------------------ */
/* transforms                                                                                        */
/* ------------------------------------------------------------------------------------------------ */

static int or_is_pow2(int64_t n) { return n >= 2 && (n & (n - 1)) == 0; }

/* cos/sin(2 pi j / n) for j < n/2, each evaluated directly */
static void or_twiddles(int64_t n, double* c, double* s) {
  for (int64_t j = 0; j < n / 2; ++j) {
    double a = OR_TWO_PI * (double)j / (double)n;
    c[j] = cos(a);
    s[j] = sin(a);
  }
}

/* in-place forward radix-2 DIT FFT: bit-reversal permutation, then log2(n) butterfly stages */
static void or_fft_core(double* re, double* im, int64_t n, const double* c, const double* s) {
  for (int64_t i = 1, j = 0; i < n; ++i) {
    int64_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double tr = re[i], ti = im[i];
      re[i] = re[j]; im[i] = im[j];
      re[j] = tr; im[j] = ti;
    }
  }
  for (int64_t len = 2; len <= n; len <<= 1) {
    int64_t half = len >> 1, step = n / len;
    for (int64_t i0 = 0; i0 < n; i0 += len) {
      for (int64_t k = 0; k < half; ++k) {
        double wr = c[k * step], wi = -s[k * step]; /* exp(-2 pi i k / len) */
        int64_t a = i0 + k, b = a + half;
        double vr = re[b] * wr - im[b] * wi;
        double vi = re[b] * wi + im[b] * wr;
        double ur = re[a], ui = im[a];
        re[a] = ur + vr; im[a] = ui + vi;
        re[b] = ur - vr; im[b] = ui - vi;
      }
    }
  }
}

int or_fft(double* re, double* im, int64_t n) {
  if (!re || !im || !or_is_pow2(n)) return OR_ERR_ARG;
  double* c = malloc(sizeof(double) * (size_t)(n / 2));
  double* s = malloc(sizeof(double) * (size_t)(n / 2));
  if (!c || !s) { free(c); free(s); return OR_ERR_MEM; }
  or_twiddles(n, c, s);
  or_fft_core(re, im, n, c, s);
  free(c); free(s);
  return OR_OK;
}

int or_dft(const double* re, const double* im, int64_t n, double* out_re, double* out_im) {
  if (!re || !im || !out_re || !out_im || n <= 0) return OR_ERR_ARG;
  for (int64_t k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double a = OR_TWO_PI * (double)((j * k) % n) / (double)n;
      double cr = cos(a), ci = -sin(a);
      sr += re[j] * cr - im[j] * ci;
      si += re[j] * ci + im[j] * cr;
    }
    out_re[k] = sr;
    out_im[k] = si;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* thread helpers: fixed frame blocks, committed to the shared sum in block order                    */
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
  pthread_mutex_t mu;
  pthread_cond_t cv;
  int64_t next_block;   /* next block to hand out */
  int64_t next_commit;  /* next block allowed to add into the shared sum */
} or_sched;

static void or_sched_init(or_sched* q) {
  pthread_mutex_init(&q->mu, NULL);
  pthread_cond_init(&q->cv, NULL);
  q->next_block = 0;
  q->next_commit = 0;
}

static void or_sched_free(or_sched* q) {
  pthread_mutex_destroy(&q->mu);
  pthread_cond_destroy(&q->cv);
}

static int64_t or_take(or_sched* q) {
  pthread_mutex_lock(&q->mu);
  int64_t b = q->next_block++;
  pthread_mutex_unlock(&q->mu);
  return b;
}

static void or_commit_begin(or_sched* q, int64_t b) {
  pthread_mutex_lock(&q->mu);
  while (q->next_commit != b) pthread_cond_wait(&q->cv, &q->mu);
}

static void or_commit_end(or_sched* q) {
  q->next_commit++;
  pthread_cond_broadcast(&q->cv);
  pthread_mutex_unlock(&q->mu);
}

static int or_thread_count(int nthreads, int64_t n_blocks) {
  int n = nthreads;
  if (n <= 0) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    n = c > 0 ? (int)c : 1;
  }
  if (n > n_blocks) n = (int)n_blocks;
  if (n < 1) n = 1;
  return n;
}

/* the windowed frame f (samples f*hop .. f*hop + N - 1) of stream s as a complex sequence (x_w, 0),
 * transformed in place */
static void or_frame_spectrum(const uint8_t* packed, int bits, int S, int64_t N, int64_t hop, int64_t f, int s,
                              const double* w, const double* c, const double* sn, double* re, double* im) {
  for (int64_t n = 0; n < N; ++n) {
    re[n] = w[n] * or_level(packed, bits, S, f * hop + n, s);
    im[n] = 0.0;
  }
  or_fft_core(re, im, N, c, sn);
}

/* ------------------------------------------------------------------------------------------------ */
/* accumulation of auto- and cross-power spectra                                                     */
/* ------------------------------------------------------------------------------------------------ */

typedef struct {
  const uint8_t* packed;
  int bits, S, P;
  const int *px, *py;
  int64_t N, C, F, hop;
  const double* w;
  const double *c, *s;
  double* acc; /* [P][4][C] */
  or_sched* q;
  int err;
} or_acc_job;

static void* or_acc_worker(void* arg) {
  or_acc_job* J = (or_acc_job*)arg;
  int64_t N = J->N, C = J->C;
  double* re = malloc(sizeof(double) * (size_t)(N * J->S));
  double* im = malloc(sizeof(double) * (size_t)(N * J->S));
  double* part = malloc(sizeof(double) * (size_t)(4 * C * J->P));
  if (!re || !im || !part) { J->err = OR_ERR_MEM; free(re); free(im); free(part); return NULL; }
  int64_t n_blocks = (J->F + OR_FRAME_BLOCK - 1) / OR_FRAME_BLOCK;
  for (;;) {
    int64_t b = or_take(J->q);
    if (b >= n_blocks) break;
    memset(part, 0, sizeof(double) * (size_t)(4 * C * J->P));
    int64_t f_end = (b + 1) * OR_FRAME_BLOCK < J->F ? (b + 1) * OR_FRAME_BLOCK : J->F;
    for (int64_t f = b * OR_FRAME_BLOCK; f < f_end; ++f) {
      for (int s = 0; s < J->S; ++s)
        or_frame_spectrum(J->packed, J->bits, J->S, N, J->hop, f, s, J->w, J->c, J->s, re + s * N, im + s * N);
      for (int p = 0; p < J->P; ++p) {
        const double *xr = re + J->px[p] * N, *xi = im + J->px[p] * N;
        const double *yr = re + J->py[p] * N, *yi = im + J->py[p] * N;
        double* a = part + (int64_t)p * 4 * C;
        for (int64_t k = 0; k < C; ++k) {
          a[k] += xr[k] * xr[k] + xi[k] * xi[k];             /* X X* */
          a[C + k] += yr[k] * yr[k] + yi[k] * yi[k];         /* Y Y* */
          a[2 * C + k] += xr[k] * yr[k] + xi[k] * yi[k];     /* Re X Y* */
          a[3 * C + k] += xi[k] * yr[k] - xr[k] * yi[k];     /* Im X Y* */
        }
      }
    }
    or_commit_begin(J->q, b);
    for (int64_t i = 0; i < 4 * C * J->P; ++i) J->acc[i] += part[i];
    or_commit_end(J->q);
  }
  free(re); free(im); free(part);
  return NULL;
}

static int or_check_pairs(int S, int P, const int* px, const int* py) {
  if (P <= 0 || !px || !py) return 0;
  for (int p = 0; p < P; ++p)
    if (px[p] < 0 || px[p] >= S || py[p] < 0 || py[p] >= S) return 0;
  return 1;
}

/* Segmentation (Sec. 3.1): frame f covers samples f*hop .. f*hop + N - 1; every whole frame of the buffer
 * is taken.  hop = N (contiguous frames) or N / 2^j (overlap of 1 - 2^-j; the paper mentions 50 %). */
static int or_hop_ok(int64_t fft_len, int64_t hop) {
  return hop > 0 && hop <= fft_len && fft_len % hop == 0 && or_is_pow2(hop);
}

static int64_t or_frame_count(int64_t n_time, int64_t fft_len, int64_t hop) {
  return n_time < fft_len ? 0 : (n_time - fft_len) / hop + 1;
}

int or_accumulate(const uint8_t* packed, int bits, int n_streams, int64_t n_time, int64_t fft_len, int64_t hop,
                  const double* w, int n_pairs, const int* pair_x, const int* pair_y, int nthreads,
                  double* acc, int64_t* n_frames) {
  if (hop == 0) hop = fft_len;
  if (!packed || !w || !acc || !or_bits_ok(bits) || !or_is_pow2(fft_len) || n_time < 0 ||
      !or_check_pairs(n_streams, n_pairs, pair_x, pair_y) || n_time % fft_len || !or_hop_ok(fft_len, hop))
    return OR_ERR_ARG;
  int64_t N = fft_len, C = N / 2, F = or_frame_count(n_time, N, hop);
  memset(acc, 0, sizeof(double) * (size_t)(4 * C * n_pairs));
  if (n_frames) *n_frames = F;
  if (F == 0) return OR_OK;
  double* c = malloc(sizeof(double) * (size_t)(N / 2));
  double* s = malloc(sizeof(double) * (size_t)(N / 2));
  if (!c || !s) { free(c); free(s); return OR_ERR_MEM; }
  or_twiddles(N, c, s);
  or_sched q;
  or_sched_init(&q);
  int64_t n_blocks = (F + OR_FRAME_BLOCK - 1) / OR_FRAME_BLOCK;
  int nt = or_thread_count(nthreads, n_blocks);
  or_acc_job job = {packed, bits, n_streams, n_pairs, pair_x, pair_y, N, C, F, hop, w, c, s, acc, &q, OR_OK};
  pthread_t* th = malloc(sizeof(pthread_t) * (size_t)nt);
  for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, or_acc_worker, &job);
  for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  free(th);
  or_sched_free(&q);
  free(c); free(s);
  return job.err;
}

/* ------------------------------------------------------------------------------------------------ */
/* calibration and Stokes (Eq. 2)                                                                    */
/* ------------------------------------------------------------------------------------------------ */

typedef double complex cplx;
typedef struct { cplx m[2][2]; } mat2;

static mat2 m2_mul(mat2 a, mat2 b) {
  mat2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j];
  return r;
}

static mat2 m2_adj(mat2 a) { /* conjugate transpose */
  mat2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = conj(a.m[j][i]);
  return r;
}

static mat2 m2_add(mat2 a, mat2 b) {
  mat2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = a.m[i][j] + b.m[i][j];
  return r;
}

static mat2 m2_scale(mat2 a, cplx s) {
  mat2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.m[i][j] = a.m[i][j] * s;
  return r;
}

static mat2 m2_inv(mat2 a) {
  cplx det = a.m[0][0] * a.m[1][1] - a.m[0][1] * a.m[1][0];
  mat2 r;
  r.m[0][0] = a.m[1][1] / det;
  r.m[0][1] = -a.m[0][1] / det;
  r.m[1][0] = -a.m[1][0] / det;
  r.m[1][1] = a.m[0][0] / det;
  return r;
}

/* Circular feeds (no formula in the paper; reading): R = (X + iY)/sqrt 2, L = (X - iY)/sqrt 2 give
 * C_rr = I + V, C_ll = I - V, C_rl = (Q + iU) at psi = 0, and the parallactic angle rotates Q + iU by
 * exp(2 i psi) as Eq. 2 does for linear feeds.  Rows act on [C_rr, C_rl, C_lr, C_ll], factor 1/2 included. */
static void or_circular_matrix(double psi, cplx m[4][4]) {
  cplx e = cexp(2.0 * I * psi), ec = conj(e);
  cplx row[4][4] = {{1.0, 0.0, 0.0, 1.0},
                    {0.0, e, ec, 0.0},
                    {0.0, -I * e, I * ec, 0.0},
                    {1.0, 0.0, 0.0, -1.0}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = 0.5 * row[i][j];
}

/* the 4x4 Stokes matrix of Eq. 2, including its factor 1/2, acting on [C_xx, C_xy, C_yx, C_yy] */
static void or_eq2_matrix(double psi, cplx m[4][4]) {
  double c2 = cos(2.0 * psi), s2 = sin(2.0 * psi);
  cplx row[4][4] = {{1.0, 0.0, 0.0, 1.0},
                    {c2, -s2, -s2, -c2},
                    {s2, c2, c2, -s2},
                    {0.0, -I, I, 0.0}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = 0.5 * row[i][j];
}

typedef struct {
  mat2 G, J, E, Fi; /* gains, leakage, E = G J, Fi = E^-1 */
} or_cal_ch;

static or_cal_ch or_cal_channel(const double* gain_x, const double* gain_y, const double* dterms, int64_t k) {
  or_cal_ch c;
  cplx gx = gain_x ? gain_x[2 * k] + I * gain_x[2 * k + 1] : 1.0;
  cplx gy = gain_y ? gain_y[2 * k] + I * gain_y[2 * k + 1] : 1.0;
  cplx dx = dterms ? dterms[0] + I * dterms[1] : 0.0;
  cplx dy = dterms ? dterms[2] + I * dterms[3] : 0.0;
  c.G = (mat2){{{gx, 0.0}, {0.0, gy}}};
  c.J = (mat2){{{1.0, dx}, {dy, 1.0}}};
  c.E = m2_mul(c.G, c.J);
  c.Fi = m2_inv(c.E);
  return c;
}

static mat2 or_normalised(const double* a, int64_t C, int64_t k, double scale) {
  cplx xy = a[2 * C + k] + I * a[3 * C + k];
  mat2 M = {{{a[k] * scale, xy * scale}, {conj(xy) * scale, a[C + k] * scale}}};
  return M;
}

int or_stokes(const double* acc, int n_pairs, int64_t n_chan, int64_t n_frames, double sumw2,
              const double* gain_x, const double* gain_y, const double* dterms, double psi, int feed,
              double* iquv) {
  if (!acc || !iquv || n_pairs <= 0 || n_chan <= 0 || n_frames <= 0 || !(sumw2 > 0.0)) return OR_ERR_ARG;
  if (feed != OR_FEED_LINEAR && feed != OR_FEED_CIRCULAR) return OR_ERR_ARG;
  int64_t C = n_chan;
  double scale = 1.0 / ((double)n_frames * sumw2);
  cplx m[4][4];
  if (feed == OR_FEED_CIRCULAR)
    or_circular_matrix(psi, m);
  else
    or_eq2_matrix(psi, m);
  for (int p = 0; p < n_pairs; ++p) {
    const double* a = acc + (int64_t)p * 4 * C;
    for (int64_t k = 0; k < C; ++k) {
      or_cal_ch cal = or_cal_channel(gain_x ? gain_x + (int64_t)p * 2 * C : NULL,
                                     gain_y ? gain_y + (int64_t)p * 2 * C : NULL,
                                     dterms ? dterms + 4 * p : NULL, k);
      mat2 M = or_normalised(a, C, k, scale);
      mat2 Cm = m2_mul(m2_mul(cal.Fi, M), m2_adj(cal.Fi));
      cplx v[4] = {Cm.m[0][0], Cm.m[0][1], Cm.m[1][0], Cm.m[1][1]};
      for (int i = 0; i < 4; ++i) {
        cplx acc_i = 0.0;
        for (int j = 0; j < 4; ++j) acc_i += m[i][j] * v[j];
        iquv[((int64_t)p * 4 + i) * C + k] = creal(acc_i);
      }
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------------ */
/* gradient of a loss on the Stokes spectra (the differentiation form)                               */
/* ------------------------------------------------------------------------------------------------ */

/*
 * Notation: for a complex quantity Z, Gb(Z) = dL/dRe Z + i dL/dIm Z, so that dL = Re sum conj(Gb(Z)) dZ.
 *   Eq. 2 adjoint: Gb(C_ij) = sum_P g_P conj(m_P,ij).
 *   C = Fi M Fi^H         ->  Gb(M) = Fi^H Gb(C) Fi,   Gb(Fi) = (Gb(C) + Gb(C)^H) Fi M
 *   Fi = E^-1             ->  Gb(E) = -Fi^H Gb(Fi) Fi^H
 *   E = G J               ->  Gb(G) = diag(Gb(E) J^H),  Gb(J) = G^H Gb(E)  (d_x at (0,1), d_y at (1,0))
 *   M = A / (F s), s = sum w^2  ->  Gb(A) = Gb(M) / (F s),  dL/dw[n] gets -2 w[n] Re tr(Gb(M)^H M) / s
 *   A = sum_f v v^H, v = [X; Y]  ->  Gb(v) = (Gb(A) + Gb(A)^H) v
 *   X[k] = sum_n w[n] x[n] e^{-2 pi i n k/N}  ->  dL/dw[n] += x[n] Re sum_{k<C} Gb(X[k]) e^{+2 pi i n k/N}
 */
typedef struct {
  const uint8_t* packed;
  int bits, S, P;
  const int *px, *py;
  int64_t N, C, F, hop;
  const double* w;
  const double *c, *s;
  const cplx* gA; /* [P][C][4]: Gb(A) entries 00, 01, 10, 11 */
  double* d_w;    /* [N] shared sum */
  or_sched* q;
  int err;
} or_grad_job;

static void* or_grad_worker(void* arg) {
  or_grad_job* J = (or_grad_job*)arg;
  int64_t N = J->N, C = J->C;
  double* re = malloc(sizeof(double) * (size_t)(N * J->S));
  double* im = malloc(sizeof(double) * (size_t)(N * J->S));
  double* hr = malloc(sizeof(double) * (size_t)N);
  double* hi = malloc(sizeof(double) * (size_t)N);
  double* part = malloc(sizeof(double) * (size_t)N);
  if (!re || !im || !hr || !hi || !part) {
    J->err = OR_ERR_MEM;
    free(re); free(im); free(hr); free(hi); free(part);
    return NULL;
  }
  int64_t n_blocks = (J->F + OR_FRAME_BLOCK - 1) / OR_FRAME_BLOCK;
  for (;;) {
    int64_t b = or_take(J->q);
    if (b >= n_blocks) break;
    memset(part, 0, sizeof(double) * (size_t)N);
    int64_t f_end = (b + 1) * OR_FRAME_BLOCK < J->F ? (b + 1) * OR_FRAME_BLOCK : J->F;
    for (int64_t f = b * OR_FRAME_BLOCK; f < f_end; ++f) {
      for (int s = 0; s < J->S; ++s)
        or_frame_spectrum(J->packed, J->bits, J->S, N, J->hop, f, s, J->w, J->c, J->s, re + s * N, im + s * N);
      for (int p = 0; p < J->P; ++p) {
        int sx = J->px[p], sy = J->py[p];
        for (int which = 0; which < 2; ++which) {
          /* Gb(X[k]) (which = 0) or Gb(Y[k]) (which = 1), as conj so one forward transform gives the sum */
          for (int64_t k = 0; k < N; ++k) { hr[k] = 0.0; hi[k] = 0.0; }
          for (int64_t k = 0; k < C; ++k) {
            const cplx* g = J->gA + ((int64_t)p * C + k) * 4;
            mat2 GA = {{{g[0], g[1]}, {g[2], g[3]}}};
            mat2 S2 = m2_add(GA, m2_adj(GA));
            cplx X = re[sx * N + k] + I * im[sx * N + k];
            cplx Y = re[sy * N + k] + I * im[sy * N + k];
            cplx gv = S2.m[which][0] * X + S2.m[which][1] * Y;
            hr[k] = creal(gv);
            hi[k] = -cimag(gv);
          }
          /* Re sum_k Gb_k e^{+i theta} = Re sum_k conj(Gb_k) e^{-i theta} */
          or_fft_core(hr, hi, N, J->c, J->s);
          int src = which == 0 ? sx : sy;
          for (int64_t n = 0; n < N; ++n) part[n] += or_level(J->packed, J->bits, J->S, f * J->hop + n, src) * hr[n];
        }
      }
    }
    or_commit_begin(J->q, b);
    for (int64_t n = 0; n < N; ++n) J->d_w[n] += part[n];
    or_commit_end(J->q);
  }
  free(re); free(im); free(hr); free(hi); free(part);
  return NULL;
}

int or_calibrate_backward(const uint8_t* packed, int bits, int n_streams, int64_t n_time, int64_t fft_len,
                          int64_t hop, const double* w, const double* taps, int n_taps, int n_pairs, const int* pair_x,
                          const int* pair_y, const double* acc, int64_t n_frames, double sumw2,
                          const double* gain_x, const double* gain_y, const double* dterms, double psi,
                          const double* g_iquv, int nthreads, double* d_gain_x, double* d_gain_y,
                          double* d_dterms, double* d_w, double* d_taps) {
  if (hop == 0) hop = fft_len;
  if (!packed || !w || !acc || !g_iquv || !or_bits_ok(bits) || !or_is_pow2(fft_len) ||
      !or_check_pairs(n_streams, n_pairs, pair_x, pair_y) || n_time % fft_len || n_frames <= 0 ||
      !or_hop_ok(fft_len, hop) || or_frame_count(n_time, fft_len, hop) != n_frames || !(sumw2 > 0.0))
    return OR_ERR_ARG;
  int64_t N = fft_len, C = N / 2, F = n_frames;
  double fs = (double)F * sumw2;
  cplx m[4][4];
  or_eq2_matrix(psi, m);
  cplx* gA = malloc(sizeof(cplx) * (size_t)(n_pairs * C * 4));
  double* dw = malloc(sizeof(double) * (size_t)N);
  if (!gA || !dw) { free(gA); free(dw); return OR_ERR_MEM; }
  memset(dw, 0, sizeof(double) * (size_t)N);
  double norm_term = 0.0;
  for (int p = 0; p < n_pairs; ++p) {
    const double* a = acc + (int64_t)p * 4 * C;
    cplx gdx = 0.0, gdy = 0.0;
    for (int64_t k = 0; k < C; ++k) {
      or_cal_ch cal = or_cal_channel(gain_x ? gain_x + (int64_t)p * 2 * C : NULL,
                                     gain_y ? gain_y + (int64_t)p * 2 * C : NULL,
                                     dterms ? dterms + 4 * p : NULL, k);
      mat2 M = or_normalised(a, C, k, 1.0 / fs);
      cplx gc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int j = 0; j < 4; ++j)
        for (int i = 0; i < 4; ++i) gc[j] += g_iquv[((int64_t)p * 4 + i) * C + k] * conj(m[i][j]);
      mat2 GC = {{{gc[0], gc[1]}, {gc[2], gc[3]}}};
      mat2 GM = m2_mul(m2_mul(m2_adj(cal.Fi), GC), cal.Fi);
      mat2 GF = m2_mul(m2_mul(m2_add(GC, m2_adj(GC)), cal.Fi), M);
      mat2 GE = m2_scale(m2_mul(m2_mul(m2_adj(cal.Fi), GF), m2_adj(cal.Fi)), -1.0);
      mat2 GG = m2_mul(GE, m2_adj(cal.J));
      mat2 GJ = m2_mul(m2_adj(cal.G), GE);
      if (d_gain_x) {
        d_gain_x[((int64_t)p * C + k) * 2] = creal(GG.m[0][0]);
        d_gain_x[((int64_t)p * C + k) * 2 + 1] = cimag(GG.m[0][0]);
      }
      if (d_gain_y) {
        d_gain_y[((int64_t)p * C + k) * 2] = creal(GG.m[1][1]);
        d_gain_y[((int64_t)p * C + k) * 2 + 1] = cimag(GG.m[1][1]);
      }
      gdx += GJ.m[0][1];
      gdy += GJ.m[1][0];
      /* Re tr(Gb(M)^H M) */
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) norm_term += creal(conj(GM.m[i][j]) * M.m[i][j]);
      cplx* g = gA + ((int64_t)p * C + k) * 4;
      g[0] = GM.m[0][0] / fs; g[1] = GM.m[0][1] / fs;
      g[2] = GM.m[1][0] / fs; g[3] = GM.m[1][1] / fs;
    }
    if (d_dterms) {
      d_dterms[4 * p + 0] = creal(gdx);
      d_dterms[4 * p + 1] = cimag(gdx);
      d_dterms[4 * p + 2] = creal(gdy);
      d_dterms[4 * p + 3] = cimag(gdy);
    }
  }
  int err = OR_OK;
  if (d_w || d_taps) {
    double* c = malloc(sizeof(double) * (size_t)(N / 2));
    double* s = malloc(sizeof(double) * (size_t)(N / 2));
    if (!c || !s) { free(c); free(s); free(gA); free(dw); return OR_ERR_MEM; }
    or_twiddles(N, c, s);
    or_sched q;
    or_sched_init(&q);
    int64_t n_blocks = (F + OR_FRAME_BLOCK - 1) / OR_FRAME_BLOCK;
    int nt = or_thread_count(nthreads, n_blocks);
    or_grad_job job = {packed, bits, n_streams, n_pairs, pair_x, pair_y, N, C, F, hop, w, c, s, gA, dw, &q, OR_OK};
    pthread_t* th = malloc(sizeof(pthread_t) * (size_t)nt);
    for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, or_grad_worker, &job);
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
    free(th);
    or_sched_free(&q);
    free(c); free(s);
    err = job.err;
    for (int64_t n = 0; n < N; ++n) dw[n] += -2.0 * w[n] * norm_term / sumw2;
    if (d_w) memcpy(d_w, dw, sizeof(double) * (size_t)N);
    if (d_taps && taps && n_taps >= 2) or_taps_adjoint(N, n_taps, dw, d_taps);
  }
  free(gA); free(dw);
  return err;
}

int or_version(void) { return 1; }
