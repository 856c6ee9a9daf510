/*
 * polaris_oracle.h -- FP64 reference of the PolariS spectrometer path (test infrastructure only).
 *
 * Every array is host memory owned by the caller.  Complex arrays are interleaved (re, im) doubles.
 * Functions return OR_OK (0) or a negative error code; none of them prints or exits.
 */
#ifndef POLARIS_ORACLE_H
#define POLARIS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_ERR_ARG = -1, OR_ERR_MEM = -2 };
enum { OR_WIN_RECT = 0, OR_WIN_HANN = 1, OR_WIN_TAPS = 2, OR_WIN_HAMMING = 3, OR_WIN_BLACKMAN = 4 };

/* Decode n_time x n_streams items of a packed buffer into levels, out[s * n_time + t]. */
int or_unpack(const uint8_t* packed, int bits, int n_streams, int64_t n_time, double* out);

/* Window samples w[0..n) and optionally sum of w^2. taps/n_taps are used by OR_WIN_TAPS only. */
int or_window(int kind, int64_t n, const double* taps, int n_taps, double* w, double* sumsq);

/* In-place forward FFT (unnormalised, exp(-2 pi i n k / n)); n a power of two. */
int or_fft(double* re, double* im, int64_t n);

/* Brute-force DFT of the same convention (any n). */
int or_dft(const double* re, const double* im, int64_t n, double* out_re, double* out_im);

/* Raw accumulated products acc[p][q][k], q = XX*, YY*, Re XY*, Im XY*; k < fft_len/2.  Frame f covers
 * samples f*hop .. f*hop + fft_len - 1 (hop 0 = fft_len; else fft_len / 2^j); frames = (n_time - fft_len)/hop + 1. */
int or_accumulate(const uint8_t* packed, int bits, int n_streams, int64_t n_time, int64_t fft_len, int64_t hop,
                  const double* w, int n_pairs, const int* pair_x, const int* pair_y, int nthreads,
                  double* acc, int64_t* n_frames);

/* Calibrated Stokes iquv[p][0..3][k] = I, Q, U, V from raw products (Eq. 2 with gains and leakage).
 * gain_x, gain_y: [p][k] complex or NULL (= 1); dterms: [p] x (d_x re, im, d_y re, im) or NULL (= 0).
 * feed: OR_FEED_LINEAR (Eq. 2) or OR_FEED_CIRCULAR (the pair's streams are R, L). */
enum { OR_FEED_LINEAR = 0, OR_FEED_CIRCULAR = 1 };
int or_stokes(const double* acc, int n_pairs, int64_t n_chan, int64_t n_frames, double sumw2,
              const double* gain_x, const double* gain_y, const double* dterms, double psi, int feed,
              double* iquv);

/* Gradient of a loss L(iquv) given g_iquv = dL/d iquv ([p][4][k]).  Complex gradients are returned as
 * (dL/dRe, dL/dIm).  d_w is dL/dw[n]; d_taps folds it onto the piecewise-linear taps.  NULL outputs are
 * skipped. */
int or_calibrate_backward(const uint8_t* packed, int bits, int n_streams, int64_t n_time, int64_t fft_len,
                          int64_t hop, const double* w, const double* taps, int n_taps, int n_pairs, const int* pair_x,
                          const int* pair_y, const double* acc, int64_t n_frames, double sumw2,
                          const double* gain_x, const double* gain_y, const double* dterms, double psi,
                          const double* g_iquv, int nthreads, double* d_gain_x, double* d_gain_y,
                          double* d_dterms, double* d_w, double* d_taps);

int or_version(void);

#ifdef __cplusplus
}
#endif
#endif
