// Post-integration reductions: launch arguments and launchers (device code in polaris_post.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ps {

constexpr int kMaxAllanLags = 64;
constexpr int64_t kAllanChunk = 4096;  // points per workgroup of a series (block form)
constexpr int kWinMaxLag = 512;        // largest lag of the LDS-window form (side-by-side series)
constexpr int64_t kMaxSplineCoef = 3072;  // basis functions of one bandpass fit (LDS of the solve)

struct ChanAvgArgs {
  const float* in;          // [n_spec][n_chan]
  int64_t n_spec, n_chan;
  int32_t factor;           // channels per bin
  const uint8_t* flags;     // [n_chan], nonzero = flagged, or nullptr
  float* out;               // [n_spec][n_chan / factor]
  int32_t* counts;          // [n_spec][n_chan / factor] or nullptr
};

struct SplineArgs {
  const float* h;           // [n_chan]
  int64_t n_chan, c0, c1;   // fit channels [c0, c1)
  int32_t K;                // knot spacing (channels)
  int64_t n_int, n_coef;    // intervals, basis functions (n_int + 3)
  double* partial;          // [n_int][14]: Gram entries (q <= p) and right-hand sides of each interval
  double* coef;             // [n_coef]
  float* smooth;            // [n_chan]
};

struct AllanArgs {
  const float* x;
  int64_t n_points, point_stride, n_series, series_stride;
  int32_t n_lags;
  int32_t normalize;
  int32_t lags[kMaxAllanLags];
  double spacing;
  double* out;              // [n_series][n_lags]
  double* part;             // [n_series][chunks][n_lags + 1][2]: per chunk sums and counts (block form)
};

// block form (series not side by side): partial sums per chunk of points; 0 for the side-by-side form
int64_t allan_part_doubles(int64_t n_points, int64_t n_series, int64_t point_stride, int64_t series_stride, int n_lags);

hipError_t launch_channel_average(const ChanAvgArgs& a, hipStream_t s);
hipError_t launch_bandpass_fit(const SplineArgs& a, hipStream_t s);

// Allocation-free bandpass fit: its work (interval partials and coefficients) lives in a static device array
// of this size on each GPU, enough for fits of up to kBandpassScratchCoef spline coefficients.
constexpr int64_t kBandpassScratchCoef = 1024;
constexpr size_t kBandpassScratchBytes = 128 * 1024;
static_assert(((kBandpassScratchCoef - 3) * 14 * 8 + 255) / 256 * 256 + ((kBandpassScratchCoef * 8 + 255) / 256 * 256) <=
                  kBandpassScratchBytes,
              "the scratch holds the work of every fit of kBandpassScratchCoef coefficients");
constexpr int kMaxDevices = 64;
// Device address of the scratch array on the GPU of stream (the current GPU for the null stream), found on
// the first call for that GPU.
hipError_t bandpass_scratch(hipStream_t stream, void** ptr);
hipError_t launch_bandpass_correct(const float* hk, int64_t n_spec, int64_t n_chan, const float* smooth,
                                   const double* gain, float* out, hipStream_t s);
hipError_t launch_band_stats(const float* x, int64_t n_spec, int64_t n_chan, double* mean_sd, hipStream_t s);
hipError_t launch_allan(const AllanArgs& a, hipStream_t s);

}  // namespace ps
