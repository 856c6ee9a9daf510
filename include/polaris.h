/*
 * polaris.h -- C ABI of the MI355X (gfx950) spectrometer library.
 *
 * The library computes, for two-polarization sampler data, the auto- and cross-power spectra of a
 * windowed long FFT per segment, accumulated over an integration, and the calibrated full-Stokes
 * spectra, as described by Mizuno et al., "Software Polarization Spectrometer PolariS" (arXiv 1412.1256):
 *   - Sec. 2, the statement of the spectrometer's four functions (accept two orthogonal polarizations,
 *     FFT them, multiply spectra into power and cross-power spectra, integrate and output);
 *   - Fig. 2 caption (data translation of 4/8-bit integers to floats, segmentation, FFT, cross products,
 *     accumulation) and Table 1 (IFs X0, X1, Y0, Y1; 4 real and 2 complex products; 1-s output);
 *   - Sec. 2.1, Eq. 2 (Stokes I, Q, U, V from the products divided by the complex gain products).
 *
 * Conventions shared by every call:
 *   - Every function returns a ps_status; none throws, prints or exits.  ps_last_error() gives a
 *     thread-local detail string for the last non-OK status.
 *   - The caller owns every device buffer, including the workspace whose size ps_plan reports.  The
 *     library never allocates or frees device memory; a plan owns host metadata only.
 *   - All device work is enqueued asynchronously on the stream given to ps_bind; no call synchronises
 *     except ps_bind itself and the descriptor upload described next.  ps_reset, ps_accumulate,
 *     ps_accumulate_stokes, ps_spectra, ps_stokes, ps_stokes_all, ps_set_window_taps and
 *     ps_calibrate_backward enqueue kernels only (no allocation or memset), so they can be captured into a
 *     hipGraph (ps_graph_begin).
 *   - Plans of several instances run each pass as grouped launches (the batching form), whose
 *     per-instance launch descriptors live in the workspace.  ps_accumulate and ps_stokes_all upload them
 *     (waiting for the stream, then one copy from pinned host memory) only when they differ from the
 *     previous call's, e.g. new buffers or frame counts; during a capture they must be unchanged.
 *   - Argument and size errors are returned before anything is enqueued (no partial work).  Kernel
 *     launch failures return PS_ERR_HIP.  Faults inside kernels surface at the caller's next
 *     synchronisation.
 *   - Layouts: "complex" arrays are interleaved (re, im) pairs; channel k of an N-point segment runs
 *     over k = 0 .. N/2 - 1 (DC kept, Nyquist dropped).
 */
#ifndef POLARIS_H
#define POLARIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PS_OK = 0,
  PS_ERR_ARG = 1,          /* a null pointer, an out-of-range field or inconsistent arguments */
  PS_ERR_SIZE = 2,         /* a sample count that is not a whole number of segments */
  PS_ERR_UNSUPPORTED = 3,  /* a valid request this build does not implement */
  PS_ERR_STATE = 4,        /* call order violated (unbound plan, no frames integrated, ...) */
  PS_ERR_WORKSPACE = 5,    /* workspace missing, too small or misaligned */
  PS_ERR_HIP = 6           /* a HIP runtime call or kernel launch failed */
} ps_status;

/* window kinds (Sec. 3.1: rectangular online; Hanning, Hamming and Blackman as apodisation), periodic forms */
enum { PS_WIN_RECT = 0, PS_WIN_HANN = 1, PS_WIN_TAPS = 2, PS_WIN_HAMMING = 3, PS_WIN_BLACKMAN = 4 };
/* arithmetic of the transform passes */
enum { PS_PREC_FP32 = 0, PS_PREC_FP16 = 1, PS_PREC_BF16 = 2 };
/* accumulator of the integration */
enum { PS_ACC_FP64 = 0, PS_ACC_KAHAN32 = 1 };

typedef struct ps_plan_s* ps_plan_t;

/*
 * One instance = one sampler stream set (Table 1).
 *   n_streams   S, 1..8 streams interleaved in one buffer (Table 1 order, e.g. X0, X1, Y0, Y1).
 *   n_pairs     P, 1..4 polarization pairs; pair p correlates stream pair_x[p] (X) with pair_y[p] (Y).
 *   bits        2 or 4 (offset-binary codes c -> level 2c - (2^b - 1)), 8 (two's-complement int8) or
 *               32 (little-endian float32, a test format).  Item t*S + s of the buffer sits at bit
 *               offset (t*S + s)*bits, least significant bits first.
 *   fft_len     N, a power of two, 2^8 .. 2^22; channels C = N/2; one segment = N samples per stream.
 *   window      PS_WIN_RECT; PS_WIN_HANN (0.5 - 0.5 cos 2 pi n/N), PS_WIN_HAMMING (0.54 - 0.46 cos) or
 *               PS_WIN_BLACKMAN (0.42 - 0.5 cos + 0.08 cos 4 pi n/N), all periodic; or PS_WIN_TAPS (n_taps
 *               control points, linear interpolation at u = n (n_taps - 1)/(N - 1); all ones until
 *               ps_set_window_taps).
 *   precision   PS_PREC_FP32: FP32 transforms.  PS_PREC_FP16 / PS_PREC_BF16 (the precision form,
 *               fft_len 2^16 .. 2^18, any window but PS_WIN_TAPS): each pass as 16 x R blocked DFT matrix
 *               products on the matrix cores with 16-bit inputs and FP32 accumulation, a 16-bit
 *               inter-pass buffer; every stage is scaled by 1/radix (exact), so FP16 values stay within
 *               the input range (|level| < 65504).
 *   accum       PS_ACC_FP64 (any precision), or PS_ACC_KAHAN32 (16-bit passes only): the products of
 *               the frames of one pass launch are summed per channel in registers, in FP64 or in
 *               compensated FP32, then added to FP64 accumulators.
 *   chunk_frames  frames processed per internal pass pair (0 = max(64, 2^25 / N)); bounds the workspace:
 *                 a plan keeps one inter-pass buffer of the largest chunk_frames x n_pairs x N x 8 bytes
 *                 of its instances (at least 128 MiB with several instances), shared by all of them.
 *   sample_rate_hz  metadata only (channel width = sample_rate_hz / N).
 *   hop         segmentation (Sec. 3.1, 50 % overlap): frame f of the stream starts at sample f * hop;
 *               0 or N = contiguous frames, N/2 = 50 % overlap, N/4 or N/8 = 75 or 87.5 %.  An integration
 *               of T samples (in any number of ps_accumulate calls) has (T - N)/hop + 1 frames; the
 *               last N - hop samples of each call are kept in the workspace and transformed with the next
 *               call's first samples.  With level histograms on, every sample is counted once (the first
 *               hop samples of each frame).
 */
typedef struct {
  int32_t n_streams;
  int32_t n_pairs;
  int32_t pair_x[4];
  int32_t pair_y[4];
  int32_t bits;
  int32_t window;
  int32_t n_taps;
  int32_t precision;
  int32_t accum;
  int32_t chunk_frames;
  int64_t fft_len;
  double sample_rate_hz;
  int64_t hop;
} ps_instance;

/*
 * Calibration for Eq. 2.  All pointers are device memory, may be NULL.
 *   gain_x, gain_y  [n_pairs][C] complex float: G_X, G_Y (voltage-domain gains); NULL = 1.
 *   dterms          [n_pairs][4] float: d_x (re, im), d_y (re, im) of the leakage matrix
 *                   J = [[1, d_x], [d_y, 1]] (observed v' = G J v); NULL = 0 (Eq. 2 exactly).
 *   psi             parallactic angle psi_m in radians.
 *   feed            PS_FEED_LINEAR (Eq. 2; pair = X, Y) or PS_FEED_CIRCULAR (pair = R, L): I = (C_rr + C_ll)/2,
 *                   V = (C_rr - C_ll)/2, Q + iU = C_rl exp(2i psi), the combination of R = (X + iY)/sqrt 2,
 *                   L = (X - iY)/sqrt 2 (so both feeds give the same Stokes for the same sky).
 */
enum { PS_FEED_LINEAR = 0, PS_FEED_CIRCULAR = 1 };
typedef struct {
  const float* gain_x;
  const float* gain_y;
  const float* dterms;
  double psi;
  int32_t feed;
  int32_t reserved;
} ps_cal;

/* Gradient outputs of ps_calibrate_backward, device memory, NULL = not wanted.  Complex gradients are
 * (dL/dRe, dL/dIm) pairs, the layout of the matching ps_cal field; d_taps has n_taps floats. */
typedef struct {
  float* d_gain_x;
  float* d_gain_y;
  float* d_dterms;
  float* d_taps;
} ps_cal_grad;

/* Validate n_inst instances, build host tables and report the workspace size (bytes, 256-aligned).  An
 * instance is one sampler stream set with its polarization pairs: Table 1's four IFs X0, X1, Y0, Y1 make one
 * instance of four streams and two pairs (X0, Y0), (X1, Y1); a plan of several instances runs them together.
 * Errors: PS_ERR_ARG for bad fields, PS_ERR_UNSUPPORTED for valid but unimplemented options. */
ps_status ps_plan(const ps_instance* inst, int32_t n_inst, ps_plan_t* out, size_t* workspace_bytes);

/*
 * Schedule of one instance's passes (what the autotuner chooses; every field 0 = the default):
 *   log2_n1         the split N = N1 x N2 of the four-step transform (default floor(log2 N / 2); with FP32
 *                   passes 7, 8, 7, 8, 9 for 2^13 .. 2^17 points, 10 for 2^19 and 9 for 2^20);
 *   colpass_cols    columns per column-pass workgroup (its LDS tile width and workgroup size);
 *   rowpass_frames  frames per row-pass workgroup batch (its workgroup size; default 8, 4 for 1024-point
 *                   rows, 2 for 2048, and 4 for 512-point rows once the row pass has 512 or more
 *                   workgroups);
 *   col_wg_per_cu   column-pass workgroups per CU that the frame grouping aims at (1 .. 8; default 4 for
 *                   2^13, 2 for 2^14 .. 2^16 points with FP32 passes, else 1);
 *   rowpass_slots   accumulator slots G (a power of two, 1 .. 64; 1 .. 8192 in a single pass): frame a of
 *                   the integration goes to slot a mod G, so G frame groups run in parallel; readers sum the
 *                   slots in order.  Default: enough for about 256 row-pass workgroups (512 up to 2^18
 *                   points; 1 for 16-bit
 *                   passes; 2^20 / (N n_pairs) rounded down to a power of two, at most 8192, in a
 *                   single pass).
 *   single_pass     0: the default (a single pass for FP32 transforms of 2^8 .. 2^12 points, else the
 *                   four-step passes); 1: a single pass (each workgroup transforms whole frames in LDS
 *                   and accumulates their products; 2^8 .. 2^12 points, FP32; only log2_n1 and
 *                   rowpass_slots apply); 2: the four-step column and row passes.
 * The results of every schedule agree within rounding; only speed differs.
 */
typedef struct {
  int32_t log2_n1;
  int32_t colpass_cols;
  int32_t rowpass_frames;
  int32_t col_wg_per_cu;
  int32_t rowpass_slots;
  int32_t single_pass;
} ps_schedule;

/* ps_plan with one schedule per instance (sched may be NULL).  PS_ERR_UNSUPPORTED for a schedule that has
 * no compiled kernels for the instance. */
ps_status ps_plan_scheduled(const ps_instance* inst, const ps_schedule* sched, int32_t n_inst, ps_plan_t* out,
                            size_t* workspace_bytes);

/* The schedules that can run an instance (host only): writes up to capacity of them to out (may be NULL)
 * and their total number to *count. */
ps_status ps_schedule_candidates(const ps_instance* inst, ps_schedule* out, int32_t capacity, int32_t* count);

/* Attach a device workspace (>= the reported size, 256-byte aligned) and a HIP stream (hipStream_t,
 * NULL = the default stream); uploads the FP64-generated twiddle and window tables of the transforms of
 * Sec. 2 (function 2) and waits for the upload.  Re-binding is allowed and resets every integration. */
ps_status ps_bind(ps_plan_t plan, void* workspace_dev, size_t bytes, void* hip_stream);

/* Set the n_taps window control points of a PS_WIN_TAPS instance from device floats (enqueued). */
ps_status ps_set_window_taps(ps_plan_t plan, int32_t inst, const float* taps_dev);

/* Start a new integration for every instance (Sec. 2, function 4: the products are integrated from here
 * on; Table 1's output period is 1 s).  Host bookkeeping only; enqueues nothing. */
ps_status ps_reset(ps_plan_t plan);

/* Add whole segments to each instance's integration: Sec. 2 functions 1-4 (accept the two polarizations,
 * Fourier-transform them, multiply the spectra into power and cross-power spectra, integrate), in the
 * Fig. 2 caption's order (data translation, segmentation, FFT, cross products, accumulation).
 *   packed_dev[i]   device pointer to instance i's packed buffer (layout above); may be NULL when
 *                   n_samples[i] == 0.
 *   n_samples[i]    samples per stream, a multiple of fft_len (PS_ERR_SIZE otherwise).
 * Frames are added in order; with FP32 passes, splitting one input over several calls gives bitwise the
 * same sums (with 16-bit passes the same up to the rounding of the per-launch sums).
 * In a plan of several instances, the FP32 instances of a call run together: per chunk round, instances of
 * one shape class (split, sample format, schedule) share a column-pass launch and a row-pass launch with
 * one workgroup per tile of all of them, in sub-batches of at most 128 MB of inter-pass data, each row
 * pass right after its column pass (up to 8 chunk rounds per call; beyond that instance by instance). */
ps_status ps_accumulate(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples);

/* ps_accumulate followed by the Stokes spectra of the integration so far (Sec. 2 functions 2-4, then Eq. 2 of
 * Sec. 2.1), for a streaming loop that outputs every integration: cal is NULL or n_inst calibrations,
 * iquv_dev NULL or n_inst device pointers ([n_pairs][4][C] floats each; NULL entries skip an instance).  The
 * results are those of ps_accumulate, then ps_stokes_all.  An instance with one accumulator slot and FP32
 * four-step passes gets its Stokes spectra from the last row pass of the call (the final sums are still in
 * registers there; no separate output launch, no re-read of the accumulators), the others from one output
 * launch after the accumulation (grouped when there are several).  PS_ERR_STATE, before anything is enqueued, when a selected
 * instance would have no frame. */
ps_status ps_accumulate_stokes(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples,
                               const ps_cal* cal, float* const* iquv_dev);

/* Raw accumulated products of instance inst into out_dev [n_pairs][4][C] doubles: Table 1's four real and
 * two complex products per pair of IFs, i.e. the sums over frames of XX*, YY*, Re XY*, Im XY* (unnormalised),
 * and the frame count (host).
 * PS_ERR_STATE if no frame has been accumulated since ps_reset. */
ps_status ps_spectra(ps_plan_t plan, int32_t inst, double* out_dev, int64_t* n_frames);

/* Calibrated full-Stokes spectra (Eq. 2) of instance inst into iquv_dev [n_pairs][4][C] floats
 * (I, Q, U, V), computed in FP64 from M = A / (F sum w^2) and C = (G J)^-1 M (G J)^-H.  cal may be NULL
 * (unit gains, no leakage, psi = 0).  The integration is read, not consumed. */
ps_status ps_stokes(ps_plan_t plan, int32_t inst, const ps_cal* cal, float* iquv_dev);

/* Stokes spectra of every instance whose iquv_dev[i] is not NULL, in one launch (the batching
 * form).  cal: NULL or an array of n_inst calibrations; iquv_dev: n_inst device pointers, each
 * [n_pairs][4][C] floats.  PS_ERR_STATE if a selected instance has no accumulated frame. */
ps_status ps_stokes_all(ps_plan_t plan, const ps_cal* cal, float* const* iquv_dev);

/* Level histograms and total power (Sec. 2: total power from the samplers' bit distributions).
 * ps_set_histograms switches counting on or off for instance inst (2-, 4- or 8-bit codes, FP32 passes;
 * PS_ERR_STATE inside an integration).  While on, the column pass counts every sample of each pair's two
 * streams; the counts start at zero with the first ps_accumulate after ps_reset.
 * ps_histograms returns, for the current integration (either pointer may be NULL):
 *   counts_dev  [n_pairs][2 (X, Y)][2^bits] uint64, bins in ascending level order (code c of a 2/4-bit
 *               sample, level + 128 of an int8 one);
 *   power_dev   [n_pairs][2][2] doubles: the mean square level (total power in level units) and, for
 *               2-bit samplers, sigma / threshold = 1 / (sqrt 2 erfinv(P)) from the fraction P of samples
 *               in the two inner levels (NaN for other formats);
 *   n_frames    frames counted.  PS_ERR_STATE when nothing has been counted since ps_reset. */
ps_status ps_set_histograms(ps_plan_t plan, int32_t inst, int32_t enable);
ps_status ps_histograms(ps_plan_t plan, int32_t inst, uint64_t* counts_dev, double* power_dev, int64_t* n_frames);

/* hipGraph capture of a sequence of calls on the plan's stream (the batching form's streaming loop):
 *   ps_graph_begin   starts capturing the bound stream (not the null stream; profiling must be off);
 *   ps_graph_end     ends the capture; keep != 0 instantiates the graph (replacing an earlier one),
 *                    keep == 0 discards what was captured (e.g. after a call failed during the capture);
 *   ps_graph_launch  replays it on the bound stream and restores the plan's host state (frame counts) to
 *                    what it was at the end of the capture.
 * A captured sequence is meant to be a whole integration: ps_reset, ps_accumulate on fixed input buffers,
 * then ps_stokes / ps_stokes_all into fixed outputs.  Make the same calls once before capturing, so the
 * launch descriptors are already in place.  PS_ERR_STATE for calls out of order. */
ps_status ps_graph_begin(ps_plan_t plan);
ps_status ps_graph_end(ps_plan_t plan, int32_t keep);
ps_status ps_graph_launch(ps_plan_t plan);

/* Gradient of a real loss L(iquv) with respect to the gains, leakage terms and window taps, given
 * dL_diquv_dev [n_pairs][4][C] floats.  Needs the current integration (the forward's accumulators,
 * not reset) and the same packed input (n_samples per stream, all frames of the integration).  When the
 * integration was one ps_accumulate call of at most chunk_frames frames and nothing has written the
 * workspace's inter-pass buffer since (no other accumulate on the plan, no graph replay), its column-pass
 * output is used as it stands; otherwise the frames are transformed again.  The call overwrites that buffer.
 * PS_ERR_STATE if the frame count does not match. */
ps_status ps_calibrate_backward(ps_plan_t plan, int32_t inst, const void* packed_dev, int64_t n_samples,
                                const ps_cal* cal, const float* dL_diquv_dev, const ps_cal_grad* grad);

/* Integration id of instance inst: a number that changes whenever the state ps_calibrate_backward reads
 * changes (ps_reset, ps_accumulate or ps_accumulate_stokes with frames, ps_set_window_taps, ps_state_import,
 * ps_graph_launch, ps_bind).  A caller that takes a gradient later, e.g. an autograd node, records the id after
 * its forward and compares it before the backward: a different id means another forward ran on the plan in
 * between, and the backward would return that forward's gradients. */
ps_status ps_integration_id(ps_plan_t plan, int32_t inst, uint64_t* id);

/* Integration state for checkpoint and resume: the accumulators and, for overlapped segmentation, the
 * samples waiting for the next call (the frame count is passed separately).  Device buffers of
 * ps_state_bytes bytes; export and import are enqueued on the plan's stream. */
ps_status ps_state_bytes(ps_plan_t plan, int32_t inst, size_t* bytes);
ps_status ps_state_export(ps_plan_t plan, int32_t inst, void* dst_dev, int64_t* n_frames);
ps_status ps_state_import(ps_plan_t plan, int32_t inst, const void* src_dev, int64_t n_frames);

/* Stand-alone data translation (Fig. 2 caption): decode n_time x n_streams items of a packed buffer into
 * out_dev[s * n_time + t] floats (exact for every format), enqueued on hip_stream. */
ps_status ps_unpack(const void* packed_dev, int32_t bits, int32_t n_streams, int64_t n_time, float* out_dev,
                    void* hip_stream);

/*
 * Post-integration reductions on integrated spectra (device buffers; each call is enqueued on hip_stream and
 * allocates nothing).  Sums are FP64 in a fixed order: results are identical from run to run.  Non-finite
 * values (e.g. channels outside a fitted band) are left out like flagged channels.
 *
 * Channel averaging (Sec. 4: 131072 channels averaged to 1.95-kHz resolution after flagging a spurious
 * channel).  in [n_spec][n_chan] float; flags [n_chan] uint8, nonzero = flagged, or NULL; factor divides
 * n_chan (else PS_ERR_SIZE); n_spec <= 65535.  out [n_spec][n_chan/factor]: the mean of the bin's unflagged
 * finite channels, NaN when there are none; counts [n_spec][n_chan/factor] (may be NULL).
 */
ps_status ps_channel_average(const float* in_dev, int64_t n_spec, int64_t n_chan, int32_t factor,
                             const uint8_t* flags_dev, float* out_dev, int32_t* counts_dev, void* hip_stream);

/*
 * Smoothed bandpass table H (Sec. 3.3.2: a long integration smoothed by a spline 128 channels wide, 6 % of
 * the band left out at each end): the least-squares cubic spline with uniform knots every knot_spacing
 * channels from c0 = floor(edge_frac n_chan), fitted to channels [c0, n_chan - c0) of h [n_chan] float;
 * smooth [n_chan] float holds the spline there and NaN outside.  The range must hold at least four knot
 * intervals (PS_ERR_SIZE) and give at most 3072 spline coefficients (PS_ERR_UNSUPPORTED).  work: a 256-byte
 * aligned device buffer of ps_bandpass_work_bytes bytes, owned by the caller.
 */
ps_status ps_bandpass_work_bytes(int64_t n_chan, int32_t knot_spacing, double edge_frac, size_t* bytes);
ps_status ps_bandpass_fit(const float* h_dev, int64_t n_chan, int32_t knot_spacing, double edge_frac,
                          void* work_dev, size_t work_bytes, float* smooth_dev, void* hip_stream);

/* ps_bandpass_fit for callers that cannot allocate device memory (code under hipGraph capture, serving
 * loops, harnesses that forbid allocation): the same kernels, with the work buffer taken from a static
 * device array of 128 KiB that each GPU holds until the process ends, enough for fits of up to 1024
 * spline coefficients (131072 channels at 128-channel knots need 905).  Allocates nothing and calls no
 * allocating routine; its first call on a GPU looks up that GPU's copy of the array.  Larger fits return
 * PS_ERR_SIZE before anything is enqueued.  Every call on one GPU uses the same array (every byte a call
 * reads is written earlier in that call, so nothing carries over), so calls that overlap on one GPU, e.g.
 * on two streams at once, race. */
ps_status ps_bandpass_fit_static(const float* h_dev, int64_t n_chan, int32_t knot_spacing, double edge_frac,
                                 float* smooth_dev, void* hip_stream);

/* Bandpass variation (Sec. 3.3.2): out[k][c] = hk[k][c] / (gain[k] smooth[c]) for spectra k < n_spec
 * (<= 65535) of n_chan channels; gain [n_spec] double (the total-power gain G_k of each integration) or NULL
 * (= 1).  FP64 arithmetic, FP32 output. */
ps_status ps_bandpass_correct(const float* hk_dev, int64_t n_spec, int64_t n_chan, const float* smooth_dev,
                              const double* gain_dev, float* out_dev, void* hip_stream);

/* Band statistics (Sec. 3.3.3): mean_sd[k] = (mean, sqrt(<x^2> - <x>^2)) of spectrum k's finite channels
 * (NaN, NaN when none), as double [n_spec][2]. */
ps_status ps_band_stats(const float* x_dev, int64_t n_spec, int64_t n_chan, double* mean_sd_dev, void* hip_stream);

/*
 * Allan variance of a second difference: Eq. 3 (time-based, TAV: a series of integrations at one channel)
 * and Eq. 4 (spectral, SAV: the channels of one spectrum).  Series s has n_points samples
 * x[s * series_stride + t * point_stride] (float, strides in elements).  For each of the n_lags (1..64) lags
 * L (host int32, >= 1): out[s][l] = mean over t of (x[t+L] - 2 x[t] + x[t-L])^2 / (2 (L spacing)^2), t with
 * all three samples finite, NaN when there is none (2 L >= n_points); spacing is the sample interval (s for
 * TAV, Hz for SAV).  normalize != 0 divides each series by the mean of its finite samples first.  out:
 * double [n_series][n_lags].  work: a device buffer of ps_allan_work_bytes bytes owned by the caller (partial
 * sums per chunk of 4096 points; 0 bytes, and NULL allowed, when the series lie side by side, series_stride 1).
 */
ps_status ps_allan_work_bytes(int64_t n_points, int64_t point_stride, int64_t n_series, int64_t series_stride,
                              int32_t n_lags, size_t* bytes);
ps_status ps_allan(const float* x_dev, int64_t n_points, int64_t point_stride, int64_t n_series,
                   int64_t series_stride, const int32_t* lags, int32_t n_lags, double spacing, int32_t normalize,
                   void* work_dev, size_t work_bytes, double* out_dev, void* hip_stream);

/* Free a plan's host metadata (never the caller's device memory). NULL is accepted. */
ps_status ps_destroy(ps_plan_t plan);

const char* ps_status_string(ps_status status);
const char* ps_last_error(void);

/* Per-kernel timing for measurement.  While enabled, every kernel a plan launches is bracketed by two
 * hipEvents recorded on the bound stream (up to 16384 launches are kept; later ones are not timed).
 * ps_profile_read waits for the recorded events, returns the summed milliseconds and launch counts per
 * kernel kind (arrays of PS_KERNEL_COUNT entries) and clears the record.  Keep profiling disabled while a
 * hipGraph is being captured. */
enum {
  PS_KERNEL_COLPASS = 0,   /* unpack + window + column transforms + four-step twiddle */
  PS_KERNEL_ROWPASS = 1,   /* row transforms + cross power + accumulation */
  PS_KERNEL_STOKES = 2,    /* calibration + Eq. 2 */
  PS_KERNEL_SPECTRA = 3,   /* raw spectra in channel order */
  PS_KERNEL_BACKWARD = 4,  /* adjoint kernels */
  PS_KERNEL_OTHER = 5,
  PS_KERNEL_COUNT = 8
};
ps_status ps_profile_enable(ps_plan_t plan, int32_t enable);
ps_status ps_profile_read(ps_plan_t plan, double* ms_total, int64_t* launches);

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t ps_version(void);

#ifdef __cplusplus
}
#endif
#endif /* POLARIS_H */
