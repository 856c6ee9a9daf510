// polaris_internal.h -- launch descriptors shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace ps {

// Frame transform of length N = N1 * N2 (four-step):
//   pass A ("column" pass): for each n2, an N1-point DFT over n1 of x[n1*N2 + n2], then the twiddle
//     W_N^(k1*n2); result T[k1][n2];
//   pass B ("row" pass): for each k1, an N2-point DFT over n2 of T[k1][n2] -> Z[k1 + N1*k2].
// The two real streams of a pair travel as one complex sequence z = x + i*y, so one length-N complex
// transform gives both spectra: X[k] = (Z[k] + conj Z[N-k]) / 2, Y[k] = (Z[k] - conj Z[N-k]) / (2i).

struct ColArgs {
  const uint8_t* in;        // packed input of the first frame of this launch
  uint32_t in_bytes;        // bytes of input in this launch (< 2^31 on the int8 two-stream path)
  int64_t N;                // frame length
  int64_t hop;              // samples from one frame's start to the next (N, or N / 2^j for overlap)
  int32_t N2;               // columns
  int32_t S, P;             // streams, pairs
  int32_t px[4], py[4];     // pair -> stream
  int32_t n_colblk;         // column blocks per (frame, pair)
  int32_t n_frames;         // frames in this launch
  int32_t frames_per_block; // frames looped over by one workgroup
  const float* win;         // window [N] or nullptr (rectangular)
  const float2* tw_col;     // W_N1^m, m < N1
  const float2* tw_hi;      // W_N^(m << lo_bits)
  const float2* tw_lo;      // W_N^m, m < 2^lo_bits
  int32_t lo_bits;
  float2* T;                // [n_frames][P][N1][N2]
  unsigned long long* hist; // level histograms [P][2][2^bits] to add to, or nullptr
  int32_t hist_rows;        // rows n1 < hist_rows (the frame's first hop samples) are counted
  int32_t pad_;
};

// Accumulator slots: absolute frame a (counted from ps_reset) is added to slot a mod G, frames of a slot in
// order; readers sum the slots 0 .. min(G, frames) - 1 in order.  G > 1 lets the row pass of short
// transforms (few row units) run frame groups in parallel, and the result does not depend on how the
// frames were split over calls.
struct RowArgs {
  const float2* T;          // [n_frames][P][N1][N2]
  int32_t N1, P, n_frames;
  const float2* tw_row;     // W_N2^m, m < N2
  double* acc;              // [G][P][N1/2][4][N2]: unit-major accumulators of 4 XX*, 4 YY*, 4 XY*
  int32_t G;                // accumulator slots
  int64_t F0;               // frames accumulated since ps_reset before this launch
  int64_t slot_stride;      // doubles per slot
};

struct OutArgs {
  const double* acc;        // [slots][P][N1/2][4][N2]
  int32_t slots;            // slots to sum (min(G, frames))
  int64_t slot_stride;
  int32_t N1, N2, P;
  int64_t C;
  // Stokes only
  double scale;             // 1 / (F * sum w^2) when sumw2_dev == nullptr
  const double* sumw2_dev;  // device sum of w^2 (taps window) or nullptr
  double n_frames;
  const float* gain_x;      // [P][C] complex or nullptr
  const float* gain_y;
  const float* dterms;      // [P][4] or nullptr
  double cos2psi, sin2psi;
  int32_t circular;         // 1: the pair's streams are R, L
  float* iquv;              // [P][4][C]
  double* spectra;          // [P][4][C] (raw sums) when producing spectra
};

// ---- precision form (FP16 / BF16 blocked-DFT passes on the matrix cores) -----------------------
//
// Each N1- and N2-point DFT is split as 16 x R (R = 16 or 32): n = R*a + b, k = kappa + 16*kb.  Stage A is
// a 16-point DFT over a for every b, stage B an R-point DFT over b for every kappa; both are products of
// the DFT matrix (as a 2r x 2r real block, FP16/BF16 hi + lo parts) with 16 vectors at a time, FP32
// accumulate.  Between the stages the twiddle W^(b*kappa) is applied in FP32 and the result rounded to
// the 16-bit format; every stage is scaled by 1/r (exact), so stored values never exceed the input range.
// The inter-pass buffer holds packed 16-bit complex values [n_frames][P][N1][N2].

struct MxMats {
  const uint32_t* a16;      // radix-16 matrix, A-operand lane layout [hi, lo][2 tiles][64 lanes][4 words]
  const uint32_t* aR;       // radix-R matrix [hi, lo][2R/16 tiles][R/16 K-steps][64 lanes][4 words]
  const float2* tws;        // W_L^m / 16, m < L (stage twiddle with the 1/16 of stage A)
};

struct MxColArgs {
  ColArgs col;              // geometry and input; col.T is unused
  MxMats m;
  uint32_t* T;              // packed 16-bit complex [n_frames][P][N1][N2]
  int32_t mode;             // input access: 0 generic, 1 int8 two streams pair (0,1), 2 int8 four streams,
                            // 3 int8 four streams as the pairs (0,2), (1,3), both in one workgroup
};

struct MxRowArgs {
  const uint32_t* T;
  int32_t N1, P, n_frames;
  MxMats m;
  double* acc;              // [P][N1/2][4][N2] FP64, unscaled
  int32_t first;
  double unscale;           // 1 / (product scale)^2 of the stages: multiplies the sums before they are stored
};


// ---- differentiation form ----------------------------------------------------------------------

struct WinArgs {            // learnable window from its control points
  const float* taps;        // the caller's control points
  float* taps_copy;         // [n_taps] the plan's copy of them (for the adjoint), written by the first block
  int32_t n_taps;
  int64_t N;
  float* win;               // [N]
  double* partial;          // per-block sums of w^2
};

struct BwChanArgs {         // per-channel adjoint of Eq. 2 and the calibration
  const double* acc;        // [slots][P][N1/2][4][N2]
  int32_t slots;
  int64_t slot_stride;
  int32_t N1, P;
  int64_t C;
  double n_frames;
  const double* sumw2;
  const float* gain_x;
  const float* gain_y;
  const float* dterms;
  double cos2psi, sin2psi;
  const float* g_iquv;      // [P][4][C] upstream gradient
  float* d_gain_x;          // [P][C] complex, or nullptr
  float* d_gain_y;
  float* d_dterms;          // [P][4], or nullptr
  float* g_a;               // [P][N1/2][4][N2] Gb(A) (00, 11, Re 01, Im 01), or nullptr
  double* red;              // [P][parts][5] partials of the units' channel slots (bw_parts per pair)
  int32_t parts;            // partials per pair
  double* norm;             // [P] Re tr(Gb(M)^H M)
};

struct BwRowArgs {          // backward row pass (in place on the inter-pass buffer)
  float2* T;
  int32_t N1, P, n_frames;
  const float2* tw_row;
  const float2* tw_hi;
  const float2* tw_lo;
  int32_t lo_bits;
  const float* g_a;
};

struct BwColArgs {          // backward column pass
  ColArgs col;              // col.T is the row pass's output; col.in the packed samples
  double* dw;               // [groups][P][N] partial dL/dw
  int32_t first;            // 1: write the partials instead of adding to them
};

struct BwTapArgs {          // tap gradient
  const double* dw;         // [groups][N] partials to sum in order
  int32_t groups;
  int64_t N;
  int32_t n_taps;
  const float* taps;
  const double* sumw2;
  const double* norm;       // [P]
  int32_t P;
  float* d_taps;
  double* part;             // [ceil(N / 256)][8] per-block tap sums of the one-pass form, or nullptr
  // one-pass form: the channel kernel's per-unit partials [P][U][5], reduced here (normaliser; leakage
  // gradients into d_dterms [P][4] when not nullptr)
  const double* red;
  int32_t U;                // partials per pair in red
  float* d_dterms;
};

// Stream of a launch, and optionally two events the dispatch itself stamps with the kernel's start and end.
struct Launch {
  hipStream_t stream;
  hipEvent_t start;
  hipEvent_t stop;
};

// ---- batching form: one launch per pass and shape over the tiles of many instances, a workgroup per tile
struct BatchArgs {
  const void* tasks;        // device array of ColArgs / RowArgs / OutArgs, one per instance
  const int32_t* tile_end;  // device array: running total of tiles up to and including each task
  int32_t n_tasks;
  int32_t total;            // tiles of all tasks (the grid; at least 1)
};

hipError_t launch_colpass_batch(int N1, int cols, int bits, int mode, const BatchArgs& b, const Launch& l);
hipError_t launch_rowpass_batch(int N2, int fb, const BatchArgs& b, const Launch& l);
hipError_t launch_output_batch(bool stokes, const BatchArgs& b, const Launch& l);
int rowpass_units_per_tile(int N2);
int output_tiles(int N1, int N2, int P);

int colpass_cols(int N1);     // default columns per column-pass workgroup
bool colpass_has(int N1, int cols);
int rowpass_frames(int N2);   // default frames per row-pass workgroup batch
bool rowpass_has(int N2, int fb);
hipError_t launch_colpass_mx(int N1, int prec, int bits, const MxColArgs& a, int n_blocks, const Launch& l);
hipError_t launch_rowpass_mx(int N2, int prec, int accum, const MxRowArgs& a, const Launch& l);

hipError_t launch_colpass(int N1, int cols, int bits, int mode, const ColArgs& a, const Launch& l);
// o != nullptr (one accumulator slot): the row pass also writes the Stokes spectra described by *o
hipError_t launch_rowpass(int N2, int fb, const RowArgs& a, const Launch& l, const OutArgs* o = nullptr);
hipError_t launch_stokes(const OutArgs& a, const Launch& l);
hipError_t launch_spectra(const OutArgs& a, const Launch& l);
hipError_t launch_unpack(const void* packed, int bits, int S, int64_t n_time, float* out, hipStream_t s);

constexpr int kMaxBwGroups = 32;  // partial dL/dw buffers of the backward column pass (groups x pairs)
int window_taps_blocks(int64_t N);
hipError_t launch_window_taps(const WinArgs& a, int n_blocks, double* sumw2, const Launch& l);
// with_reduce: also the per-pair reduction of the unit partials (leakage gradients, normaliser); without
// it, the one-pass tap gradient reduces them
hipError_t launch_bw_channel(int N2, const BwChanArgs& a, const Launch& l, bool with_reduce = true);
hipError_t launch_bw_rowpass(int N2, const BwRowArgs& a, const Launch& l);
int bw_parts(int N1, int N2);  // partials per pair of the per-channel adjoint
hipError_t launch_bw_colpass(int N1, int bits, bool fast, const BwColArgs& a, const Launch& l);
hipError_t launch_bw_taps(const BwTapArgs& a, const Launch& l);
bool bw_taps_block_form(int64_t N, int n_taps);  // the one-pass tap gradient applies (else two kernels)
int64_t bw_taps_part_doubles(int64_t N);         // its per-block sums
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_hist_power(const unsigned long long* counts, int n_streams, int bits, double* power,
                             const Launch& l);

}  // namespace ps
