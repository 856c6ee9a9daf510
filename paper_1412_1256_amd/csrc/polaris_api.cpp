// polaris_api.cpp -- host side of the C ABI declared in include/polaris.h.
//
// Validation, workspace layout, FP64-generated twiddle and window tables, integration bookkeeping and
// the launch sequence of each call.  No device memory is allocated here: the caller's workspace holds
// every table, the FP32 inter-pass buffer and the FP64 accumulators.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/polaris.h"
#include "polaris_internal.h"
#include "polaris_post.h"
#include "polaris_fused.h"

namespace {

thread_local std::string g_last_error;

ps_status fail(ps_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ps_status fail(ps_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

ps_status hip_fail(hipError_t e, const char* what) {
  return fail(PS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr double kTwoPi = 6.283185307179586476925286766559;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int ilog2_exact(int64_t n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int m = 0;
  while ((int64_t(1) << m) < n) ++m;
  return m;
}

// W_len^m = exp(-2 pi i m / len) for m < count, evaluated in FP64 at exactly reduced arguments and
// rounded once to FP32.
void twiddle_table(std::vector<float>& out, int64_t len, int64_t count) {
  out.resize(2 * (size_t)count);
  for (int64_t m = 0; m < count; ++m) {
    const double a = kTwoPi * (double)(m % len) / (double)len;
    out[2 * m] = (float)std::cos(a);
    out[2 * m + 1] = (float)-std::sin(a);
  }
}

struct Inst {
  ps_instance cfg{};
  int m = 0, m1 = 0, m2 = 0;
  int64_t N = 0, C = 0, N1 = 0, N2 = 0, chunk = 0;
  int load_mode = 0;  // column-pass loader: 0 decode at use, 1 two-stream words, 2 four-stream words
  size_t off_tw_col = 0, off_tw_row = 0, off_tw_lo = 0, off_win = 0, off_taps = 0, off_sumw2 = 0;
  size_t off_T = 0, off_acc = 0, end = 0;
  // differentiation form: window partial sums, Gb(A), per-unit partials, normaliser terms, partial dL/dw
  size_t off_wpart = 0, off_ga = 0, off_red = 0, off_norm = 0, off_dw = 0, off_tpart = 0;
  bool taps() const { return cfg.window == PS_WIN_TAPS; }
  std::vector<float> tw_col, tw_row, tw_lo, win, ones;
  // schedule (autotuner's choices): columns per column-pass workgroup, frames per row-pass batch,
  // column-pass workgroups per CU aimed at by the frame grouping
  int cols = 0, fb = 0, col_wgs = 1;
  int G = 1;  // accumulator slots (row-pass frame groups)
  // single pass: whole frames transformed in LDS (short FP32 transforms), with the table W_N^m, m < N
  bool fused = false;
  size_t off_tw_full = 0;
  std::vector<float> tw_full;
  // level histograms (total power): counted by the column pass while on; zeroed by the first accumulate
  // after a reset
  bool hist_on = false, hist_zeroed = false;
  int64_t hist_frames = 0;
  size_t off_hist = 0;
  int64_t hist_bins() const { return cfg.bits <= 8 ? (int64_t(1) << cfg.bits) : 0; }
  // precision form: 16-bit DFT matrices of radix 16 and 32 (hi, lo), stage twiddles of the two passes
  bool mx() const { return cfg.precision != PS_PREC_FP32; }
  size_t off_mx16 = 0, off_mx32 = 0, off_tws_col = 0, off_tws_row = 0;
  std::vector<uint32_t> mx16, mx32;
  std::vector<float> tws_col, tws_row;
  double sumw2 = 0.0;
  bool first = true;
  int64_t n_frames = 0;
  // segmentation: frame f at sample f * hop; with overlap the last N - hop samples of a call wait in the
  // first half of the staging buffer [2][N - hop samples]
  int64_t hop = 0;
  size_t off_stage = 0;
  bool overlap() const { return hop < N; }
  int64_t bits_per_sample() const { return (int64_t)cfg.n_streams * cfg.bits; }
  size_t tail_bytes() const { return (size_t)((N - hop) * bits_per_sample() / 8); }
  int64_t frames_in(int64_t T) const { return T < N ? 0 : (T - N) / hop + 1; }
  size_t slot_doubles() const { return (size_t)cfg.n_pairs * (size_t)(N1 / 2) * 4 * (size_t)N2; }
  size_t acc_bytes() const { return (size_t)G * slot_doubles() * sizeof(double); }
  int slots_used() const { return (int)std::min<int64_t>(G, n_frames); }
  // readers of more than kDirectSlots slots take their sum from a reduction into one slot
  size_t off_sumacc = 0, off_sumpart = 0;
  bool use_reduced() const { return slots_used() > ps::kDirectSlots; }
  // accumulate-and-Stokes request of the current call: output, calibration (may be null), and whether the
  // last row pass wrote the Stokes spectra itself
  float* fuse_iquv = nullptr;
  const ps_cal* fuse_cal = nullptr;
  bool fuse_done = false;
  bool can_fuse() const { return !fused && !mx() && G == 1; }
  // integration id: changes whenever the state a gradient would be taken of changes (reset, frames added,
  // window taps set, state imported, graph replayed, plan re-bound)
  uint64_t gen = 0;
};

}  // namespace

struct ps_plan_s {
  std::vector<Inst> inst;
  size_t ws_bytes = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  int n_cu = 256;  // compute units of the bound device
  size_t off_T = 0, t_bytes = 0;  // the inter-pass buffer shared by every instance
  // per-kernel timing (measurement only)
  bool prof = false;
  std::vector<hipEvent_t> ev;       // pairs (start, stop)
  std::vector<int> ev_kind;         // kernel kind of each recorded pair
  size_t ev_used = 0;
  // batching form: launch descriptors of the grouped passes (device copy in the workspace, host copy
  // in pinned memory), uploaded only when they change
  struct Desc {
    size_t off = 0, cap = 0;                 // device region
    unsigned char* host = nullptr;           // pinned staging
    std::vector<unsigned char> current;      // what the device region holds
  };
  Desc acc_desc, out_desc;
  // graph of a captured integration and the host state it leaves behind
  hipGraphExec_t gexec = nullptr;
  bool capturing = false;
  struct InstState {
    bool first, hist_zeroed;
    int64_t n_frames, hist_frames;
  };
  std::vector<InstState> graph_state;
  uint64_t gen_counter = 0;
  // The inter-pass buffer still holds the column-pass output of instance t_inst's whole integration
  // (generation t_gen, every frame in one launch) when t_inst >= 0: the adjoint then uses it instead of
  // recomputing the column pass.  Any other write of the buffer, or change of the integration, clears it.
  int t_inst = -1;
  uint64_t t_gen = 0;
  void touch(Inst& I) {
    I.gen = ++gen_counter;
    t_inst = -1;
  }
  ~ps_plan_s() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (acc_desc.host) (void)hipHostFree(acc_desc.host);
    if (out_desc.host) (void)hipHostFree(out_desc.host);
    if (gexec) (void)hipGraphExecDestroy(gexec);
  }
};

namespace {

ps_status validate_instance(const ps_instance& c, int idx) {
  if (c.n_streams < 1 || c.n_streams > 8) return fail(PS_ERR_ARG, "instance %d: n_streams %d not in 1..8", idx, c.n_streams);
  if (c.n_pairs < 1 || c.n_pairs > 4) return fail(PS_ERR_ARG, "instance %d: n_pairs %d not in 1..4", idx, c.n_pairs);
  for (int p = 0; p < c.n_pairs; ++p) {
    if (c.pair_x[p] < 0 || c.pair_x[p] >= c.n_streams || c.pair_y[p] < 0 || c.pair_y[p] >= c.n_streams)
      return fail(PS_ERR_ARG, "instance %d: pair %d (%d, %d) outside 0..%d", idx, p, c.pair_x[p], c.pair_y[p],
                  c.n_streams - 1);
  }
  if (c.bits != 2 && c.bits != 4 && c.bits != 8 && c.bits != 32)
    return fail(PS_ERR_ARG, "instance %d: bits %d not in {2, 4, 8, 32}", idx, c.bits);
  const int m = ilog2_exact(c.fft_len);
  if (m < 0) return fail(PS_ERR_ARG, "instance %d: fft_len %lld is not a power of two", idx, (long long)c.fft_len);
  if (m < 8 || m > 22)
    return fail(PS_ERR_UNSUPPORTED, "instance %d: fft_len 2^%d outside the supported 2^8 .. 2^22", idx, m);
  if (c.window != PS_WIN_RECT && c.window != PS_WIN_HANN && c.window != PS_WIN_TAPS && c.window != PS_WIN_HAMMING &&
      c.window != PS_WIN_BLACKMAN)
    return fail(PS_ERR_ARG, "instance %d: unknown window %d", idx, c.window);
  if (c.hop != 0 && c.hop != c.fft_len && c.hop != c.fft_len / 2 && c.hop != c.fft_len / 4 && c.hop != c.fft_len / 8)
    return fail(PS_ERR_ARG, "instance %d: hop %lld is not 0, fft_len, fft_len/2, /4 or /8", idx, (long long)c.hop);
  if (c.window == PS_WIN_TAPS && (c.n_taps < 2 || c.n_taps > 4096))
    return fail(PS_ERR_ARG, "instance %d: n_taps %d not in 2..4096", idx, c.n_taps);
  if (c.precision != PS_PREC_FP32 && c.precision != PS_PREC_FP16 && c.precision != PS_PREC_BF16)
    return fail(PS_ERR_ARG, "instance %d: unknown precision %d", idx, c.precision);
  if (c.accum != PS_ACC_FP64 && c.accum != PS_ACC_KAHAN32)
    return fail(PS_ERR_ARG, "instance %d: unknown accumulator %d", idx, c.accum);
  if (c.precision == PS_PREC_FP32 && c.accum != PS_ACC_FP64)
    return fail(PS_ERR_UNSUPPORTED, "instance %d: FP32 passes accumulate in FP64 only", idx);
  if (c.precision != PS_PREC_FP32) {
    if (m < 16 || m > 18)
      return fail(PS_ERR_UNSUPPORTED, "instance %d: 16-bit passes are built for fft_len 2^16 .. 2^18, not 2^%d", idx, m);
    if (c.window == PS_WIN_TAPS)
      return fail(PS_ERR_UNSUPPORTED, "instance %d: the learnable window runs with FP32 passes only", idx);
  }
  if (c.chunk_frames < 0 || c.chunk_frames > 65536)
    return fail(PS_ERR_ARG, "instance %d: chunk_frames %d not in 0..65536", idx, c.chunk_frames);
  return PS_OK;
}

// x rounded to nearest even in a binary format with p significand bits and minimum normal exponent emin
// (subnormals below it), evaluated exactly in FP64.
double round_to_format(double x, int p, int emin) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e = 0;
  (void)std::frexp(x, &e);  // |x| = f 2^e, f in [0.5, 1): unit in the last place 2^(e - p)
  int q = e - p;
  if (e - 1 < emin) q = emin - p + 1;
  return std::ldexp(std::nearbyint(std::ldexp(x, -q)), q);
}

// bit pattern of a value already representable in the format
uint16_t format_bits(double v, int prec) {
  if (prec == PS_PREC_BF16) {
    const float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
  }
  if (v == 0.0) return std::signbit(v) ? 0x8000 : 0;
  const uint16_t sign = v < 0 ? 0x8000 : 0;
  const double a = std::fabs(v);
  int e = 0;
  const double f = std::frexp(a, &e);  // a = f 2^e
  if (e - 1 >= -14) {
    const uint32_t mant = (uint32_t)std::ldexp(2.0 * f - 1.0, 10);
    return (uint16_t)(sign | (uint32_t)(e - 1 + 15) << 10 | mant);
  }
  return (uint16_t)(sign | (uint32_t)std::ldexp(a, 24));  // subnormal: multiples of 2^-24
}

// DFT matrix of radix r (outputs q, inputs c: W_r^(q c)) as a 2r x 2r real block in the A-operand lane
// layout of the 16x16x32 matrix instructions, split as hi + lo in the 16-bit format:
//   [hl][tile t = 2*qb + part][K-step s][lane l][word jj], lane l = 16 g + i:
//   output q = 16 qb + i (real part for part 0, imaginary for 1);
//   word jj holds the coefficients of input c = 16 s + 4 g + jj: real input in the low half, imaginary high.
// Re Y = cos * xr + sin * xi, Im Y = -sin * xr + cos * xi with the angle 2 pi q c / r.
void dft_matrix(std::vector<uint32_t>& out, int r, int prec) {
  const int NT = 2 * r / 16, NS = r / 16;
  const int p = prec == PS_PREC_BF16 ? 8 : 11, emin = prec == PS_PREC_BF16 ? -126 : -14;
  out.assign((size_t)2 * NT * NS * 64 * 4, 0u);
  for (int hl = 0; hl < 2; ++hl)
    for (int t = 0; t < NT; ++t)
      for (int s = 0; s < NS; ++s)
        for (int l = 0; l < 64; ++l)
          for (int jj = 0; jj < 4; ++jj) {
            const int q = 16 * (t / 2) + l % 16, part = t % 2, c = 16 * s + 4 * (l / 16) + jj;
            const double a = kTwoPi * (double)((q * c) % r) / (double)r;
            const double cs = std::cos(a), sn = std::sin(a);
            const double v[2] = {part == 0 ? cs : -sn, part == 0 ? sn : cs};  // coefficient of xr, xi
            uint32_t word = 0;
            for (int k = 0; k < 2; ++k) {
              const double hi = round_to_format(v[k], p, emin);
              const double val = hl == 0 ? hi : round_to_format(v[k] - hi, p, emin);
              word |= (uint32_t)format_bits(val, prec) << (16 * k);
            }
            out[((((size_t)hl * NT + t) * NS + s) * 64 + l) * 4 + jj] = word;
          }
}

// W_len^m / 16 for m < len (stage twiddle of a 16 x R split, with the scale of the radix-16 stage)
void stage_twiddles(std::vector<float>& out, int64_t len) {
  out.resize(2 * (size_t)len);
  for (int64_t m = 0; m < len; ++m) {
    const double a = kTwoPi * (double)m / (double)len;
    out[2 * m] = (float)(std::cos(a) / 16.0);
    out[2 * m + 1] = (float)(-std::sin(a) / 16.0);
  }
}

void build_tables(Inst& I) {
  if (I.mx()) {
    dft_matrix(I.mx16, 16, I.cfg.precision);
    if (I.N1 == 512 || I.N2 == 512) dft_matrix(I.mx32, 32, I.cfg.precision);
    stage_twiddles(I.tws_col, I.N1);
    stage_twiddles(I.tws_row, I.N2);
  }
  if (I.fused) twiddle_table(I.tw_full, I.N, I.N);  // W_N^m, m < N
  twiddle_table(I.tw_col, I.N1, I.N1);
  twiddle_table(I.tw_row, I.N2, I.N2);
  twiddle_table(I.tw_lo, I.N, I.N2);  // W_N^m, m < N2; W_N^(q*N2) = W_N1^q reuses tw_col
  I.win.clear();
  double s = 0.0;
  if (I.cfg.window == PS_WIN_HANN || I.cfg.window == PS_WIN_HAMMING || I.cfg.window == PS_WIN_BLACKMAN) {
    // periodic cosine-sum windows a0 - a1 cos(2 pi n/N) + a2 cos(4 pi n/N), evaluated in FP64
    double a0 = 0.5, a1 = 0.5, a2 = 0.0;
    if (I.cfg.window == PS_WIN_HAMMING) a0 = 0.54, a1 = 0.46;
    if (I.cfg.window == PS_WIN_BLACKMAN) a0 = 0.42, a1 = 0.5, a2 = 0.08;
    I.win.resize((size_t)I.N);
    for (int64_t n = 0; n < I.N; ++n) {
      const double ph = kTwoPi * (double)n / (double)I.N;
      const double w = a0 - a1 * std::cos(ph) + a2 * std::cos(2.0 * ph);
      I.win[(size_t)n] = (float)w;
      s += w * w;
    }
  } else if (I.cfg.window == PS_WIN_TAPS) {
    I.win.assign((size_t)I.N, 1.0f);  // all control points 1 until set
    s = (double)I.N;
  } else {
    s = (double)I.N;
    if (I.fused) I.win.assign((size_t)I.N, 1.0f);  // the single pass always reads a window table
  }
  I.sumw2 = s;
}

ps_status check_plan(ps_plan_t plan, bool need_bound) {
  if (!plan) return fail(PS_ERR_ARG, "null plan");
  if (need_bound && !plan->bound) return fail(PS_ERR_STATE, "plan is not bound to a workspace (call ps_bind)");
  return PS_OK;
}

ps_status check_inst(ps_plan_t plan, int32_t i) {
  if (i < 0 || i >= (int32_t)plan->inst.size())
    return fail(PS_ERR_ARG, "instance %d outside 0..%d", i, (int)plan->inst.size() - 1);
  return PS_OK;
}

template <class T>
T* ws_ptr(ps_plan_t plan, size_t off) {
  return reinterpret_cast<T*>(plan->ws + off);
}

constexpr size_t kMaxTimed = 16384;
constexpr size_t kMaxRounds = 8;  // chunks per call handled by the grouped launches
constexpr int64_t kBatchT = int64_t(128) << 20;  // inter-pass bytes per grouped sub-batch (cache-sized)

// Launch f(launch) on the plan's stream; while profiling, the dispatch stamps a pair of events with the
// kernel's own start and end.
template <class F>
hipError_t timed(ps_plan_t plan, int kind, F&& f) {
  if (!plan->prof || plan->ev_used >= plan->ev_kind.size()) return f(ps::Launch{plan->stream, nullptr, nullptr});
  const ps::Launch l{plan->stream, plan->ev[2 * plan->ev_used], plan->ev[2 * plan->ev_used + 1]};
  hipError_t e = f(l);
  if (e != hipSuccess) return e;
  plan->ev_kind[plan->ev_used++] = kind;
  return hipSuccess;
}

ps_status upload(ps_plan_t plan, size_t off, const void* src, size_t bytes) {
  if (!bytes) return PS_OK;
  hipError_t e = hipMemcpyAsync(plan->ws + off, src, bytes, hipMemcpyHostToDevice, plan->stream);
  if (e != hipSuccess) return hip_fail(e, "table upload");
  return PS_OK;
}

// Default split N = N1 x N2 (log2 N1) of the four-step passes: N1 = 2^floor(m/2), except where timing on the
// device favours another.  Default FP32 schedules of the four-step passes, from whole-integration timings on
// the device (2^25 samples per stream and integration, int8 and 2-bit): 2^13 .. 2^17 run with the longer
// column pass first and 2 or 4 column-pass workgroups per CU; 2^19 as 512 x 1024 for 8-bit and wider codes
// (the 1024-point rows held 16 points per lane; 455 against 418 Gsamples/s as 1024 x 512, whose 8-column
// blocks of 1024-point columns read byte-sized input slowly) and 1024 x 512 for 2- and 4-bit codes; 2^20 as
// 512 x 2048.
int default_log2_n1(const ps_instance& c) {
  const int m = ilog2_exact(c.fft_len);
  if (c.precision != PS_PREC_FP32) return m / 2;
  switch (m) {
    case 13: return 7;
    case 14: return 8;
    case 15: return 7;
    case 16: return 8;
    case 17: return 9;
    case 19: return c.bits >= 8 ? 9 : 10;
    case 20: return 9;
    default: return m / 2;
  }
}

int default_col_wgs(const ps_instance& c) {
  const int m = ilog2_exact(c.fft_len);
  if (c.precision != PS_PREC_FP32) return 1;
  if (m == 13) return 4;
  return (m >= 14 && m <= 16) ? 2 : 1;
}

// the single pass runs FP32 transforms of 2^8 .. 2^12 points
bool fused_eligible(const ps_instance& c) {
  const int m = ilog2_exact(c.fft_len);
  return c.precision == PS_PREC_FP32 && m >= ps::kFusedMinLog2 && m <= ps::kFusedMaxLog2;
}

bool uses_fused(const ps_instance& c, const ps_schedule* s) {
  if (!fused_eligible(c)) return false;
  return !s || s->single_pass != 2;
}

// N/8-thread workgroups, one per slot and pair: about 2^20 / N of them (some 2000 waves, each then walking
// twice as many frames as with 2^21 / N, which measured 7-17 % slower at 2^10 .. 2^12), and the slots hold
// 16 MiB whatever N is
int default_slots_fused(const ps_instance& c) {
  const int64_t target = (int64_t(1) << 20) / c.fft_len;
  int G = 1;
  while (2 * G * c.n_pairs <= target && 2 * G <= 8192) G *= 2;
  return G;
}

// Accumulator slots: enough row-pass frame groups that units x pairs x slots reach about 512 workgroups for
// frames of at most 2^18 points and 256 beyond (twice the slots measured faster up to 2^18), and 1 for the
// 16-bit passes, whose row pass spreads frames over its waves.
int rowpass_tiles(const ps_instance& c, int N1, int N2) {
  return N1 / 2 / ps::rowpass_units_per_tile(N2) * c.n_pairs;
}

int default_slots(const ps_instance& c, int N1, int N2) {
  if (c.precision != PS_PREC_FP32) return 1;
  const int tiles = rowpass_tiles(c, N1, N2);
  const int target = c.fft_len <= (1 << 18) ? 512 : 256;
  int G = 1;
  while (G < 64 && G * tiles < target) G *= 2;
  return G;
}

// Row-pass frames per batch: 512-point rows in batches of 4 (512-thread workgroups, two per CU) once there
// are at least 512 row-pass workgroups (2^18, one pair: 73.0 vs 74.7 us per integration, where batches of 4
// with half the workgroups, or of 8 with twice the slots, were slower; 2^19: 6 % faster).
int default_rowpass_frames(const ps_instance& c, int N1, int N2, int G) {
  if (c.precision == PS_PREC_FP32 && N2 == 512 && rowpass_tiles(c, N1, N2) * G >= 512) return 4;
  return ps::rowpass_frames(N2);
}

// Why a schedule cannot run an instance (nullptr when it can).  why: optional message buffer (160 bytes).
const char* schedule_error(const ps_instance& c, const ps_schedule& s, char* why) {
  static thread_local char buf[160];
  char* w = why ? why : buf;
  const int m = ilog2_exact(c.fft_len);
  const int m1 = s.log2_n1 ? s.log2_n1 : default_log2_n1(c), m2 = m - m1;
  if (s.single_pass < 0 || s.single_pass > 2) {
    snprintf(w, 160, "single_pass %d not in 0..2", s.single_pass);
    return w;
  }
  if (s.single_pass == 1 && !fused_eligible(c)) {
    snprintf(w, 160, "the single pass runs FP32 transforms of 2^%d .. 2^%d points", ps::kFusedMinLog2,
             ps::kFusedMaxLog2);
    return w;
  }
  if (uses_fused(c, &s)) {
    if (s.colpass_cols || s.rowpass_frames || s.col_wg_per_cu) {
      snprintf(w, 160, "a single pass takes only log2_n1 and rowpass_slots");
      return w;
    }
    if (m1 < 4 || m2 < 4) {
      snprintf(w, 160, "split 2^%d x 2^%d: both factors at least 2^4", m1, m2);
      return w;
    }
    if (s.rowpass_slots < 0 || s.rowpass_slots > 8192 || (s.rowpass_slots & (s.rowpass_slots - 1))) {
      snprintf(w, 160, "rowpass_slots %d is not a power of two in 1..8192", s.rowpass_slots);
      return w;
    }
    return nullptr;
  }
  if (c.precision != PS_PREC_FP32) {
    if (m1 != m / 2 || s.colpass_cols || s.rowpass_frames || s.col_wg_per_cu > 1 || s.rowpass_slots > 1) {
      snprintf(w, 160, "16-bit passes run with the default schedule only");
      return w;
    }
    return nullptr;
  }
  if (m1 < 4 || m1 > 11 || m2 < 4 || m2 > 11) {
    snprintf(w, 160, "split 2^%d x 2^%d outside 2^4 .. 2^11 per pass", m1, m2);
    return w;
  }
  if (c.window == PS_WIN_TAPS && (m2 > 9 || m1 > 9)) {
    snprintf(w, 160, "the learnable window's backward needs both passes of at most 2^9 points");
    return w;
  }
  const int N1 = 1 << m1, N2 = 1 << m2;
  const int cols = s.colpass_cols ? s.colpass_cols : ps::colpass_cols(N1);
  const int fb = s.rowpass_frames ? s.rowpass_frames : ps::rowpass_frames(N2);
  if (!ps::colpass_has(N1, cols) || N2 % cols) {
    snprintf(w, 160, "no column pass of %d columns for N1 = %d", cols, N1);
    return w;
  }
  if (!ps::rowpass_has(N2, fb)) {
    snprintf(w, 160, "no row pass of %d frames per batch for N2 = %d", fb, N2);
    return w;
  }
  if (s.col_wg_per_cu < 0 || s.col_wg_per_cu > 8) {
    snprintf(w, 160, "col_wg_per_cu %d not in 0..8", s.col_wg_per_cu);
    return w;
  }
  if (s.rowpass_slots < 0 || s.rowpass_slots > 64 || (s.rowpass_slots & (s.rowpass_slots - 1))) {
    snprintf(w, 160, "rowpass_slots %d is not a power of two in 1..64", s.rowpass_slots);
    return w;
  }
  return nullptr;
}

// Column-pass arguments of frames f0 .. f0+nf-1 of instance I.  groups: frame groups of the tile grid (0:
// as many as make the tiles about one per CU).  *mode: the column-pass loader mode of this launch.
ps::ColArgs col_args(ps_plan_t plan, const Inst& I, const uint8_t* base, int64_t f0, int nf, int64_t groups,
                     int* mode) {
  ps::ColArgs ca{};
  ca.in = base + f0 * I.hop * I.bits_per_sample() / 8;
  const int64_t in_bytes = ((int64_t)(nf - 1) * I.hop + I.N) * I.bits_per_sample() / 8;
  ca.in_bytes = in_bytes < (int64_t(1) << 31) ? (uint32_t)in_bytes : 0u;
  *mode = in_bytes < (int64_t(1) << 31) && I.N * 8 < (int64_t(1) << 31) ? I.load_mode : 0;
  ca.N = I.N;
  ca.hop = I.hop;
  ca.hist_rows = (int32_t)(I.hop / I.N2);
  ca.N2 = (int32_t)I.N2;
  ca.S = I.cfg.n_streams;
  ca.P = I.cfg.n_pairs;
  for (int p = 0; p < 4; ++p) {
    ca.px[p] = I.cfg.pair_x[p];
    ca.py[p] = I.cfg.pair_y[p];
  }
  ca.n_colblk = (int32_t)(I.N2 / I.cols);
  ca.n_frames = nf;
  const int64_t per_frame = (int64_t)ca.n_colblk * ca.P;
  if (groups <= 0) groups = ((int64_t)I.col_wgs * plan->n_cu + per_frame / 2) / per_frame;
  if (groups < 1) groups = 1;
  if (groups > nf) groups = nf;
  ca.frames_per_block = (int32_t)((nf + groups - 1) / groups);
  ca.win = I.win.empty() ? nullptr : ws_ptr<float>(plan, I.off_win);
  ca.tw_col = ws_ptr<float2>(plan, I.off_tw_col);
  ca.tw_hi = ca.tw_col;
  ca.tw_lo = ws_ptr<float2>(plan, I.off_tw_lo);
  ca.lo_bits = I.m2;
  ca.T = ws_ptr<float2>(plan, I.off_T);
  ca.hist = I.hist_on ? ws_ptr<unsigned long long>(plan, I.off_hist) : nullptr;
  return ca;
}

int col_tiles(const ps::ColArgs& ca) {
  const int groups = (ca.n_frames + ca.frames_per_block - 1) / ca.frames_per_block;
  return groups * ca.P * ca.n_colblk;
}

// Row-pass arguments of nf frames following the F0 frames already in the integration.
ps::RowArgs row_args(ps_plan_t plan, const Inst& I, int nf, int64_t F0) {
  ps::RowArgs ra{};
  ra.T = ws_ptr<float2>(plan, I.off_T);
  ra.N1 = (int32_t)I.N1;
  ra.P = I.cfg.n_pairs;
  ra.n_frames = nf;
  ra.tw_row = ws_ptr<float2>(plan, I.off_tw_row);
  ra.acc = ws_ptr<double>(plan, I.off_acc);
  ra.G = I.G;
  ra.F0 = F0;
  ra.slot_stride = (int64_t)I.slot_doubles();
  return ra;
}

// Put a descriptor image into its device region, unless the region already holds exactly these bytes.
ps_status upload_desc(ps_plan_t plan, ps_plan_s::Desc& d, const std::vector<unsigned char>& bytes) {
  if (bytes == d.current) return PS_OK;
  if (bytes.size() > d.cap) return fail(PS_ERR_SIZE, "launch descriptors of %zu bytes exceed the %zu reserved", bytes.size(), d.cap);
  if (plan->capturing)
    return fail(PS_ERR_STATE, "launch descriptors changed during graph capture: make the same calls once before capturing");
  hipError_t e = hipSuccess;
  if (!d.host) {
    e = hipHostMalloc(reinterpret_cast<void**>(&d.host), d.cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      d.host = nullptr;
      return hip_fail(e, "pinned descriptor buffer");
    }
  }
  // an earlier copy out of the staging buffer may still be queued
  e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload wait");
  std::memcpy(d.host, bytes.data(), bytes.size());
  e = hipMemcpyAsync(plan->ws + d.off, d.host, bytes.size(), hipMemcpyHostToDevice, plan->stream);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  d.current = bytes;
  return PS_OK;
}

template <class T>
void append_bytes(std::vector<unsigned char>& v, const T* p, size_t n) {
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
  v.insert(v.end(), b, b + n * sizeof(T));
}

// Batching form: every FP32 instance of the call in one column-pass launch per (N1, format) and one row-pass
// launch per N2, per chunk round; each launch has one workgroup per tile of all its instances.
ps_status accumulate_grouped(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples,
                             std::vector<char>& done) {
  plan->t_inst = -1;
  int64_t rounds = 0;
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    const Inst& I = plan->inst[i];
    if (I.mx() || I.hist_on || I.fused) continue;
    const int64_t F = I.frames_in(n_samples[i]);
    rounds = std::max(rounds, (F + I.chunk - 1) / I.chunk);
  }
  if (rounds == 0 || rounds > (int64_t)kMaxRounds) return PS_OK;  // nothing to group, or too many chunks
  std::vector<ps::ColArgs> cols;
  std::vector<ps::RowArgs> rows;
  std::vector<int32_t> cend, rend;
  struct L1 {
    int kind, len, bits;
    int mode;  // column-pass loader mode
    int var;  // columns per workgroup (column pass) or frames per batch (row pass)
    size_t task0, n;
    int total;
  };
  std::vector<L1> launches;
  for (int64_t r = 0; r < rounds; ++r) {
    // Instances of one shape class (N1, N2, format, schedule) share a column-pass and a row-pass launch.
    // A class is cut into sub-batches whose inter-pass buffers total at most kBatchT bytes, and each
    // sub-batch's row pass follows its column pass directly, so the intermediate written by one is still in
    // the last-level cache when the other reads it.
    struct Member {
      ps::ColArgs ca;
      ps::RowArgs ra;
      int64_t t_bytes;
    };
    std::vector<std::pair<std::vector<int>, std::vector<Member>>> classes;
    for (size_t i = 0; i < plan->inst.size(); ++i) {
      const Inst& I = plan->inst[i];
      if (I.mx() || I.hist_on || I.fused) continue;
      const int64_t F = I.frames_in(n_samples[i]), f0 = r * I.chunk;
      if (f0 >= F) continue;
      const int nf = (int)std::min<int64_t>(I.chunk, F - f0);
      int mode = 0;
      // the instance's own frame grouping: long transforms keep long frame groups per tile
      const ps::ColArgs ca = col_args(plan, I, static_cast<const uint8_t*>(packed_dev[i]), f0, nf, 0, &mode);
      const ps::RowArgs ra = row_args(plan, I, nf, I.n_frames + f0);
      const std::vector<int> key = {(int)I.N1, (int)I.N2, I.cfg.bits, mode, I.cols, I.fb};
      auto it = std::find_if(classes.begin(), classes.end(), [&](const auto& c) { return c.first == key; });
      if (it == classes.end()) {
        classes.push_back({key, {}});
        it = classes.end() - 1;
      }
      it->second.push_back(Member{ca, ra, (int64_t)nf * I.cfg.n_pairs * I.N * 8});
    }
    for (const auto& c : classes) {
      const std::vector<int>& key = c.first;
      size_t m = 0;
      while (m < c.second.size()) {
        size_t e = m;
        int64_t bytes = 0;
        while (e < c.second.size() && (e == m || bytes + c.second[e].t_bytes <= kBatchT)) bytes += c.second[e++].t_bytes;
        L1 lc{0, key[0], key[2], key[3], key[4], cols.size(), e - m, 0};
        L1 lr{1, key[1], 0, 0, key[5], rows.size(), e - m, 0};
        int ct = 0, rt = 0;
        size_t t_off = 0;  // the sub-batch's members take consecutive regions of the shared inter-pass buffer
        for (size_t q = m; q < e; ++q) {
          ps::ColArgs ca = c.second[q].ca;
          ps::RowArgs ra = c.second[q].ra;
          ca.T = reinterpret_cast<float2*>(plan->ws + plan->off_T + t_off);
          ra.T = ca.T;
          t_off += (size_t)c.second[q].t_bytes;
          if (t_off > plan->t_bytes) return fail(PS_ERR_STATE, "grouped sub-batch exceeds the inter-pass buffer");
          cols.push_back(ca);
          ct += col_tiles(ca);
          cend.push_back(ct);
          rows.push_back(ra);
          rt += ra.N1 / 2 / ps::rowpass_units_per_tile(key[1]) * ra.P * ra.G;
          rend.push_back(rt);
        }
        lc.total = ct;
        lr.total = rt;
        launches.push_back(lc);
        launches.push_back(lr);
        m = e;
      }
    }
  }
  std::vector<unsigned char> img;
  append_bytes(img, cols.data(), cols.size());
  const size_t rows_at = img.size();
  append_bytes(img, rows.data(), rows.size());
  const size_t cend_at = img.size();
  append_bytes(img, cend.data(), cend.size());
  const size_t rend_at = img.size();
  append_bytes(img, rend.data(), rend.size());
  ps_status st = upload_desc(plan, plan->acc_desc, img);
  if (st != PS_OK) return st;
  char* dev = plan->ws + plan->acc_desc.off;
  for (const L1& l : launches) {
    ps::BatchArgs b{};
    b.n_tasks = (int32_t)l.n;
    b.total = l.total;
    hipError_t e;
    if (l.kind == 0) {
      b.tasks = dev + l.task0 * sizeof(ps::ColArgs);
      b.tile_end = reinterpret_cast<const int32_t*>(dev + cend_at) + l.task0;
      e = timed(plan, PS_KERNEL_COLPASS, [&](const ps::Launch& x) { return ps::launch_colpass_batch(l.len, l.var, l.bits, l.mode, b, x); });
    } else {
      b.tasks = dev + rows_at + l.task0 * sizeof(ps::RowArgs);
      b.tile_end = reinterpret_cast<const int32_t*>(dev + rend_at) + l.task0;
      e = timed(plan, PS_KERNEL_ROWPASS, [&](const ps::Launch& x) { return ps::launch_rowpass_batch(l.len, l.var, b, x); });
    }
    if (e != hipSuccess) return hip_fail(e, "grouped pass launch");
  }
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    Inst& I = plan->inst[i];
    if (I.mx() || I.hist_on || I.fused) continue;
    done[i] = 1;
    const int64_t F = I.frames_in(n_samples[i]);
    if (F > 0) {
      I.first = false;
      I.n_frames += F;
    }
  }
  return PS_OK;
}

// Precision form of one chunk: 16-bit column pass (16 columns per workgroup, about two workgroups per CU) and
// 16-bit row pass with FP64 or compensated FP32 sums (one workgroup per unit and pair).
ps_status accumulate_mx(ps_plan_t plan, Inst& I, const ps::ColArgs& ca) {
  plan->t_inst = -1;
  ps::MxColArgs m{};
  m.col = ca;
  m.col.n_colblk = (int32_t)(I.N2 / 16);
  const ps_instance& c = I.cfg;
  m.mode = 0;
  if (c.bits == 8 && c.n_streams == 2 && c.n_pairs == 1 && c.pair_x[0] == 0 && c.pair_y[0] == 1) m.mode = 1;
  if (c.bits == 8 && c.n_streams == 4) m.mode = 2;
  // four streams as the pairs (0, 2) and (1, 3): one workgroup transforms both from the words it reads
  if (m.mode == 2 && c.n_pairs == 2 && c.pair_x[0] == 0 && c.pair_y[0] == 2 && c.pair_x[1] == 1 && c.pair_y[1] == 3)
    m.mode = 3;
  if (ca.in_bytes == 0) m.mode = 0;  // the word paths address the launch's input with 32-bit offsets
  const int64_t per_frame = (int64_t)m.col.n_colblk * (m.mode == 3 ? 1 : ca.P);
  // two or three workgroups fit on a CU: aim at two per CU, each looping over a group of frames
  int64_t groups = (2 * plan->n_cu + per_frame / 2) / per_frame;
  if (groups < 1) groups = 1;
  if (groups > ca.n_frames) groups = ca.n_frames;
  m.col.frames_per_block = (int32_t)((ca.n_frames + groups - 1) / groups);
  groups = (ca.n_frames + m.col.frames_per_block - 1) / m.col.frames_per_block;
  m.m.a16 = ws_ptr<uint32_t>(plan, I.off_mx16);
  m.m.aR = ws_ptr<uint32_t>(plan, I.N1 == 512 ? I.off_mx32 : I.off_mx16);
  m.m.tws = ws_ptr<float2>(plan, I.off_tws_col);
  m.T = ws_ptr<uint32_t>(plan, I.off_T);
  const int n_blocks = (int)(groups * per_frame);
  hipError_t e = timed(plan, PS_KERNEL_COLPASS, [&](const ps::Launch& l) {
    return ps::launch_colpass_mx((int)I.N1, c.precision, c.bits, m, n_blocks, l);
  });
  if (e != hipSuccess) return hip_fail(e, "16-bit column pass launch");
  ps::MxRowArgs r{};
  r.T = m.T;
  r.N1 = (int32_t)I.N1;
  r.P = c.n_pairs;
  r.n_frames = ca.n_frames;
  r.m.a16 = m.m.a16;
  r.m.aR = ws_ptr<uint32_t>(plan, I.N2 == 512 ? I.off_mx32 : I.off_mx16);
  r.m.tws = ws_ptr<float2>(plan, I.off_tws_row);
  r.acc = ws_ptr<double>(plan, I.off_acc);
  r.first = I.first ? 1 : 0;
  // the stages scale Z by 1 / (16 * (N1 / 16) * 16) = 1 / (16 N1); products by its square
  r.unscale = std::ldexp(1.0, 2 * (4 + I.m1));
  e = timed(plan, PS_KERNEL_ROWPASS, [&](const ps::Launch& l) {
    return ps::launch_rowpass_mx((int)I.N2, c.precision, c.accum, r, l);
  });
  if (e != hipSuccess) return hip_fail(e, "16-bit row pass launch");
  return PS_OK;
}

// Arguments of the Stokes output of instance I over its first n_frames frames (Eq. 2 with cal, or unit
// gains, no leakage and psi = 0 when cal is null).
ps::OutArgs stokes_args(ps_plan_t plan, const Inst& I, int64_t n_frames, const ps_cal* cal, float* iquv) {
  ps::OutArgs o{};
  const bool reduced = std::min<int64_t>(I.G, n_frames) > ps::kDirectSlots;
  o.acc = ws_ptr<double>(plan, reduced ? I.off_sumacc : I.off_acc);
  o.slots = reduced ? 1 : (int32_t)std::min<int64_t>(I.G, n_frames);
  o.slot_stride = (int64_t)I.slot_doubles();
  o.N1 = (int32_t)I.N1;
  o.N2 = (int32_t)I.N2;
  o.P = I.cfg.n_pairs;
  o.C = I.C;
  o.n_frames = (double)n_frames;
  o.sumw2_dev = ws_ptr<double>(plan, I.off_sumw2);
  o.scale = 1.0 / ((double)n_frames * I.sumw2);
  const double psi = cal ? cal->psi : 0.0;
  o.cos2psi = std::cos(2.0 * psi);
  o.sin2psi = std::sin(2.0 * psi);
  o.circular = (cal && cal->feed == PS_FEED_CIRCULAR) ? 1 : 0;
  if (cal) {
    o.gain_x = cal->gain_x;
    o.gain_y = cal->gain_y;
    o.dterms = cal->dterms;
  }
  o.iquv = iquv;
  return o;
}

// Frames 0 .. F-1 of the buffer at base (frame f at sample f * hop) in chunks of the instance's chunk size:
// the column and row passes (or their 16-bit forms) of each chunk, frames in order.  With fuse and a
// pending accumulate-and-Stokes request that the instance can take (one accumulator slot, FP32 four-step
// passes), the last chunk's row pass also writes the Stokes spectra.
ps_status run_frames(ps_plan_t plan, Inst& I, const uint8_t* base, int64_t F, bool fuse = false) {
  plan->t_inst = -1;
  if (I.fused && !I.hist_on) {
    // single pass: no inter-pass buffer, so one launch takes up to 2^28 frames
    constexpr int64_t kMaxFused = int64_t(1) << 28;
    for (int64_t f0 = 0; f0 < F; f0 += kMaxFused) {
      const int nf = (int)std::min<int64_t>(kMaxFused, F - f0);
      ps::FusedArgs fa{};
      fa.in = base + f0 * I.hop * I.bits_per_sample() / 8;
      fa.hop = I.hop;
      fa.S = I.cfg.n_streams;
      fa.P = I.cfg.n_pairs;
      for (int p = 0; p < 4; ++p) {
        fa.px[p] = I.cfg.pair_x[p];
        fa.py[p] = I.cfg.pair_y[p];
      }
      fa.n_frames = nf;
      fa.win = ws_ptr<float>(plan, I.off_win);  // a table of ones for the rectangular window
      fa.tw = ws_ptr<float2>(plan, I.off_tw_full);
      fa.acc = ws_ptr<double>(plan, I.off_acc);
      fa.G = I.G;
      fa.N1 = (int32_t)I.N1;
      fa.N2 = (int32_t)I.N2;
      fa.F0 = I.n_frames;
      fa.slot_stride = (int64_t)I.slot_doubles();
      hipError_t e = timed(plan, PS_KERNEL_COLPASS, [&](const ps::Launch& l) { return ps::launch_fused((int)I.N, I.cfg.bits, fa, l); });
      if (e != hipSuccess) return hip_fail(e, "single-pass launch");
      I.first = false;
      I.n_frames += nf;
    }
    return PS_OK;
  }
  for (int64_t f0 = 0; f0 < F; f0 += I.chunk) {
    const int nf = (int)((F - f0) < I.chunk ? (F - f0) : I.chunk);
    int mode = 0;
    // one workgroup per CU: each loops over a group of frames, so that groups x pairs x blocks ~ CUs
    const ps::ColArgs ca = col_args(plan, I, base, f0, nf, 0, &mode);
    if (I.mx()) {
      ps_status ms = accumulate_mx(plan, I, ca);
      if (ms != PS_OK) return ms;
      I.first = false;
      I.n_frames += nf;
      continue;
    }
    hipError_t e = timed(plan, PS_KERNEL_COLPASS,
                         [&](const ps::Launch& l) { return ps::launch_colpass((int)I.N1, I.cols, I.cfg.bits, mode, ca, l); });
    if (e != hipSuccess) return hip_fail(e, "column pass launch");
    if (!plan->capturing && I.n_frames == 0 && f0 == 0 && nf == F) {  // the whole integration in one launch
      plan->t_inst = (int)(&I - plan->inst.data());
      plan->t_gen = I.gen;
    }
    const ps::RowArgs ra = row_args(plan, I, nf, I.n_frames);
    const bool fuse_now = fuse && I.fuse_iquv && I.can_fuse() && f0 + nf == F;
    ps::OutArgs o{};
    if (fuse_now) o = stokes_args(plan, I, I.n_frames + nf, I.fuse_cal, I.fuse_iquv);
    e = timed(plan, PS_KERNEL_ROWPASS, [&](const ps::Launch& l) {
      return ps::launch_rowpass((int)I.N2, I.fb, ra, l, fuse_now ? &o : nullptr);
    });
    if (e != hipSuccess) return hip_fail(e, "row pass launch");
    if (fuse_now) I.fuse_done = true;
    I.first = false;
    I.n_frames += nf;
  }
  return PS_OK;
}

// Overlapped segmentation across calls (T samples in this one).  The previous call's last N - hop samples
// wait in the first half of the staging buffer; this call's first N - hop samples are copied behind them,
// and the (N - hop) / hop frames that start in the waiting samples are transformed from there.  Then this
// call's last N - hop samples take the first half.  Stream order keeps the copies and passes apart.
ps_status overlap_frames(ps_plan_t plan, Inst& I, const uint8_t* base, int64_t T) {
  uint8_t* stage = ws_ptr<uint8_t>(plan, I.off_stage);
  const size_t half = I.tail_bytes();
  if (I.n_frames > 0) {
    hipError_t e = ps::launch_copy(base, stage + half, half, plan->stream);
    if (e != hipSuccess) return hip_fail(e, "overlap staging copy");
    ps_status st = run_frames(plan, I, stage, (I.N - I.hop) / I.hop);
    if (st != PS_OK) return st;
  }
  const size_t call_bytes = (size_t)(T * I.bits_per_sample() / 8);
  hipError_t e = ps::launch_copy(base + call_bytes - half, stage, half, plan->stream);
  if (e != hipSuccess) return hip_fail(e, "overlap tail copy");
  return PS_OK;
}

}  // namespace

extern "C" {

ps_status ps_plan(const ps_instance* inst, int32_t n_inst, ps_plan_t* out, size_t* workspace_bytes) {
  return ps_plan_scheduled(inst, nullptr, n_inst, out, workspace_bytes);
}

ps_status ps_schedule_candidates(const ps_instance* inst, ps_schedule* out, int32_t capacity, int32_t* count) {
  if (!inst || !count) return fail(PS_ERR_ARG, "null argument to ps_schedule_candidates");
  ps_status st = validate_instance(*inst, 0);
  if (st != PS_OK) return st;
  std::vector<ps_schedule> v;
  const int m = ilog2_exact(inst->fft_len);
  if (inst->precision != PS_PREC_FP32) {
    v.push_back(ps_schedule{m / 2, 0, 0, 0, 1, 0});
  } else {
    if (fused_eligible(*inst)) {
      const int G0 = default_slots_fused(*inst);
      for (int G = std::max(1, G0 / 4); G <= std::min(8192, 2 * G0); G *= 2) v.push_back(ps_schedule{m / 2, 0, 0, 0, G, 1});
    }
    for (int m1 = m / 2 - 1; m1 <= m / 2 + 1; ++m1) {
      const int N1 = 1 << m1, N2 = 1 << (m - m1);
      if (m1 < 4 || m - m1 < 4 || m1 > 11 || m - m1 > 11) continue;
      const int G0 = default_slots(*inst, N1, N2);
      for (int cols = 4; cols <= 16; cols *= 2)
        for (int fb = 2; fb <= 8; fb *= 2)
          for (int wg = 1; wg <= 4; wg *= 2)
            for (int G = std::max(1, G0 / 2); G <= std::min(64, 2 * G0); G *= 2) {
              const ps_schedule c{m1, cols, fb, wg, G, fused_eligible(*inst) ? 2 : 0};
              if (schedule_error(*inst, c, nullptr) == nullptr) v.push_back(c);
            }
    }
  }
  *count = (int32_t)v.size();
  if (out)
    for (int32_t i = 0; i < capacity && i < (int32_t)v.size(); ++i) out[i] = v[(size_t)i];
  return PS_OK;
}

ps_status ps_plan_scheduled(const ps_instance* inst, const ps_schedule* sched, int32_t n_inst, ps_plan_t* out,
                            size_t* workspace_bytes) {
  if (!inst || !out || !workspace_bytes) return fail(PS_ERR_ARG, "null argument to ps_plan");
  *out = nullptr;
  if (n_inst < 1 || n_inst > 4096) return fail(PS_ERR_ARG, "n_inst %d not in 1..4096", n_inst);
  for (int i = 0; i < n_inst; ++i) {
    ps_status st = validate_instance(inst[i], i);
    if (st != PS_OK) return st;
    if (sched) {
      char why[160];
      if (schedule_error(inst[i], sched[i], why)) return fail(PS_ERR_UNSUPPORTED, "instance %d: %s", i, why);
    }
  }
  ps_plan_s* plan = new (std::nothrow) ps_plan_s;
  if (!plan) return fail(PS_ERR_ARG, "out of host memory");
  size_t off = 0, t_pool = 0;
  plan->inst.resize((size_t)n_inst);
  for (int i = 0; i < n_inst; ++i) {
    Inst& I = plan->inst[(size_t)i];
    I.cfg = inst[i];
    I.N = inst[i].fft_len;
    I.m = ilog2_exact(I.N);
    I.m1 = (sched && sched[i].log2_n1) ? sched[i].log2_n1 : default_log2_n1(I.cfg);
    I.m2 = I.m - I.m1;
    I.N1 = int64_t(1) << I.m1;
    I.N2 = int64_t(1) << I.m2;
    I.C = I.N / 2;
    I.hop = inst[i].hop ? inst[i].hop : I.N;
    I.cols = (sched && sched[i].colpass_cols) ? sched[i].colpass_cols : ps::colpass_cols((int)I.N1);
    I.col_wgs = (sched && sched[i].col_wg_per_cu) ? sched[i].col_wg_per_cu : default_col_wgs(inst[i]);
    I.fused = uses_fused(I.cfg, sched ? &sched[i] : nullptr);
    I.G = (sched && sched[i].rowpass_slots) ? sched[i].rowpass_slots
                                             : (I.fused ? default_slots_fused(I.cfg) : default_slots(I.cfg, (int)I.N1, (int)I.N2));
    I.fb = (sched && sched[i].rowpass_frames) ? sched[i].rowpass_frames
                                              : default_rowpass_frames(I.cfg, (int)I.N1, (int)I.N2, (int)I.G);
    // a pass pair covers 2^25 points (a 256 MiB inter-pass buffer per pair, shared by the plan's instances),
    // at least 64 frames, so its fixed cost (first loads, last stores, setup) is spread over many frames:
    // 6-11 % faster than 2^24 points for 2^25-sample integrations of 2^13 .. 2^18-point frames
    I.chunk = inst[i].chunk_frames ? inst[i].chunk_frames : (int64_t)std::max<int64_t>(64, (int64_t(1) << 25) / I.N);
    // word loads of the column pass: 2-, 4- and 8-bit codes of two streams correlated as (0, 1), or of four
    // streams (any pairs)
    if (inst[i].bits <= 8 && inst[i].n_streams == 2 && inst[i].n_pairs == 1 && inst[i].pair_x[0] == 0 &&
        inst[i].pair_y[0] == 1)
      I.load_mode = 1;
    else if (inst[i].bits <= 8 && inst[i].n_streams == 4)
      I.load_mode = 2;
    build_tables(I);
    I.off_tw_col = off; off = align_up(off + (size_t)I.N1 * 8);
    I.off_tw_row = off; off = align_up(off + (size_t)I.N2 * 8);
    I.off_tw_lo = off; off = align_up(off + (size_t)I.N2 * 8);
    I.off_win = off; off = align_up(off + (I.win.empty() ? 0 : (size_t)I.N * 4));
    I.off_taps = off; off = align_up(off + (I.cfg.window == PS_WIN_TAPS ? (size_t)I.cfg.n_taps * 4 : 0));
    I.off_sumw2 = off; off = align_up(off + 8);
    if (I.mx()) {
      I.off_mx16 = off; off = align_up(off + I.mx16.size() * 4);
      I.off_mx32 = off; off = align_up(off + I.mx32.size() * 4);
      I.off_tws_col = off; off = align_up(off + I.tws_col.size() * 4);
      I.off_tws_row = off; off = align_up(off + I.tws_row.size() * 4);
    }
    I.off_hist = off; off = align_up(off + (size_t)I.cfg.n_pairs * 2 * (size_t)I.hist_bins() * 8);
    I.off_tw_full = off; off = align_up(off + I.tw_full.size() * 4);
    I.off_stage = off; off = align_up(off + 2 * I.tail_bytes());
    t_pool = std::max(t_pool, (size_t)I.chunk * (size_t)I.cfg.n_pairs * (size_t)I.N * 8);
    I.off_acc = off; off = align_up(off + I.acc_bytes());
    if (I.G > ps::kDirectSlots) {
      I.off_sumacc = off; off = align_up(off + I.slot_doubles() * 8);
      I.off_sumpart = off; off = align_up(off + (size_t)ps::slot_reduce_chunks(I.G) * I.slot_doubles() * 8);
    }
    const size_t P = (size_t)I.cfg.n_pairs;
    I.off_red = off; off = align_up(off + P * (size_t)ps::bw_parts((int)I.N1, (int)I.N2) * 5 * sizeof(double));
    I.off_norm = off; off = align_up(off + P * sizeof(double));
    if (I.taps()) {
      I.off_wpart = off; off = align_up(off + (size_t)ps::window_taps_blocks(I.N) * sizeof(double));
      I.off_ga = off; off = align_up(off + P * (size_t)I.C * 4 * sizeof(float));
      I.off_dw = off; off = align_up(off + (size_t)ps::kMaxBwGroups * (size_t)I.N * sizeof(double));
      I.off_tpart = off; off = align_up(off + (size_t)ps::bw_taps_part_doubles(I.N) * sizeof(double));
    }
    I.end = off;
  }
  // One inter-pass buffer for the whole plan: the passes of its instances run one after another on the
  // plan's stream, and a grouped sub-batch holds at most kBatchT bytes of inter-pass data (or a single
  // instance's chunk), so the largest chunk or kBatchT suffices (64 instances: 0.5 GB instead of 10 GB).
  if (n_inst > 1) t_pool = std::max(t_pool, (size_t)kBatchT);
  plan->off_T = off;
  plan->t_bytes = t_pool;
  off = align_up(off + t_pool);
  for (Inst& I : plan->inst) I.off_T = plan->off_T;
  // descriptors of the grouped launches: up to kMaxRounds chunks per call, one task per instance and pass
  {
    const size_t n = (size_t)n_inst;
    plan->acc_desc.cap = kMaxRounds * n * (sizeof(ps::ColArgs) + sizeof(ps::RowArgs) + 2 * sizeof(int32_t)) + 64;
    plan->acc_desc.off = off;
    off = align_up(off + plan->acc_desc.cap);
    plan->out_desc.cap = n * (sizeof(ps::OutArgs) + sizeof(int32_t)) + 64;
    plan->out_desc.off = off;
    off = align_up(off + plan->out_desc.cap);
  }
  plan->ws_bytes = off;
  *out = plan;
  *workspace_bytes = off;
  return PS_OK;
}

ps_status ps_bind(ps_plan_t plan, void* workspace_dev, size_t bytes, void* hip_stream) {
  plan->t_inst = -1;
  ps_status st = check_plan(plan, false);
  if (st != PS_OK) return st;
  if (!workspace_dev) return fail(PS_ERR_WORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign)
    return fail(PS_ERR_WORKSPACE, "workspace is not %zu-byte aligned", kAlign);
  if (bytes < plan->ws_bytes)
    return fail(PS_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu the plan needs", bytes,
                plan->ws_bytes);
  plan->ws = static_cast<char*>(workspace_dev);
  plan->stream = static_cast<hipStream_t>(hip_stream);
  plan->bound = false;
  {
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    plan->n_cu = ncu > 0 ? ncu : 256;
  }
  for (Inst& I : plan->inst) {
    if ((st = upload(plan, I.off_tw_col, I.tw_col.data(), I.tw_col.size() * 4)) != PS_OK) return st;
    if ((st = upload(plan, I.off_tw_row, I.tw_row.data(), I.tw_row.size() * 4)) != PS_OK) return st;
    if ((st = upload(plan, I.off_tw_lo, I.tw_lo.data(), I.tw_lo.size() * 4)) != PS_OK) return st;
    if ((st = upload(plan, I.off_win, I.win.data(), I.win.size() * 4)) != PS_OK) return st;
    if ((st = upload(plan, I.off_sumw2, &I.sumw2, 8)) != PS_OK) return st;
    if ((st = upload(plan, I.off_tw_full, I.tw_full.data(), I.tw_full.size() * 4)) != PS_OK) return st;
    if (I.mx()) {
      if ((st = upload(plan, I.off_mx16, I.mx16.data(), I.mx16.size() * 4)) != PS_OK) return st;
      if ((st = upload(plan, I.off_mx32, I.mx32.data(), I.mx32.size() * 4)) != PS_OK) return st;
      if ((st = upload(plan, I.off_tws_col, I.tws_col.data(), I.tws_col.size() * 4)) != PS_OK) return st;
      if ((st = upload(plan, I.off_tws_row, I.tws_row.data(), I.tws_row.size() * 4)) != PS_OK) return st;
    }
    if (I.taps()) {
      I.ones.assign((size_t)I.cfg.n_taps, 1.0f);
      if ((st = upload(plan, I.off_taps, I.ones.data(), I.ones.size() * 4)) != PS_OK) return st;
    }
    I.first = true;
    I.n_frames = 0;
    I.hist_zeroed = false;
    I.hist_frames = 0;
    plan->touch(I);
  }
  // the descriptor regions of the new workspace hold nothing yet (the cached images describe the old one,
  // and a new workspace at the same address still starts uninitialised)
  plan->acc_desc.current.clear();
  plan->out_desc.current.clear();
  hipError_t e = hipStreamSynchronize(plan->stream);
  if (e != hipSuccess) return hip_fail(e, "ps_bind synchronise");
  plan->bound = true;
  return PS_OK;
}

ps_status ps_set_window_taps(ps_plan_t plan, int32_t inst, const float* taps_dev) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  Inst& I = plan->inst[(size_t)inst];
  if (!I.taps()) return fail(PS_ERR_ARG, "instance %d does not use a PS_WIN_TAPS window", inst);
  if (!taps_dev) return fail(PS_ERR_ARG, "null taps");
  plan->touch(I);
  // the window kernel reads the caller's taps and keeps a copy in the workspace for the adjoint
  ps::WinArgs w{};
  w.taps = taps_dev;
  w.taps_copy = ws_ptr<float>(plan, I.off_taps);
  w.n_taps = I.cfg.n_taps;
  w.N = I.N;
  w.win = ws_ptr<float>(plan, I.off_win);
  w.partial = ws_ptr<double>(plan, I.off_wpart);
  hipError_t e = timed(plan, PS_KERNEL_OTHER, [&](const ps::Launch& l) {
    return ps::launch_window_taps(w, ps::window_taps_blocks(I.N), ws_ptr<double>(plan, I.off_sumw2), l);
  });
  if (e != hipSuccess) return hip_fail(e, "window launch");
  return PS_OK;
}

ps_status ps_reset(ps_plan_t plan) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  for (Inst& I : plan->inst) {
    I.first = true;
    I.n_frames = 0;
    I.hist_zeroed = false;
    I.hist_frames = 0;
    plan->touch(I);
  }
  return PS_OK;
}

static ps_status check_accumulate(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (!packed_dev || !n_samples) return fail(PS_ERR_ARG, "null packed or n_samples array");
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    const Inst& I = plan->inst[i];
    if (n_samples[i] < 0) return fail(PS_ERR_ARG, "instance %zu: negative sample count", i);
    if (n_samples[i] % I.N)
      return fail(PS_ERR_SIZE, "instance %zu: %lld samples is not a multiple of fft_len %lld", i,
                  (long long)n_samples[i], (long long)I.N);
    if (n_samples[i] > 0 && !packed_dev[i]) return fail(PS_ERR_ARG, "instance %zu: null packed buffer", i);
    if (n_samples[i] / I.N > (int64_t(1) << 40)) return fail(PS_ERR_SIZE, "instance %zu: too many frames", i);
  }
  return PS_OK;
}

// Frames of instance I in the integration once a call of T samples has been added.
static int64_t frames_after(const Inst& I, int64_t T) {
  if (T == 0) return I.n_frames;
  return I.n_frames + I.frames_in(T) + (I.overlap() && I.n_frames > 0 ? (I.N - I.hop) / I.hop : 0);
}

static ps_status accumulate_impl(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples) {
  ps_status st = PS_OK;
  for (size_t i = 0; i < plan->inst.size(); ++i)
    if (n_samples[i] > 0) plan->touch(plan->inst[i]);
  // First, per instance: the histogram clear and, with overlapped frames, the frames that span the
  // previous call and this one (they precede this call's own frames in the integration).
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    Inst& I = plan->inst[i];
    const int64_t T = n_samples[i];
    if (T == 0) continue;
    if (I.hist_on) {
      if (!I.hist_zeroed) {
        hipError_t e = ps::launch_zero_u64(ws_ptr<unsigned long long>(plan, I.off_hist),
                                           (int64_t)I.cfg.n_pairs * 2 * I.hist_bins(), plan->stream);
        if (e != hipSuccess) return hip_fail(e, "histogram clear");
        I.hist_zeroed = true;
      }
      I.hist_frames += I.frames_in(T) + (I.overlap() && I.n_frames > 0 ? (I.N - I.hop) / I.hop : 0);
    }
    if (I.overlap()) {
      st = overlap_frames(plan, I, static_cast<const uint8_t*>(packed_dev[i]), T);
      if (st != PS_OK) return st;
    }
  }
  std::vector<char> done(plan->inst.size(), 0);
  if (plan->inst.size() > 1) {
    st = accumulate_grouped(plan, packed_dev, n_samples, done);
    if (st != PS_OK) return st;
  }
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    if (done[i]) continue;
    Inst& I = plan->inst[i];
    st = run_frames(plan, I, static_cast<const uint8_t*>(packed_dev[i]), I.frames_in(n_samples[i]), true);
    if (st != PS_OK) return st;
  }
  return PS_OK;
}

ps_status ps_accumulate(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples) {
  ps_status st = check_accumulate(plan, packed_dev, n_samples);
  if (st != PS_OK) return st;
  return accumulate_impl(plan, packed_dev, n_samples);
}

ps_status ps_accumulate_stokes(ps_plan_t plan, const void* const* packed_dev, const int64_t* n_samples,
                               const ps_cal* cal, float* const* iquv_dev) {
  ps_status st = check_accumulate(plan, packed_dev, n_samples);
  if (st != PS_OK) return st;
  const size_t n = plan->inst.size();
  if (iquv_dev) {
    for (size_t i = 0; i < n; ++i) {
      if (!iquv_dev[i]) continue;
      if (cal && cal[i].feed != PS_FEED_LINEAR && cal[i].feed != PS_FEED_CIRCULAR)
        return fail(PS_ERR_ARG, "instance %zu: unknown feed %d", i, cal[i].feed);
      if (frames_after(plan->inst[i], n_samples[i]) == 0)
        return fail(PS_ERR_STATE, "instance %zu would have no accumulated frames", i);
    }
  }
  for (size_t i = 0; i < n; ++i) {
    Inst& I = plan->inst[i];
    I.fuse_iquv = iquv_dev ? iquv_dev[i] : nullptr;
    I.fuse_cal = cal ? &cal[i] : nullptr;
    I.fuse_done = false;
  }
  st = accumulate_impl(plan, packed_dev, n_samples);
  std::vector<float*> rest(n, nullptr);
  int n_rest = 0, last = -1;
  for (size_t i = 0; i < n; ++i) {
    Inst& I = plan->inst[i];
    if (I.fuse_iquv && !I.fuse_done) {
      rest[i] = I.fuse_iquv;
      ++n_rest;
      last = (int)i;
    }
    I.fuse_iquv = nullptr;
    I.fuse_cal = nullptr;
  }
  if (st != PS_OK || n_rest == 0) return st;
  // instances whose Stokes did not come out of their last row pass: one output launch (its arguments passed
  // directly when there is one instance, so that a loop over changing outputs can be captured), else one
  // grouped launch
  if (n_rest == 1) return ps_stokes(plan, last, cal ? &cal[last] : nullptr, rest[(size_t)last]);
  return ps_stokes_all(plan, cal, rest.data());
}

// Sum the slots of an instance that uses many of them into one (readers then see a single slot).
static ps_status reduce_slots(ps_plan_t plan, const Inst& I) {
  if (!I.use_reduced()) return PS_OK;
  hipError_t e = timed(plan, PS_KERNEL_OTHER, [&](const ps::Launch& l) {
    return ps::launch_slot_reduce(ws_ptr<double>(plan, I.off_acc), (int64_t)I.slot_doubles(), I.slots_used(),
                                  (int64_t)I.slot_doubles(), ws_ptr<double>(plan, I.off_sumpart),
                                  ws_ptr<double>(plan, I.off_sumacc), l);
  });
  if (e != hipSuccess) return hip_fail(e, "slot reduction launch");
  return PS_OK;
}

static ps::OutArgs out_args(ps_plan_t plan, const Inst& I) {
  ps::OutArgs o{};
  o.acc = ws_ptr<double>(plan, I.use_reduced() ? I.off_sumacc : I.off_acc);
  o.slots = I.use_reduced() ? 1 : I.slots_used();
  o.slot_stride = (int64_t)I.slot_doubles();
  o.N1 = (int32_t)I.N1;
  o.N2 = (int32_t)I.N2;
  o.P = I.cfg.n_pairs;
  o.C = I.C;
  return o;
}

ps_status ps_spectra(ps_plan_t plan, int32_t inst, double* out_dev, int64_t* n_frames) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  const Inst& I = plan->inst[(size_t)inst];
  if (!out_dev) return fail(PS_ERR_ARG, "null output");
  if (I.n_frames == 0) return fail(PS_ERR_STATE, "instance %d has no accumulated frames", inst);
  if ((st = reduce_slots(plan, I)) != PS_OK) return st;
  ps::OutArgs o = out_args(plan, I);
  o.spectra = out_dev;
  hipError_t e = timed(plan, PS_KERNEL_SPECTRA, [&](const ps::Launch& l) { return ps::launch_spectra(o, l); });
  if (e != hipSuccess) return hip_fail(e, "spectra launch");
  if (n_frames) *n_frames = I.n_frames;
  return PS_OK;
}

ps_status ps_stokes(ps_plan_t plan, int32_t inst, const ps_cal* cal, float* iquv_dev) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  const Inst& I = plan->inst[(size_t)inst];
  if (!iquv_dev) return fail(PS_ERR_ARG, "null output");
  if (I.n_frames == 0) return fail(PS_ERR_STATE, "instance %d has no accumulated frames", inst);
  if (cal && cal->feed != PS_FEED_LINEAR && cal->feed != PS_FEED_CIRCULAR)
    return fail(PS_ERR_ARG, "unknown feed %d", cal->feed);
  if ((st = reduce_slots(plan, I)) != PS_OK) return st;
  const ps::OutArgs o = stokes_args(plan, I, I.n_frames, cal, iquv_dev);
  hipError_t e = timed(plan, PS_KERNEL_STOKES, [&](const ps::Launch& l) { return ps::launch_stokes(o, l); });
  if (e != hipSuccess) return hip_fail(e, "stokes launch");
  return PS_OK;
}

ps_status ps_stokes_all(ps_plan_t plan, const ps_cal* cal, float* const* iquv_dev) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (!iquv_dev) return fail(PS_ERR_ARG, "null output array");
  std::vector<ps::OutArgs> outs;
  std::vector<int32_t> ends;
  int32_t total = 0;
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    if (!iquv_dev[i]) continue;
    const Inst& I = plan->inst[i];
    if (I.n_frames == 0) return fail(PS_ERR_STATE, "instance %zu has no accumulated frames", i);
    if (cal && cal[i].feed != PS_FEED_LINEAR && cal[i].feed != PS_FEED_CIRCULAR)
      return fail(PS_ERR_ARG, "instance %zu: unknown feed %d", i, cal[i].feed);
    const ps::OutArgs o = stokes_args(plan, I, I.n_frames, cal ? &cal[i] : nullptr, iquv_dev[i]);
    outs.push_back(o);
    total += ps::output_tiles(o.N1, o.N2, o.P);
    ends.push_back(total);
  }
  if (outs.empty()) return PS_OK;
  for (size_t i = 0; i < plan->inst.size(); ++i)
    if (iquv_dev[i] && (st = reduce_slots(plan, plan->inst[i])) != PS_OK) return st;
  std::vector<unsigned char> img;
  append_bytes(img, outs.data(), outs.size());
  const size_t ends_at = img.size();
  append_bytes(img, ends.data(), ends.size());
  if ((st = upload_desc(plan, plan->out_desc, img)) != PS_OK) return st;
  char* dev = plan->ws + plan->out_desc.off;
  ps::BatchArgs b{};
  b.tasks = dev;
  b.tile_end = reinterpret_cast<const int32_t*>(dev + ends_at);
  b.n_tasks = (int32_t)outs.size();
  b.total = total;
  hipError_t e = timed(plan, PS_KERNEL_STOKES, [&](const ps::Launch& l) { return ps::launch_output_batch(true, b, l); });
  if (e != hipSuccess) return hip_fail(e, "grouped stokes launch");
  return PS_OK;
}

ps_status ps_set_histograms(ps_plan_t plan, int32_t inst, int32_t enable) {
  if (!plan) return fail(PS_ERR_ARG, "null plan");
  ps_status st = check_inst(plan, inst);
  if (st != PS_OK) return st;
  Inst& I = plan->inst[(size_t)inst];
  if (enable && (I.mx() || I.hist_bins() == 0))
    return fail(PS_ERR_UNSUPPORTED, "instance %d: level histograms need 2-, 4- or 8-bit codes and FP32 passes", inst);
  if ((enable != 0) != I.hist_on && I.n_frames > 0)
    return fail(PS_ERR_STATE, "instance %d: switch histograms between integrations (after ps_reset)", inst);
  I.hist_on = enable != 0;
  I.hist_zeroed = false;
  I.hist_frames = 0;
  return PS_OK;
}

ps_status ps_histograms(ps_plan_t plan, int32_t inst, uint64_t* counts_dev, double* power_dev, int64_t* n_frames) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  const Inst& I = plan->inst[(size_t)inst];
  if (!I.hist_on || !I.hist_zeroed) return fail(PS_ERR_STATE, "instance %d has no histograms in this integration", inst);
  const int64_t nb = (int64_t)I.cfg.n_pairs * 2 * I.hist_bins();
  unsigned long long* h = ws_ptr<unsigned long long>(plan, I.off_hist);
  hipError_t e = hipSuccess;
  if (counts_dev) {
    e = ps::launch_copy(h, counts_dev, (size_t)nb * 8, plan->stream);
    if (e != hipSuccess) return hip_fail(e, "histogram copy");
  }
  if (power_dev) {
    e = timed(plan, PS_KERNEL_OTHER, [&](const ps::Launch& l) {
      return ps::launch_hist_power(h, I.cfg.n_pairs * 2, I.cfg.bits, power_dev, l);
    });
    if (e != hipSuccess) return hip_fail(e, "histogram power launch");
  }
  if (n_frames) *n_frames = I.hist_frames;
  return PS_OK;
}

ps_status ps_graph_begin(ps_plan_t plan) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (plan->capturing) return fail(PS_ERR_STATE, "a capture is already in progress");
  if (plan->prof) return fail(PS_ERR_STATE, "turn per-kernel profiling off before capturing");
  if (!plan->stream) return fail(PS_ERR_STATE, "graph capture needs the plan bound to a stream other than the null stream");
  hipError_t e = hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "begin capture");
  plan->capturing = true;
  return PS_OK;
}

ps_status ps_graph_end(ps_plan_t plan, int32_t keep) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (!plan->capturing) return fail(PS_ERR_STATE, "no capture in progress");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(plan->stream, &g);
  plan->capturing = false;
  if (e != hipSuccess) return hip_fail(e, "end capture");
  if (!keep) {
    (void)hipGraphDestroy(g);
    return PS_OK;
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
  plan->gexec = x;
  plan->graph_state.clear();
  for (const Inst& I : plan->inst) plan->graph_state.push_back({I.first, I.hist_zeroed, I.n_frames, I.hist_frames});
  return PS_OK;
}

ps_status ps_graph_launch(ps_plan_t plan) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (!plan->gexec) return fail(PS_ERR_STATE, "no captured graph");
  if (plan->capturing) return fail(PS_ERR_STATE, "cannot replay while capturing");
  hipError_t e = hipGraphLaunch(plan->gexec, plan->stream);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  for (size_t i = 0; i < plan->inst.size(); ++i) {
    Inst& I = plan->inst[i];
    const ps_plan_s::InstState& g = plan->graph_state[i];
    I.first = g.first;
    I.n_frames = g.n_frames;
    I.hist_zeroed = g.hist_zeroed;
    I.hist_frames = g.hist_frames;
    plan->touch(I);
  }
  return PS_OK;
}

ps_status ps_calibrate_backward(ps_plan_t plan, int32_t inst, const void* packed_dev, int64_t n_samples,
                                const ps_cal* cal, const float* dL_diquv_dev, const ps_cal_grad* grad) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  Inst& I = plan->inst[(size_t)inst];
  if (!dL_diquv_dev || !grad) return fail(PS_ERR_ARG, "null upstream gradient or gradient outputs");
  if (I.n_frames == 0) return fail(PS_ERR_STATE, "instance %d has no accumulated frames", inst);
  if (cal && cal->feed != PS_FEED_LINEAR)
    return fail(PS_ERR_UNSUPPORTED, "the adjoint is built for linear feeds (Eq. 2)");
  const bool want_taps = grad->d_taps != nullptr;
  if (want_taps) {
    if (!I.taps()) return fail(PS_ERR_ARG, "d_taps requested for an instance without a PS_WIN_TAPS window");
    if (I.N1 > 512 || I.N2 > 512)
      return fail(PS_ERR_UNSUPPORTED, "the window adjoint is built for passes of at most 512 points (fft_len <= 2^18)");
    if (!packed_dev) return fail(PS_ERR_ARG, "null packed input");
    if (n_samples < 0 || n_samples % I.N) return fail(PS_ERR_SIZE, "n_samples is not a multiple of fft_len");
    if (I.frames_in(n_samples) != I.n_frames)
      return fail(PS_ERR_STATE, "the input has %lld frames but the integration has %lld",
                  (long long)I.frames_in(n_samples), (long long)I.n_frames);
  }
  if (I.N1 > 512 || I.N2 > 512)
    return fail(PS_ERR_UNSUPPORTED, "the adjoint is built for passes of at most 512 points (fft_len <= 2^18)");
  if ((st = reduce_slots(plan, I)) != PS_OK) return st;
  ps::BwChanArgs ca{};
  ca.acc = ws_ptr<double>(plan, I.use_reduced() ? I.off_sumacc : I.off_acc);
  ca.slots = I.use_reduced() ? 1 : I.slots_used();
  ca.slot_stride = (int64_t)I.slot_doubles();
  ca.N1 = (int32_t)I.N1;
  ca.P = I.cfg.n_pairs;
  ca.C = I.C;
  ca.n_frames = (double)I.n_frames;
  ca.sumw2 = ws_ptr<double>(plan, I.off_sumw2);
  const double psi = cal ? cal->psi : 0.0;
  ca.cos2psi = std::cos(2.0 * psi);
  ca.sin2psi = std::sin(2.0 * psi);
  if (cal) {
    ca.gain_x = cal->gain_x;
    ca.gain_y = cal->gain_y;
    ca.dterms = cal->dterms;
  }
  ca.g_iquv = dL_diquv_dev;
  ca.d_gain_x = grad->d_gain_x;
  ca.d_gain_y = grad->d_gain_y;
  ca.d_dterms = grad->d_dterms;
  ca.g_a = want_taps ? ws_ptr<float>(plan, I.off_ga) : nullptr;
  ca.red = ws_ptr<double>(plan, I.off_red);
  ca.parts = ps::bw_parts((int)I.N1, (int)I.N2);
  ca.norm = ws_ptr<double>(plan, I.off_norm);
  // with the one-pass tap gradient, that kernel also reduces the channel kernel's unit partials
  const bool taps_reduce = want_taps && ps::bw_taps_block_form(I.N, I.cfg.n_taps);
  hipError_t e = timed(plan, PS_KERNEL_BACKWARD,
                       [&](const ps::Launch& l) { return ps::launch_bw_channel((int)I.N2, ca, l, !taps_reduce); });
  if (e != hipSuccess) return hip_fail(e, "backward channel launch");
  if (!want_taps) return PS_OK;

  const int64_t F = I.n_frames;
  const uint8_t* base = static_cast<const uint8_t*>(packed_dev);
  int groups_used = 0;
  // the forward's column-pass output of this integration, if the inter-pass buffer still holds all of it
  const bool reuse_T = !plan->capturing && plan->t_inst == inst && plan->t_gen == I.gen && F <= I.chunk;
  for (int64_t f0 = 0; f0 < F; f0 += I.chunk) {
    const int nf = (int)((F - f0) < I.chunk ? (F - f0) : I.chunk);
    ps::ColArgs col{};
    col.in = base + f0 * I.hop * I.bits_per_sample() / 8;
    const int64_t in_bytes = ((int64_t)(nf - 1) * I.hop + I.N) * I.bits_per_sample() / 8;
    col.in_bytes = in_bytes < (int64_t(1) << 31) ? (uint32_t)in_bytes : 0u;
    const int mode = in_bytes < (int64_t(1) << 31) ? I.load_mode : 0;
    const bool fast = mode == 1;  // the backward's own column pass has the int8 two-stream word loader
    col.N = I.N;
    col.hop = I.hop;
    col.N2 = (int32_t)I.N2;
    col.S = I.cfg.n_streams;
    col.P = I.cfg.n_pairs;
    for (int p = 0; p < 4; ++p) {
      col.px[p] = I.cfg.pair_x[p];
      col.py[p] = I.cfg.pair_y[p];
    }
    col.n_colblk = (int32_t)(I.N2 / ps::colpass_cols((int)I.N1));  // default tiling for the recompute
    col.n_frames = nf;
    {
      const int64_t per_frame = (int64_t)col.n_colblk * col.P;
      int64_t groups = (plan->n_cu + per_frame / 2) / per_frame;
      if (groups < 1) groups = 1;
      if (groups > nf) groups = nf;
      col.frames_per_block = (int32_t)((nf + groups - 1) / groups);
    }
    col.win = ws_ptr<float>(plan, I.off_win);
    col.tw_col = ws_ptr<float2>(plan, I.off_tw_col);
    col.tw_hi = col.tw_col;
    col.tw_lo = ws_ptr<float2>(plan, I.off_tw_lo);
    col.lo_bits = I.m2;
    col.T = ws_ptr<float2>(plan, I.off_T);
    if (!reuse_T) {
      e = timed(plan, PS_KERNEL_BACKWARD, [&](const ps::Launch& l) { return ps::launch_colpass((int)I.N1, ps::colpass_cols((int)I.N1), I.cfg.bits, mode, col, l); });
      if (e != hipSuccess) return hip_fail(e, "backward forward-recompute launch");
    }
    plan->t_inst = -1;  // the backward row pass writes T' over T
    ps::BwRowArgs ra{};
    ra.T = col.T;
    ra.N1 = (int32_t)I.N1;
    ra.P = I.cfg.n_pairs;
    ra.n_frames = nf;
    ra.tw_row = ws_ptr<float2>(plan, I.off_tw_row);
    ra.tw_hi = col.tw_hi;
    ra.tw_lo = col.tw_lo;
    ra.lo_bits = I.m2;
    ra.g_a = ca.g_a;
    e = timed(plan, PS_KERNEL_BACKWARD, [&](const ps::Launch& l) { return ps::launch_bw_rowpass((int)I.N2, ra, l); });
    if (e != hipSuccess) return hip_fail(e, "backward row pass launch");
    ps::BwColArgs ba{};
    ba.col = col;
    ba.col.win = nullptr;
    {
      // at most kMaxBwGroups groups of frames, each with its own partial dL/dw
      const int64_t per_frame = (int64_t)col.n_colblk * col.P;
      int64_t groups = (plan->n_cu + per_frame / 2) / per_frame;
      if (groups < 1) groups = 1;
      const int64_t cap = ps::kMaxBwGroups / col.P > 0 ? ps::kMaxBwGroups / col.P : 1;
      if (groups > cap) groups = cap;
      if (groups > nf) groups = nf;
      ba.col.frames_per_block = (int32_t)((nf + groups - 1) / groups);
      const int used = (int)((nf + ba.col.frames_per_block - 1) / ba.col.frames_per_block);
      if (f0 == 0) groups_used = used;
    }
    ba.dw = ws_ptr<double>(plan, I.off_dw);
    ba.first = f0 == 0 ? 1 : 0;
    e = timed(plan, PS_KERNEL_BACKWARD, [&](const ps::Launch& l) { return ps::launch_bw_colpass((int)I.N1, I.cfg.bits, fast, ba, l); });
    if (e != hipSuccess) return hip_fail(e, "backward column pass launch");
  }
  ps::BwTapArgs ta{};
  ta.dw = ws_ptr<double>(plan, I.off_dw);
  ta.groups = groups_used * I.cfg.n_pairs;
  ta.N = I.N;
  ta.n_taps = I.cfg.n_taps;
  ta.taps = ws_ptr<float>(plan, I.off_taps);
  ta.sumw2 = ws_ptr<double>(plan, I.off_sumw2);
  ta.norm = ca.norm;
  ta.P = I.cfg.n_pairs;
  ta.d_taps = grad->d_taps;
  ta.part = ws_ptr<double>(plan, I.off_tpart);
  ta.red = ca.red;
  ta.U = ca.parts;
  ta.d_dterms = taps_reduce ? grad->d_dterms : nullptr;
  e = timed(plan, PS_KERNEL_BACKWARD, [&](const ps::Launch& l) { return ps::launch_bw_taps(ta, l); });
  if (e != hipSuccess) return hip_fail(e, "tap gradient launch");
  return PS_OK;
}

ps_status ps_state_bytes(ps_plan_t plan, int32_t inst, size_t* bytes) {
  ps_status st = check_plan(plan, false);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  if (!bytes) return fail(PS_ERR_ARG, "null bytes");
  const Inst& I = plan->inst[(size_t)inst];
  *bytes = I.acc_bytes() + (I.overlap() ? I.tail_bytes() : 0);
  return PS_OK;
}

ps_status ps_state_export(ps_plan_t plan, int32_t inst, void* dst_dev, int64_t* n_frames) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  const Inst& I = plan->inst[(size_t)inst];
  if (!dst_dev) return fail(PS_ERR_ARG, "null destination");
  if (I.n_frames == 0) return fail(PS_ERR_STATE, "instance %d has no accumulated frames", inst);
  hipError_t e = ps::launch_copy(plan->ws + I.off_acc, dst_dev, I.acc_bytes(), plan->stream);
  if (e == hipSuccess && I.overlap())
    e = ps::launch_copy(plan->ws + I.off_stage, static_cast<char*>(dst_dev) + I.acc_bytes(), I.tail_bytes(), plan->stream);
  if (e != hipSuccess) return hip_fail(e, "state export");
  if (n_frames) *n_frames = I.n_frames;
  return PS_OK;
}

ps_status ps_state_import(ps_plan_t plan, int32_t inst, const void* src_dev, int64_t n_frames) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if ((st = check_inst(plan, inst)) != PS_OK) return st;
  Inst& I = plan->inst[(size_t)inst];
  if (!src_dev) return fail(PS_ERR_ARG, "null source");
  if (n_frames <= 0) return fail(PS_ERR_ARG, "n_frames must be positive");
  hipError_t e = ps::launch_copy(src_dev, plan->ws + I.off_acc, I.acc_bytes(), plan->stream);
  if (e == hipSuccess && I.overlap())
    e = ps::launch_copy(static_cast<const char*>(src_dev) + I.acc_bytes(), plan->ws + I.off_stage, I.tail_bytes(), plan->stream);
  if (e != hipSuccess) return hip_fail(e, "state import");
  I.n_frames = n_frames;
  I.first = false;
  plan->touch(I);
  return PS_OK;
}

ps_status ps_integration_id(ps_plan_t plan, int32_t inst, uint64_t* id) {
  if (!plan) return fail(PS_ERR_ARG, "null plan");
  ps_status st = check_inst(plan, inst);
  if (st != PS_OK) return st;
  if (!id) return fail(PS_ERR_ARG, "null id");
  *id = plan->inst[(size_t)inst].gen;
  return PS_OK;
}

ps_status ps_unpack(const void* packed_dev, int32_t bits, int32_t n_streams, int64_t n_time, float* out_dev,
                    void* hip_stream) {
  if (!packed_dev || !out_dev) return fail(PS_ERR_ARG, "null buffer");
  if (bits != 2 && bits != 4 && bits != 8 && bits != 32) return fail(PS_ERR_ARG, "bits %d not in {2, 4, 8, 32}", bits);
  if (n_streams < 1 || n_streams > 8) return fail(PS_ERR_ARG, "n_streams %d not in 1..8", n_streams);
  if (n_time < 0) return fail(PS_ERR_ARG, "negative n_time");
  if (n_time == 0) return PS_OK;
  hipError_t e = ps::launch_unpack(packed_dev, bits, n_streams, n_time, out_dev, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "unpack launch");
  return PS_OK;
}

ps_status ps_profile_enable(ps_plan_t plan, int32_t enable) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (enable && plan->ev.empty()) {
    plan->ev.resize(2 * kMaxTimed, nullptr);
    for (size_t i = 0; i < plan->ev.size(); ++i) {
      hipError_t e = hipEventCreate(&plan->ev[i]);
      if (e != hipSuccess) return hip_fail(e, "profiling event create");
    }
    plan->ev_kind.assign(kMaxTimed, 0);
  }
  plan->prof = enable != 0;
  return PS_OK;
}

ps_status ps_profile_read(ps_plan_t plan, double* ms_total, int64_t* launches) {
  ps_status st = check_plan(plan, true);
  if (st != PS_OK) return st;
  if (!ms_total || !launches) return fail(PS_ERR_ARG, "null output");
  for (int k = 0; k < PS_KERNEL_COUNT; ++k) {
    ms_total[k] = 0.0;
    launches[k] = 0;
  }
  if (plan->ev_used) {
    hipError_t e = hipEventSynchronize(plan->ev[2 * plan->ev_used - 1]);
    if (e != hipSuccess) return hip_fail(e, "profiling event wait");
  }
  for (size_t i = 0; i < plan->ev_used; ++i) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, plan->ev[2 * i], plan->ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "profiling elapsed time");
    ms_total[plan->ev_kind[i]] += (double)ms;
    launches[plan->ev_kind[i]] += 1;
  }
  plan->ev_used = 0;
  return PS_OK;
}

ps_status ps_destroy(ps_plan_t plan) {
  delete plan;
  return PS_OK;
}

// ------------------------------------------------------------------------------------------------
// post-integration reductions

ps_status ps_channel_average(const float* in_dev, int64_t n_spec, int64_t n_chan, int32_t factor,
                             const uint8_t* flags_dev, float* out_dev, int32_t* counts_dev, void* hip_stream) {
  if (!in_dev || !out_dev) return fail(PS_ERR_ARG, "null spectra or output");
  if (n_spec < 0 || n_spec > 65535) return fail(PS_ERR_ARG, "n_spec %lld not in 0..65535", (long long)n_spec);
  if (n_chan < 1 || factor < 1 || n_chan % factor)
    return fail(PS_ERR_SIZE, "factor %d does not divide n_chan %lld", factor, (long long)n_chan);
  if (n_chan / factor > (int64_t(1) << 31) - 1) return fail(PS_ERR_SIZE, "too many bins");
  if (n_spec == 0) return PS_OK;
  ps::ChanAvgArgs a{in_dev, n_spec, n_chan, factor, flags_dev, out_dev, counts_dev};
  hipError_t e = ps::launch_channel_average(a, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "channel average launch");
  return PS_OK;
}

static ps_status spline_args(int64_t n_chan, int32_t knot_spacing, double edge_frac, ps::SplineArgs* a) {
  if (knot_spacing < 4) return fail(PS_ERR_ARG, "knot spacing %d below 4 channels", knot_spacing);
  if (!(edge_frac >= 0.0 && edge_frac < 0.5)) return fail(PS_ERR_ARG, "edge fraction %g not in [0, 0.5)", edge_frac);
  if (n_chan < 1 || n_chan > (int64_t(1) << 31)) return fail(PS_ERR_ARG, "n_chan %lld out of range", (long long)n_chan);
  a->n_chan = n_chan;
  a->c0 = (int64_t)std::floor(edge_frac * (double)n_chan);
  a->c1 = n_chan - a->c0;
  a->K = knot_spacing;
  if (a->c1 - a->c0 < 4 * (int64_t)knot_spacing)
    return fail(PS_ERR_SIZE, "the fit range of %lld channels holds fewer than four knot intervals",
                (long long)(a->c1 - a->c0));
  a->n_int = (a->c1 - a->c0 + knot_spacing - 1) / knot_spacing;
  a->n_coef = a->n_int + 3;
  if (a->n_coef > ps::kMaxSplineCoef)
    return fail(PS_ERR_UNSUPPORTED, "%lld spline coefficients exceed the %lld of one solve", (long long)a->n_coef,
                (long long)ps::kMaxSplineCoef);
  return PS_OK;
}

static size_t spline_work_bytes(const ps::SplineArgs& a) {
  return align_up((size_t)a.n_int * 14 * 8) + align_up((size_t)a.n_coef * 8);
}

ps_status ps_bandpass_work_bytes(int64_t n_chan, int32_t knot_spacing, double edge_frac, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "null bytes");
  ps::SplineArgs a{};
  ps_status st = spline_args(n_chan, knot_spacing, edge_frac, &a);
  if (st != PS_OK) return st;
  *bytes = spline_work_bytes(a);
  return PS_OK;
}

static ps_status bandpass_fit_in(ps::SplineArgs& a, const float* h_dev, char* work, float* smooth_dev,
                                  void* hip_stream) {
  a.h = h_dev;
  a.partial = reinterpret_cast<double*>(work);
  a.coef = reinterpret_cast<double*>(work + align_up((size_t)a.n_int * 14 * 8));
  a.smooth = smooth_dev;
  hipError_t e = ps::launch_bandpass_fit(a, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "bandpass fit launch");
  return PS_OK;
}

ps_status ps_bandpass_fit(const float* h_dev, int64_t n_chan, int32_t knot_spacing, double edge_frac,
                          void* work_dev, size_t work_bytes, float* smooth_dev, void* hip_stream) {
  if (!h_dev || !smooth_dev) return fail(PS_ERR_ARG, "null spectrum or output");
  ps::SplineArgs a{};
  ps_status st = spline_args(n_chan, knot_spacing, edge_frac, &a);
  if (st != PS_OK) return st;
  if (!work_dev || reinterpret_cast<uintptr_t>(work_dev) % kAlign)
    return fail(PS_ERR_WORKSPACE, "null or misaligned work buffer");
  if (work_bytes < spline_work_bytes(a))
    return fail(PS_ERR_WORKSPACE, "work buffer of %zu bytes is smaller than the %zu needed", work_bytes,
                spline_work_bytes(a));
  return bandpass_fit_in(a, h_dev, static_cast<char*>(work_dev), smooth_dev, hip_stream);
}

ps_status ps_bandpass_fit_static(const float* h_dev, int64_t n_chan, int32_t knot_spacing, double edge_frac,
                                 float* smooth_dev, void* hip_stream) {
  if (!h_dev || !smooth_dev) return fail(PS_ERR_ARG, "null spectrum or output");
  ps::SplineArgs a{};
  ps_status st = spline_args(n_chan, knot_spacing, edge_frac, &a);
  if (st != PS_OK) return st;
  if (spline_work_bytes(a) > ps::kBandpassScratchBytes)
    return fail(PS_ERR_SIZE, "%lld spline coefficients need %zu bytes of scratch; the static buffer holds %zu (%lld coefficients)",
                (long long)a.n_coef, spline_work_bytes(a), ps::kBandpassScratchBytes,
                (long long)ps::kBandpassScratchCoef);
  void* work = nullptr;
  hipError_t e = ps::bandpass_scratch(static_cast<hipStream_t>(hip_stream), &work);
  if (e != hipSuccess) return hip_fail(e, "static scratch address");
  return bandpass_fit_in(a, h_dev, static_cast<char*>(work), smooth_dev, hip_stream);
}

ps_status ps_bandpass_correct(const float* hk_dev, int64_t n_spec, int64_t n_chan, const float* smooth_dev,
                              const double* gain_dev, float* out_dev, void* hip_stream) {
  if (!hk_dev || !smooth_dev || !out_dev) return fail(PS_ERR_ARG, "null spectra, bandpass or output");
  if (n_spec < 0 || n_spec > 65535) return fail(PS_ERR_ARG, "n_spec %lld not in 0..65535", (long long)n_spec);
  if (n_chan < 1 || n_chan > (int64_t(1) << 31)) return fail(PS_ERR_ARG, "n_chan %lld out of range", (long long)n_chan);
  if (n_spec == 0) return PS_OK;
  hipError_t e = ps::launch_bandpass_correct(hk_dev, n_spec, n_chan, smooth_dev, gain_dev, out_dev,
                                             static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "bandpass correction launch");
  return PS_OK;
}

ps_status ps_band_stats(const float* x_dev, int64_t n_spec, int64_t n_chan, double* mean_sd_dev, void* hip_stream) {
  if (!x_dev || !mean_sd_dev) return fail(PS_ERR_ARG, "null spectra or output");
  if (n_spec < 0 || n_spec > (int64_t(1) << 31) - 1 || n_chan < 1)
    return fail(PS_ERR_ARG, "n_spec %lld or n_chan %lld out of range", (long long)n_spec, (long long)n_chan);
  if (n_spec == 0) return PS_OK;
  hipError_t e = ps::launch_band_stats(x_dev, n_spec, n_chan, mean_sd_dev, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "band statistics launch");
  return PS_OK;
}

ps_status ps_allan_work_bytes(int64_t n_points, int64_t point_stride, int64_t n_series, int64_t series_stride,
                              int32_t n_lags, size_t* bytes) {
  if (!bytes) return fail(PS_ERR_ARG, "null bytes");
  if (n_lags < 1 || n_lags > ps::kMaxAllanLags) return fail(PS_ERR_ARG, "n_lags %d not in 1..%d", n_lags, ps::kMaxAllanLags);
  if (n_points < 0 || n_series < 0 || n_series > (int64_t(1) << 31) - 1 || point_stride < 0 || series_stride < 0)
    return fail(PS_ERR_ARG, "negative size or stride, or too many series");
  *bytes = (size_t)ps::allan_part_doubles(n_points, n_series, point_stride, series_stride, n_lags) * 8;
  return PS_OK;
}

ps_status ps_allan(const float* x_dev, int64_t n_points, int64_t point_stride, int64_t n_series,
                   int64_t series_stride, const int32_t* lags, int32_t n_lags, double spacing, int32_t normalize,
                   void* work_dev, size_t work_bytes, double* out_dev, void* hip_stream) {
  if (!x_dev || !lags || !out_dev) return fail(PS_ERR_ARG, "null series, lags or output");
  size_t need = 0;
  ps_status st = ps_allan_work_bytes(n_points, point_stride, n_series, series_stride, n_lags, &need);
  if (st != PS_OK) return st;
  if ((int64_t)(n_points > 0 ? (n_points + ps::kAllanChunk - 1) / ps::kAllanChunk : 1) > 65535)
    return fail(PS_ERR_SIZE, "%lld points per series exceed the block form's 65535 chunks", (long long)n_points);
  if (need && (!work_dev || work_bytes < need))
    return fail(PS_ERR_WORKSPACE, "work buffer of %zu bytes is smaller than the %zu needed", work_bytes, need);
  if (!(spacing > 0.0)) return fail(PS_ERR_ARG, "spacing must be positive");
  ps::AllanArgs a{};
  for (int i = 0; i < n_lags; ++i) {
    if (lags[i] < 1) return fail(PS_ERR_ARG, "lag %d is %d (must be >= 1)", i, lags[i]);
    a.lags[i] = lags[i];
  }
  if (n_series == 0) return PS_OK;
  a.x = x_dev;
  a.n_points = n_points;
  a.point_stride = point_stride;
  a.n_series = n_series;
  a.series_stride = series_stride;
  a.n_lags = n_lags;
  a.normalize = normalize ? 1 : 0;
  a.spacing = spacing;
  a.out = out_dev;
  a.part = static_cast<double*>(work_dev);
  hipError_t e = ps::launch_allan(a, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "Allan variance launch");
  return PS_OK;
}

const char* ps_status_string(ps_status s) {
  switch (s) {
    case PS_OK: return "PS_OK";
    case PS_ERR_ARG: return "PS_ERR_ARG";
    case PS_ERR_SIZE: return "PS_ERR_SIZE";
    case PS_ERR_UNSUPPORTED: return "PS_ERR_UNSUPPORTED";
    case PS_ERR_STATE: return "PS_ERR_STATE";
    case PS_ERR_WORKSPACE: return "PS_ERR_WORKSPACE";
    case PS_ERR_HIP: return "PS_ERR_HIP";
  }
  return "PS_UNKNOWN";
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

int32_t ps_version(void) { return 100; }

}  // extern "C"
