// Single-pass short transforms: launch arguments and launcher (device code in polaris_fused.hip).
#pragma once

#include "polaris_internal.h"

namespace ps {

struct FusedArgs {
  const uint8_t* in;        // packed input of frame 0 of this launch
  int64_t hop;              // samples between frame starts
  int32_t S, P;
  int32_t px[4], py[4];
  int32_t n_frames;         // frames in this launch
  const float* win;         // window [N] (all ones for the rectangular window)
  const float2* tw;         // W_N^m, m < N
  double* acc;              // accumulator slots, the layout of the four-step row pass ([G][P][N1/2][4][N2])
  int32_t G;                // slots
  int32_t N1, N2;           // the split that fixes the accumulator layout
  int64_t F0;               // frames of the integration before this launch
  int64_t slot_stride;      // doubles per slot
};

constexpr int kFusedMinLog2 = 8, kFusedMaxLog2 = 12;
int fused_threads(int N);
hipError_t launch_fused(int N, int bits, const FusedArgs& a, const Launch& l);

// Many accumulator slots (beyond kDirectSlots) are summed by a two-stage reduction before the readers run:
// chunks of kReduceChunk slots in slot order, then the chunk sums in chunk order (a fixed order, so results
// are identical from run to run and independent of how the frames were split over calls).
constexpr int kDirectSlots = 64, kReduceChunk = 32;
inline int64_t slot_reduce_chunks(int slots) { return (slots + kReduceChunk - 1) / kReduceChunk; }
hipError_t launch_slot_reduce(const double* acc, int64_t elems, int slots, int64_t slot_stride, double* part,
                              double* out, const Launch& l);

}  // namespace ps
