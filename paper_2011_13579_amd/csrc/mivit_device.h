// Device-side descriptors shared by the host plan code and the kernels of the
// Viterbi decoder library.  Internal header (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mivit {

constexpr int kMaxK = 9;
constexpr int kMaxStates = 1 << (kMaxK - 1);

// A code as the kernels see it (copied from mivit_code after validation).
struct DevCode {
  int32_t K;
  int32_t beta;
  uint32_t gen[4];
};

// One independent run of the trellis: a whole frame or one chunk window.
struct Item {
  int64_t llr_off;    // element index of stage 0, soft value 0
  int64_t surv_off;   // uint64-word index of this item's decision block
  int64_t bit_off;    // output bit index of emitted bit 0 (multiple of 32)
  int32_t n_stages;   // S
  int32_t out_begin;  // first stage whose decoded bit is emitted
  int32_t n_out;      // number of decoded bits emitted
  int32_t code;       // index into the code table
  int32_t start_known;
  int32_t end_state;  // >= 0: fixed final state, -1: best final state
  int32_t frame;      // frame whose metric/end state this item reports, or -1
  int32_t slot;       // index of this item in per-item scratch arrays
};

// Frame facts the gradient kernel needs.
struct GradFrame {
  int64_t llr_off;
  int64_t bit_off;
  int32_t n_stages;
  int32_t n_out;   // decoded bits stored; stages >= n_out carry input 0
  int32_t code;
  int32_t pad;
};

// Workgroups a persistent grid of 'kernel' keeps resident on the device
// (compute units times resident workgroups per unit), 0 if unknown.
template <typename Kernel>
inline int resident_workgroups(Kernel kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess)
    return 0;
  return cus * per;
}

// Decision words per stage for a code with 2^(K-1) states.
__host__ __device__ inline int words_per_stage(int K) {
  int ns = 1 << (K - 1);
  return ns <= 64 ? 1 : ns / 64;
}

// Survivor memory of one work item, in uint64 words, per survivor layout
// (rounded up to an even count so every item starts 16-byte aligned):
//   rotating radix 2 (K <= 7) and bytes-by-position (K = 8, 9): whole
//     32-stage blocks of 2^(K-1) 32-bit words;
//   packed radix 4 (one frame pair): 2^(K-1) 32-bit words per 8 iterations;
//   natural layouts: words_per_stage(K) per stage.
__host__ __device__ inline int64_t even_words(int64_t w) { return (w + 1) & ~(int64_t)1; }
__host__ __device__ inline int64_t surv_words_blocks32(int K, int S) {
  return even_words((int64_t)((S + 31) / 32) * (1 << (K - 1)) / 2);
}
__host__ __device__ inline int64_t surv_words_r4p(int K, int S) {
  return even_words((int64_t)((S / 2 + 7) / 8) * (1 << (K - 1)) / 2);
}
__host__ __device__ inline int64_t surv_words_natural(int K, int S) {
  return even_words((int64_t)S * words_per_stage(K));
}
// The traceback reads whole staging blocks past an item's end: slack words
// after the last item.
constexpr int64_t kSurvSlackWords = 32;

}  // namespace mivit
