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

// Most parts a frame is split into in time (see SplitUnit).
constexpr int kMaxSplitParts = 8;

// One unit of work of a forward kernel that splits frames in time.  For the
// packed radix-4 kernel: the frames of one wavefront-table entry (first
// item, count) over the iterations [it_begin, it_end); for the K = 8, 9
// radix-2 kernel: item `first` (count 1) over the stages [it_begin, it_end).  An entry decoded whole is one unit (part 0 of 1).  An
// entry split in time is n_parts units that run concurrently: unit p > 0
// first runs `warm` iterations before it_begin from all-zero path metrics
// (an unknown start, as for the windows of §III) and keeps no decisions from
// them.  Its decisions are exact when its metrics at it_begin differ from
// the true ones by a constant, which a check after the forward pass
// establishes; otherwise a repair unit restarts the frames at it_begin from
// the metrics part p-1 left there.
struct SplitUnit {
  int32_t first, count;
  int32_t it_begin, it_end;
  int32_t warm;
  int32_t part, n_parts;
  int32_t bnd;  // split entries: index of the entry's first boundary record, else -1
};

// The two sides of boundary k of a split entry (between parts k and k+1, at
// iteration it_begin of part k+1), per lane (and register, for the kernel
// with four states per lane: 256 words, else the first 64): packed metrics
// (low two bits cleared, after the range control of that iteration), and
// per frame of the entry (up to 8) the metric of state 0 there, each part
// counting from its own origin.
struct R4Bound {
  uint32_t v_start[256];  // part k+1 after its warm-up
  uint32_t v_end[256];    // part k at its end
  int64_t m_start[8];
  int64_t m_end[8];
  int32_t it_at;         // the boundary's iteration (part k+1's it_begin)
  int32_t pad;
};

// Boundary k of a frame split in time in the K = 8, 9 radix-2 kernel: the
// metric of every position (2^(K-1), lane + 64 r) after the range control
// at stage it_at, for part k at its end and part k+1 after its warm-up, and
// each part's metric of state 0 there from its own origin.
struct WideBound {
  int32_t v_start[256];
  int32_t v_end[256];
  int64_t m_start;
  int64_t m_end;
  int32_t it_at;
  int32_t pad;
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

// Dragonfly groups of a K = 7 rate-1/2 code for the matrix-core radix-4
// kernel (§VIII-D-2): dragonfly f's super-branch outputs are those of
// leader[group[f]] with the left index y replaced by y ^ a[f].  Unused
// groups have leader -1.
struct MfmaGroups {
  int32_t group[16];
  int32_t a[16];
  int32_t leader[4];
};
// Fills G from the code; false when the code is not K = 7, rate 1/2 or
// needs more than four groups.
bool mfma_groups(int K, int beta, const uint32_t* gen, MfmaGroups* G);

// Decoded bits of one traceback lane, emitted from the highest stage down:
// bit k (relative to the item's first emitted stage) goes to bit k % 32 of
// output word (bit_off + k) / 32.  Finished words are held until the
// aligned group of four words they belong to is complete (or the chase
// ends) and then stored together, so each 16-byte piece of the output
// reaches memory in one burst instead of four partial-line writes spread
// over the whole chase.  Lanes own whole words, so the stores never
// overlap.
struct GroupEmitter {
  uint32_t word = 0;
  uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0;
  uint32_t valid = 0;  // pending words, bit i for word gbase + i
  int64_t gbase = 0;
  __device__ __forceinline__ void flush(uint32_t* bits) {
    if (valid & 1u) bits[gbase] = q0;
    if (valid & 2u) bits[gbase + 1] = q1;
    if (valid & 4u) bits[gbase + 2] = q2;
    if (valid & 8u) bits[gbase + 3] = q3;
    valid = 0;
  }
  __device__ __forceinline__ void put(int k, uint32_t u, uint32_t* bits, int64_t bit_off) {
    word |= u << (k & 31);
    if ((k & 31) == 0) {
      const int64_t w = (bit_off + k) >> 5;
      const int64_t g = w & ~(int64_t)3;
      if (valid && g != gbase) flush(bits);
      gbase = g;
      const int i = (int)(w & 3);
      q0 = i == 0 ? word : q0;
      q1 = i == 1 ? word : q1;
      q2 = i == 2 ? word : q2;
      q3 = i == 3 ? word : q3;
      valid |= 1u << i;
      word = 0;
      if (i == 0) flush(bits);
    }
  }
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

// Shift a decision into a lane's word: acc = 2*acc + d in one add-with-carry,
// the carry-in being the wave mask of the comparison.  The wait state covers
// a VALU-written SGPR read as carry by the next VALU instruction.
__device__ __forceinline__ uint32_t push_decision(uint32_t acc, uint64_t mask) {
  uint32_t out;
  uint64_t carry_out;
  asm("s_nop 1\n\tv_addc_co_u32_e64 %0, %1, %2, %2, %3"
         : "=v"(out), "=s"(carry_out)
         : "v"(acc), "s"(mask));
  return out;
}

}  // namespace mivit
