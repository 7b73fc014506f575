// Parallel traceback (Algorithm 2) of one trellis per wavefront.
//
// The emitted stages of an item are cut into at most 64 segments of L stages
// (L a multiple of 32, so every segment owns whole output words).  Lane g
// traces segment g.  The lane whose chase reaches the item's last stage
// starts from the true final state and is exact.  Every other lane starts
// `warm` stages above its segment from a guessed state; survivor paths merge
// quickly going backwards, so it usually meets the true path before reaching
// its segment.  Exactness does not rest on that: lane g records the state y_g
// it passes at its segment's upper boundary and its final state x_g at the
// lower boundary.  When y_g equals x_{g+1} of the lane above (itself exact),
// lane g followed the true path through its whole segment.  A ballot finds
// the lanes where this fails; they trace again from x_{g+1} and the check
// repeats, at most G times, until every boundary agrees.
//
// Survivor words are read one block (64 words) per lane at a time.  All lanes
// advance block by block in lockstep rounds; the blocks of the next round are
// streamed by the lanes straight into the other half of a double-buffered LDS
// area (global_load_lds, no register staging) while the current round is
// chased.  In buffer k, word w of lane l sits at ((k*16 + w/4)*64 + l)*4 +
// w%4, the layout one 16-byte global_load_lds per lane and chunk produces.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mivit_device.h"

namespace mivit {

// survivor layouts
enum : int {
  kLayoutNatR2 = 0,  // per stage, ceil(NS/64) uint64 words, bit j = decision of state j
  kLayoutNatR4 = 1,  // same words; stage pairs (t, t+1) from 0 hold bits 0 and 1 of y
  kLayoutNatR8 = 5,  // same words; stage triples (t, t+1, t+2) from 0 hold bits 0..2 of y,
                     // the S mod 3 last stages radix-2 decisions
  kLayoutRotR2 = 2,  // per 32 stages, NS uint32 words; rotating state-to-word map
  kLayoutRotByte = 4,  // per 8 stages, NS bytes: byte p = decisions at position p (stage
                       // 8g + i at bit 7 - i); the state j after stage t is at position
                       // rotl(j, (t+1) mod (K-1))
};

template <int LAYOUT>
struct TbGeom {
  int K, KM1, NS, W;  // W: uint64 words per stage (natural layouts)
  int SB;             // stages per block
  int WB;             // uint32 words per block
  __device__ TbGeom(int K_) : K(K_), KM1(K_ - 1), NS(1 << (K_ - 1)) {
    W = words_per_stage(K_);
    if (LAYOUT == kLayoutRotR2) {
      SB = 32;
      WB = NS;
    } else if (LAYOUT == kLayoutRotByte) {
      SB = 2048 / NS;  // 64 words of NS / 4 words per 8 stages
      WB = 64;
    } else if (LAYOUT == kLayoutNatR8) {
      SB = (32 / W) / 3 * 3;  // whole triples per block: 30, 15 or 6 stages
      WB = SB * 2 * W;
    } else {
      SB = 32 / W;
      WB = 64;
    }
  }
};

// Rotating radix-2 layout: the chase holds the state as the byte offset, in
// a staged buffer, of the word of its position p: (p >> 2) * 1024 +
// (p & 3) * 4 (plus the lane's 16-byte slot).  Position bit q is offset bit
// pos_bit(q).
__device__ __forceinline__ int pos_off(int p) { return ((p >> 2) << 10) | ((p & 3) << 2); }
__device__ __forceinline__ int pos_bit(int q) { return q < 2 ? q + 2 : q + 8; }

__device__ __forceinline__ int rotl_bits(int x, int r, int n) {
  // rotate the n-bit value x left by r (0 <= r < n)
  return ((x << r) | (x >> (n - r))) & ((1 << n) - 1);
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Stream this lane's 64-word block starting at src into LDS buffer buf_k
// (for the lanes currently active).  Always 64 words: a block of fewer words
// is followed by more survivor words or by the allocation's padding.
__device__ __forceinline__ void fetch_block(const uint32_t* src, uint32_t* buf_k) {
#pragma unroll
  for (int c = 0; c < 16; ++c)
    __builtin_amdgcn_global_load_lds((const void*)(src + 4 * c), (lds_ptr_t)(buf_k + c * 256),
                                     16, 0, 0);
}

__device__ __forceinline__ uint32_t word_at(const uint32_t* buf_k, int w, int lane) {
  return buf_k[((w >> 2) * 64 + lane) * 4 + (w & 3)];
}

// Per-lane chase state.  Times are stage boundaries: time t is the state
// entering stage t.  In the rotating layouts the states j, x, y are held as
// the state's position at that time (radix 2: as its offset, pos_off), which
// compare like states at one time.  In the natural radix-4 layout the decisions of a stage
// pair (2k, 2k+1) only name the state two stages back, so states are known
// (and compared between segments) at pair-aligned times: even times and S.
// In the radix-8 layout they are the multiples of 3 and the times of the
// radix-2 stages at the end.
struct Chase {
  int top, a, b;  // from time top down to time a; bits of [a, b) are emitted
  int j;          // current state
  int xa, yb;     // pair-aligned times at or above a and b
  int x, y;       // states at times xa and yb
};

// All lanes with go set chase their range; the others idle.  Returns with
// c.j = state where the chase ended, c.x and c.y set.
template <int LAYOUT>
__device__ __forceinline__ void chase_all(const TbGeom<LAYOUT>& g, const uint32_t* __restrict__ sv,
                                          uint32_t* lds, Chase& c, bool go, int ob, int S,
                                          uint32_t* bits, int64_t bit_off) {
  const int lane = threadIdx.x;
  const int SB = g.SB, WB = g.WB;
  GroupEmitter em;
  if (go && c.top == c.yb) c.y = c.j;
  if (go && c.top == c.xa) c.x = c.j;
  const int B0 = go ? (c.top - 1) / SB : 0;
  const int nb = go ? B0 - c.a / SB + 1 : 0;
  int t = c.top - 1;  // next stage to step over
  // rotating layouts: rotation (t + 1) mod (K-1) of the positions, stepped
  // down with t (no division in the chase)
  int rot = (go && (LAYOUT == kLayoutRotR2 || LAYOUT == kLayoutRotByte)) ? c.top % g.KM1 : 0;
  if (nb > 0) fetch_block(sv + (int64_t)B0 * WB, lds);
  for (int r = 0;; ++r) {
    if (__ballot(r < nb) == 0) break;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    uint32_t* cur = lds + (r & 1) * 4096;
    uint32_t* nxt = lds + ((r + 1) & 1) * 4096;
    if (r + 1 < nb) fetch_block(sv + (int64_t)(B0 - r - 1) * WB, nxt);
    if (r < nb) {
      const int B = B0 - r;
      const int t0 = B * SB;  // first stage of the block: t - t0 = t mod SB
      int j = c.j;
      if (LAYOUT == kLayoutNatR4) {
        if ((S & 1) && t == S - 1 && t >= t0) {
          // odd stage count: the last stage was a radix-2 stage
          const int w = (t - t0) * 2 * g.W + (j >> 5);
          const int d = (word_at(cur, w, lane) >> (j & 31)) & 1;
          if (t >= c.a && t < c.b) em.put(t - ob, (uint32_t)(j >> (g.KM1 - 1)), bits, bit_off);
          j = ((j << 1) | d) & (g.NS - 1);
          if (t == c.yb) c.y = j;
          if (t == c.xa) c.x = j;
          --t;
        }
        // pairs (t-1, t), t odd; pairs never straddle a block
        for (; t > t0 && t >= c.a; t -= 2) {
          const int w0 = (t - 1 - t0) * 2 * g.W + (j >> 5);
          const int w1 = (t - t0) * 2 * g.W + (j >> 5);
          const int yy = ((word_at(cur, w0, lane) >> (j & 31)) & 1) |
                         (((word_at(cur, w1, lane) >> (j & 31)) & 1) << 1);
          if (t < c.b) em.put(t - ob, (uint32_t)(j >> (g.KM1 - 1)), bits, bit_off);
          if (t - 1 >= c.a && t - 1 < c.b)
            em.put(t - 1 - ob, (uint32_t)((j >> (g.KM1 - 2)) & 1), bits, bit_off);
          j = 4 * (j & ((g.NS >> 2) - 1)) + yy;
          if (t - 1 == c.yb) c.y = j;
          if (t - 1 == c.xa) c.x = j;
        }
      } else if (LAYOUT == kLayoutNatR8) {
        // the S mod 3 last stages were radix-2 stages
        for (; t >= S - S % 3 && t >= t0 && t >= c.a; --t) {
          const int w = (t - t0) * 2 * g.W + (j >> 5);
          const int d = (word_at(cur, w, lane) >> (j & 31)) & 1;
          if (t < c.b) em.put(t - ob, (uint32_t)(j >> (g.KM1 - 1)), bits, bit_off);
          j = ((j << 1) | d) & (g.NS - 1);
          if (t == c.yb) c.y = j;
          if (t == c.xa) c.x = j;
        }
        // triples (t-2, t-1, t), t = 2 mod 3; triples never straddle a block
        for (; t >= t0 + 2 && t >= c.a; t -= 3) {
          const int sh = j & 31;
          const int w2 = (t - t0) * 2 * g.W + (j >> 5);
          const int w1 = w2 - 2 * g.W, w0 = w1 - 2 * g.W;
          const int yy = ((word_at(cur, w0, lane) >> sh) & 1) |
                         (((word_at(cur, w1, lane) >> sh) & 1) << 1) |
                         (((word_at(cur, w2, lane) >> sh) & 1) << 2);
          if (t < c.b) em.put(t - ob, (uint32_t)(j >> (g.KM1 - 1)), bits, bit_off);
          if (t - 1 >= c.a && t - 1 < c.b)
            em.put(t - 1 - ob, (uint32_t)((j >> (g.KM1 - 2)) & 1), bits, bit_off);
          if (t - 2 >= c.a && t - 2 < c.b)
            em.put(t - 2 - ob, (uint32_t)((j >> (g.KM1 - 3)) & 1), bits, bit_off);
          j = 8 * (j & ((g.NS >> 3) - 1)) + yy;
          if (t - 2 == c.yb) c.y = j;
          if (t - 2 == c.xa) c.x = j;
        }
      } else if (LAYOUT == kLayoutRotR2) {
        // j: position offset at time t + 1.  Stepping over stage t replaces
        // position bit t mod (K-1) by the decision (the predecessor's
        // position); that bit held the stage's decoded input bit.
        const char* cl = (const char*)cur + lane * 16;
        const int lo = max(c.a, t0);
        for (; t >= lo; --t) {
          const int q = rot == 0 ? g.KM1 - 1 : rot - 1;  // t mod (K-1)
          const int a = pos_bit(q);
          const uint32_t word = *(const uint32_t*)(cl + j);
          const int d = (int)((word >> (31 - (t & 31))) & 1u);
          if (t < c.b) em.put(t - ob, (uint32_t)((j >> a) & 1), bits, bit_off);
          j = (j & ~(1 << a)) | (d << a);
          if (t == c.yb) c.y = j;
          if (t == c.xa) c.x = j;
          rot = q;
        }
      } else if (LAYOUT == kLayoutRotByte) {
        // j: position at time t + 1 (as for the rotating radix-2 layout,
        // a step replaces position bit t mod (K-1) by the decision)
        const int lo = max(c.a, t0);
        for (; t >= lo; --t) {
          const int q = rot == 0 ? g.KM1 - 1 : rot - 1;  // t mod (K-1)
          const int w = ((t - t0) >> 3) * (g.NS >> 2) + (j >> 2);
          const int d = (word_at(cur, w, lane) >> (8 * (j & 3) + 7 - (t & 7))) & 1;
          if (t < c.b) em.put(t - ob, (uint32_t)((j >> q) & 1), bits, bit_off);
          j = (j & ~(1 << q)) | (d << q);
          if (t == c.yb) c.y = j;
          if (t == c.xa) c.x = j;
          rot = q;
        }
      } else {
        const int lo = max(c.a, t0);
        for (; t >= lo; --t) {
          const int w = (t - t0) * 2 * g.W + (j >> 5);
          const int d = (word_at(cur, w, lane) >> (j & 31)) & 1;
          if (t < c.b) em.put(t - ob, (uint32_t)(j >> (g.KM1 - 1)), bits, bit_off);
          j = ((j << 1) | d) & (g.NS - 1);
          if (t == c.yb) c.y = j;
          if (t == c.xa) c.x = j;
        }
      }
      c.j = j;
    }
  }
  em.flush(bits);
}

template <int LAYOUT>
__global__ __launch_bounds__(64) void k_tb_seg(const DevCode* __restrict__ codes,
                                               const Item* __restrict__ items,
                                               const uint64_t* __restrict__ surv,
                                               const int32_t* __restrict__ item_end,
                                               uint32_t* __restrict__ bits, int warm) {
  __shared__ uint32_t lds[2 * 4096];
  const Item it = items[blockIdx.x];
  if (it.n_out <= 0) return;
  const DevCode code = codes[it.code];
  const TbGeom<LAYOUT> g(code.K);
  const int lane = threadIdx.x;
  const uint32_t* sv = (const uint32_t*)(surv + it.surv_off);
  const int S = it.n_stages, ob = it.out_begin, n = it.n_out;
  // the next time at or above t where states are known (every time for
  // radix 2; even times and S for radix 4; multiples of 3 and the times from
  // S - S mod 3 on for radix 8)
  auto align = [&](int t) {
    if (LAYOUT == kLayoutNatR4) return ((t & 1) && t < S) ? t + 1 : t;
    if (LAYOUT == kLayoutNatR8) return (t % 3 && t < S - S % 3) ? t + 3 - t % 3 : t;
    return t;
  };
  // segment geometry: G segments of L stages, L a multiple of 32
  int G = min(64, (n + 31) / 32);
  const int L = (((n + G - 1) / G) + 31) & ~31;
  G = (n + L - 1) / L;
  const bool active = lane < G;
  Chase c;
  c.a = ob + lane * L;
  c.b = min(ob + (lane + 1) * L, ob + n);
  c.xa = align(c.a);
  c.yb = align(c.b);
  c.top = active ? ((lane == G - 1) ? S : min(S, align(c.b + warm))) : c.a;
  const bool exact = active && c.top == S;
  c.j = exact ? item_end[it.slot] : 0;
  // rotating layouts chase positions: the state's at time S
  if (LAYOUT == kLayoutRotByte && exact) c.j = rotl_bits(c.j, S % g.KM1, g.KM1);
  if (LAYOUT == kLayoutRotR2 && exact) c.j = pos_off(rotl_bits(c.j, S % g.KM1, g.KM1));
  // mask of the state bits (of the offset bits for the rotating radix-2 layout)
  const int state_mask = LAYOUT == kLayoutRotR2 ? pos_off(g.NS - 1) : g.NS - 1;
  c.x = c.y = -1;
  chase_all<LAYOUT>(g, sv, lds, c, active && c.top > c.a, ob, S, bits, it.bit_off);
  // repair rounds: lane g is right when its state at yb equals lane g+1's
  // state at its xa (the same time)
  for (int round = 0; round <= G; ++round) {
    const int x_up = __shfl_down(c.x, 1) & state_mask;
    const bool bad = active && !exact && lane < G - 1 && c.y != x_up;
    if (__ballot(bad) == 0) break;
    // lanes that agree with their neighbour stay idle this round
    Chase r = c;
    r.top = c.yb;
    r.j = x_up;
    chase_all<LAYOUT>(g, sv, lds, r, bad, ob, S, bits, it.bit_off);
    if (bad) {
      c.j = r.j;
      c.x = r.x;
      c.y = x_up;
    }
  }
}

hipError_t launch_tb_seg(int layout, const DevCode* codes, const Item* items, int n_items,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits,
                         int warm, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items), block(64);
  switch (layout) {
    case kLayoutNatR2:
      hipLaunchKernelGGL(k_tb_seg<kLayoutNatR2>, grid, block, 0, st, codes, items, surv,
                         item_end, bits, warm);
      break;
    case kLayoutNatR4:
      hipLaunchKernelGGL(k_tb_seg<kLayoutNatR4>, grid, block, 0, st, codes, items, surv,
                         item_end, bits, warm);
      break;
    case kLayoutNatR8:
      hipLaunchKernelGGL(k_tb_seg<kLayoutNatR8>, grid, block, 0, st, codes, items, surv,
                         item_end, bits, warm);
      break;
    case kLayoutRotR2:
      hipLaunchKernelGGL(k_tb_seg<kLayoutRotR2>, grid, block, 0, st, codes, items, surv,
                         item_end, bits, warm);
      break;
    case kLayoutRotByte:
      hipLaunchKernelGGL(k_tb_seg<kLayoutRotByte>, grid, block, 0, st, codes, items, surv,
                         item_end, bits, warm);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mivit
