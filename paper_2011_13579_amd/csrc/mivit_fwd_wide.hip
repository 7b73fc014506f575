// Radix-2 forward procedure for K = 8 and 9 (128 and 256 states): one
// wavefront per frame, R = 2^(K-1)/64 states per lane held in registers.
//
// The state-to-position map rotates as in the K <= 7 kernel: at time t the
// state s sits at position rotl_n(s, t mod n), n = K-1, and position p is
// register p >> 6 of lane p & 63.  At stage t (phase q = t mod n) both
// previous states (Eq. (radix2:S): 2f and 2f+1) of the state at position p
// sit at the positions p with bit q cleared and set, and the new state stays
// at p.  For q < 6 that is an exchange between lanes, done for each of the R
// registers: DPP quad permutations fetch both previous metrics for bits 0
// and 1, v_permlane16/32_swap for bits 4 and 5.  For bits 2 and 3, float
// metrics stay in the VALU: a lane keeps its own previous state's metric and
// fetches its partner's (lane ^ 4: row half-mirror then quad reverse; lane ^
// 8: row rotate by 8); integer metrics fetch both through ds_swizzle, which
// measured faster for them.  For q >= 6 the two previous states are two
// registers of the same lane and nothing moves.  The R registers are independent dependency
// chains, which keeps a lone wavefront busy.
//
// Branch metrics: Eq. (BM) for the even previous state on the new state's
// input; by the corollary of §IV the odd previous state's branch has the
// opposite value.  A per-wavefront LDS table holds the 2^beta pattern values
// of each stage of a 32-stage block.
//
// Decisions: d = 1 when the odd previous state wins (strict, so a tie keeps
// the even, lower-index one).  Every position shifts its decision into a
// 32-bit word; every 32 stages its four bytes go out: per group of 8 stages, 2^(K-1) bytes, byte p
// holding position p's decisions with stage 8g + i at bit 7 - i.  A group of
// 8 stages is then 64 (K = 9) or 32 (K = 8) words, the unit the traceback
// stages through LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mivit_device.h"

namespace mivit {

namespace wide {

template <int DT>
struct Ty;
template <>
struct Ty<0> {
  static constexpr bool kInt = false;
  using T = float;
  using In = float;
  __device__ static float unreachable() { return -__builtin_inff(); }
  __device__ static int bits(float x) { return __builtin_bit_cast(int, x); }
  __device__ static float from(int x) { return __builtin_bit_cast(float, x); }
};
template <>
struct Ty<1> {
  static constexpr bool kInt = true;
  using T = int;
  using In = int8_t;
  __device__ static int unreachable() { return -(1 << 29); }
  __device__ static int bits(int x) { return x; }
  __device__ static int from(int x) { return x; }
};
template <>
struct Ty<2> : Ty<0> {
  using In = _Float16;
};

__device__ __forceinline__ int parity(uint32_t x) { return __popc(x) & 1; }

__device__ __forceinline__ int branch_out(const DevCode& c, int i, int u) {
  const uint32_t reg = ((uint32_t)u << (c.K - 1)) | (uint32_t)i;
  int w = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if (b < c.beta) w |= parity(c.gen[b] & reg) << b;
  return w;
}

__device__ __forceinline__ int rotl(int x, int r, int n) {
  return r == 0 ? x : (((x << r) | (x >> (n - r))) & ((1 << n) - 1));
}
__device__ __forceinline__ int rotr(int x, int r, int n) { return rotl(x, (n - r) % n, n); }

// Metrics of the even and odd previous states across lane bit Q (Q < 6).
template <int Q, int DT>
__device__ __forceinline__ void pair_fetch(typename Ty<DT>::T x, typename Ty<DT>::T& e,
                                           typename Ty<DT>::T& o) {
  const int xi = Ty<DT>::bits(x);
  int ei, oi;
  if constexpr (Q == 0) {
    ei = __builtin_amdgcn_mov_dpp(xi, 0xA0, 0xF, 0xF, true);  // quad_perm [0,0,2,2]
    oi = __builtin_amdgcn_mov_dpp(xi, 0xF5, 0xF, 0xF, true);  // quad_perm [1,1,3,3]
  } else if constexpr (Q == 1) {
    ei = __builtin_amdgcn_mov_dpp(xi, 0x44, 0xF, 0xF, true);  // quad_perm [0,1,0,1]
    oi = __builtin_amdgcn_mov_dpp(xi, 0xEE, 0xF, 0xF, true);  // quad_perm [2,3,2,3]
  } else if constexpr (Q <= 3) {
    // bit-mask mode within 32 lanes: lane' = (lane & and_mask) | or_mask
    ei = __builtin_amdgcn_ds_swizzle(xi, 0x1F & ~(1 << Q));
    oi = __builtin_amdgcn_ds_swizzle(xi, 0x1F | ((1 << Q) << 5));
  } else if constexpr (Q == 4) {
    // even rows of 16 to every row, odd rows to every row
    const auto r = __builtin_amdgcn_permlane16_swap(xi, xi, false, false);
    ei = r[0];
    oi = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(xi, xi, false, false);
    ei = r[0];
    oi = r[1];
  }
  e = Ty<DT>::from(ei);
  o = Ty<DT>::from(oi);
}

// Stages at lane bits 2 and 3 in own/partner form (float metrics).
template <int DT, int Q>
constexpr bool own_partner() {
  return (Q == 2 || Q == 3) && !Ty<DT>::kInt;
}

// Metric of the partner lane (lane ^ 2^Q) for Q = 2, 3.
template <int Q, int DT>
__device__ __forceinline__ typename Ty<DT>::T partner_fetch(typename Ty<DT>::T x) {
  const int xi = Ty<DT>::bits(x);
  int pi;
  if constexpr (Q == 2) {
    const int hm = __builtin_amdgcn_mov_dpp(xi, 0x141, 0xF, 0xF, true);  // row_half_mirror: ^7
    pi = __builtin_amdgcn_mov_dpp(hm, 0x1B, 0xF, 0xF, true);            // quad_perm [3,2,1,0]: ^3
  } else {
    pi = __builtin_amdgcn_mov_dpp(xi, 0x128, 0xF, 0xF, true);  // row_ror:8
  }
  return Ty<DT>::from(pi);
}

template <int DT, int R>
struct Wave {
  using T = typename Ty<DT>::T;
  T pm[R];           // metric of the state at position 64 (R w + r) + lane
  uint32_t acc[R];   // decisions of that position in the current block
  uint32_t pend[R];  // the previous block's decision words, not yet stored
  // several wavefronts per frame: LDS exchange area of the frame, the
  // number of wavefronts, this one's index w in the frame, and the exchange
  // buffer in use
  T* xch;
  int nw, fw, xb;
};

// All wavefronts of a frame at one point, LDS writes before it visible to
// LDS reads after it.  One wavefront per frame: program order suffices;
// several (kWorkgroup): the frame is the workgroup, a barrier.
template <bool kWorkgroup>
__device__ __forceinline__ void frame_sync() {
  if constexpr (!kWorkgroup) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
}


// The larger of two metrics: v_max for floats too, so that the select does
// not wait on the comparison's mask (no NaN arises: finite soft values, and
// -inf plus finite branch metrics for unreachable float states).
__device__ __forceinline__ float tmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ int tmax(int a, int b) { return a > b ? a : b; }

// push_decision for every register of a stage: one wait state pair for all
// of them (a VALU-written SGPR read as carry needs two).
template <int R>
__device__ __forceinline__ void push_decisions(uint32_t (&acc)[R], const uint64_t (&d)[R]) {
  if constexpr (R == 4) {
    uint64_t c0, c1, c2, c3;
    asm("s_nop 1\n\t"
        "v_addc_co_u32_e64 %0, %4, %0, %0, %8\n\t"
        "v_addc_co_u32_e64 %1, %5, %1, %1, %9\n\t"
        "v_addc_co_u32_e64 %2, %6, %2, %2, %10\n\t"
        "v_addc_co_u32_e64 %3, %7, %3, %3, %11"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "=s"(c0), "=s"(c1), "=s"(c2),
          "=s"(c3)
        : "s"(d[0]), "s"(d[1]), "s"(d[2]), "s"(d[3]));
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = push_decision(acc[r], d[r]);
  }
}

// One stage at phase Q; bm[r] the branch metric of position 64r + lane: of
// its even previous state, or in own/partner form of its own previous state
// (the state at position 64r + lane before the stage).  Own/partner form: the
// candidates are own + bm and partner - bm in every lane (by the corollary
// the other previous state's branch has the opposite value); the odd
// previous state won when partner > own where the lane's bit Q is 0 and
// own > partner where it is 1, strictly, so a tie keeps the even state.
template <int KM1, int DT, int R, int Q>
__device__ __forceinline__ void stage(Wave<DT, R>& W, const typename Ty<DT>::T (&bm)[R]) {
  using T = typename Ty<DT>::T;
  T nv[R];
  uint64_t d[R];  // lanes whose odd previous state won
  if constexpr (Q >= 6 && (1 << (Q - 6)) >= R) {
    // bit Q is bit wb of the wavefront index (several per frame): the
    // wavefronts with that bit clear hold the even previous states, their
    // partners (index ^ wb) the odd ones, at the same register and lane;
    // each writes its metrics to the exchange buffer and reads its partner's
    constexpr int wb = (1 << (Q - 6)) / R;
    const int lane = threadIdx.x & 63;
    const int nw = W.nw;
    T* mine = W.xch + (nw * W.xb + W.fw) * (64 * R);
    const T* theirs = W.xch + (nw * W.xb + (W.fw ^ wb)) * (64 * R);
#pragma unroll
    for (int r = 0; r < R; ++r) mine[64 * r + lane] = W.pm[r];
    frame_sync<true>();
    const bool odd = (W.fw & wb) != 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T other = theirs[64 * r + lane];
      const T e = odd ? other : W.pm[r], o = odd ? W.pm[r] : other;
      const T ce = e + bm[r], co = o - bm[r];
      nv[r] = tmax(ce, co);
      d[r] = __builtin_amdgcn_ballot_w64(co > ce);
    }
    // double buffered: the next exchange writes the other buffer, and the
    // one after it comes after a barrier that follows these reads
    W.xb ^= 1;
  } else if constexpr (own_partner<DT, Q>()) {
    // lanes with bit Q set hold the odd previous state
    constexpr uint64_t odd = Q == 2 ? 0xF0F0F0F0F0F0F0F0ull : 0xFF00FF00FF00FF00ull;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T cp = partner_fetch<Q, DT>(W.pm[r]) - bm[r];
      const T co = W.pm[r] + bm[r];
      nv[r] = tmax(cp, co);
      d[r] = (__builtin_amdgcn_ballot_w64(cp > co) & ~odd) |
             (__builtin_amdgcn_ballot_w64(co > cp) & odd);
    }
  } else if constexpr (Q < 6) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T e, o;
      pair_fetch<Q, DT>(W.pm[r], e, o);
      const T ce = e + bm[r], co = o - bm[r];
      nv[r] = tmax(ce, co);
      d[r] = __builtin_amdgcn_ballot_w64(co > ce);
    }
  } else {
    constexpr int rb = 1 << (Q - 6);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int re = r & ~rb, ro = r | rb;
      const T ce = W.pm[re] + bm[r], co = W.pm[ro] - bm[r];
      nv[r] = tmax(ce, co);
      d[r] = __builtin_amdgcn_ballot_w64(co > ce);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) W.pm[r] = nv[r];
  push_decisions<R>(W.acc, d);
}

// Branch metrics are read from LDS kPrefetch stages ahead of their use: a
// lone wavefront (the longest frame of a batch, once the others are done)
// otherwise waits out the LDS latency at every stage.
constexpr int kPrefetch = 3;

template <int KM1, int DT, int R, int NP, int P0, int K>
__device__ __forceinline__ void fetch_bm(typename Ty<DT>::T (&dst)[R],
                                         const typename Ty<DT>::T* bmt,
                                         const int (&pat)[KM1][R]) {
  constexpr int Q = (P0 + K) % KM1;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[r] = bmt[K * NP + pat[Q][r]];
}

// Stages K0..31 of a full block starting at phase P0 (static phases); q
// holds the branch metrics of stages K0 .. K0 + kPrefetch - 1.
template <int KM1, int DT, int R, int NP, int P0, int K0>
__device__ __forceinline__ void stages_full(Wave<DT, R>& W, const typename Ty<DT>::T* bmt,
                                            const int (&pat)[KM1][R],
                                            typename Ty<DT>::T (&q)[kPrefetch][R]) {
  if constexpr (K0 < 32) {
    constexpr int Q = (P0 + K0) % KM1;
    typename Ty<DT>::T bm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) bm[r] = q[K0 % kPrefetch][r];
    if constexpr (K0 + kPrefetch < 32)
      fetch_bm<KM1, DT, R, NP, P0, K0 + kPrefetch>(q[K0 % kPrefetch], bmt, pat);
    stage<KM1, DT, R, Q>(W, bm);
    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of their stages
    stages_full<KM1, DT, R, NP, P0, K0 + 1>(W, bmt, pat, q);
  }
}

template <int KM1, int DT, int R, int NP, int P0, int K>
__device__ __forceinline__ void prefetch_first(typename Ty<DT>::T (&q)[kPrefetch][R],
                                               const typename Ty<DT>::T* bmt,
                                               const int (&pat)[KM1][R]) {
  if constexpr (K < kPrefetch) {
    fetch_bm<KM1, DT, R, NP, P0, K>(q[K], bmt, pat);
    prefetch_first<KM1, DT, R, NP, P0, K + 1>(q, bmt, pat);
  }
}

// A stage whose phase is only known at run time (the last, partial block).
template <int KM1, int DT, int R, int NP, int Q>
__device__ __forceinline__ void stage_dyn(Wave<DT, R>& W, const typename Ty<DT>::T* bmrow,
                                          const int (&pat)[KM1][R], int q) {
  if constexpr (Q < KM1) {
    if (q == Q) {
      typename Ty<DT>::T bm[R];
#pragma unroll
      for (int r = 0; r < R; ++r) bm[r] = bmrow[pat[Q][r]];
      stage<KM1, DT, R, Q>(W, bm);
    } else {
      stage_dyn<KM1, DT, R, NP, Q + 1>(W, bmrow, pat, q);
    }
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

struct Ctx {
  int64_t offset;  // integer metrics: total subtracted by renormalisation
  int S, lane;     // S: one past the last stage this unit runs
  int t_store;     // first stage whose decisions are stored
  int32_t* v_start;  // split part after the first: boundary record to fill at t_store
  int64_t* m_start;
  uint8_t* pend_dst;  // where the pending decision words go, or null
  int pos0;           // first position held by this wavefront (64 R w)
};

// Store one block's decision words: four groups of 8 stages, group g of the
// block being byte 3 - g of the word.
template <int KM1, int R>
__device__ __forceinline__ void store_block(uint8_t* dst, const uint32_t (&a)[R]) {
  constexpr int NS = 1 << KM1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int g = 0; g < 4; ++g) dst[g * NS + 64 * r] = (uint8_t)(a[r] >> (24 - 8 * g));
  }
}

// One block of up to 32 stages starting at tb; BI its index in the period
// of the phase pattern.  lv: this lane's soft values of stage tb + lane
// (lanes < 32), replaced by those of the next block.
template <int KM1, int DT, int BETA, int BI, int R>
__device__ __forceinline__ void one_block(Wave<DT, R>& W, Ctx& cx, typename Ty<DT>::T* bmt,
                                          const typename Ty<DT>::In* llr,
                                          typename Ty<DT>::T (&lv)[BETA],
                                          const int (&pat)[KM1][R], uint64_t* sv, int tb) {
  using T = typename Ty<DT>::T;
  constexpr int NP = 1 << BETA;
  const int n = min(32, cx.S - tb);
  if (cx.lane < 32) {
#pragma unroll
    for (int p = 0; p < NP / 2; ++p) {
      T v = (T)0;
#pragma unroll
      for (int b = 0; b < BETA; ++b) v += ((p >> b) & 1) ? -lv[b] : lv[b];
      bmt[cx.lane * NP + p] = v;
      bmt[cx.lane * NP + (NP - 1 - p)] = -v;
    }
  }
  {
    const int t = tb + 32 + cx.lane;
    const bool ok = cx.lane < 32 && t < cx.S;
#pragma unroll
    for (int b = 0; b < BETA; ++b) lv[b] = ok ? (T)llr[(int64_t)t * BETA + b] : (T)0;
  }
  // the previous block's decisions go out here, after the next soft values
  // are requested: the memory counter the next block start waits on (for
  // those soft values) covers stores too, so stores issued at the end of a
  // block would hold up the start of the next
  if (cx.pend_dst) store_block<KM1, R>(cx.pend_dst, W.pend);
  if constexpr (Ty<DT>::kInt) {
    if (tb > 0) {
      // renormalise by the metric of state 0 (always position 0: lane 0, register 0)
      const T ref = __builtin_amdgcn_readfirstlane(W.pm[0]);
#pragma unroll
      for (int r = 0; r < R; ++r) W.pm[r] -= ref;
      cx.offset += ref;
    }
    if (cx.v_start && tb == cx.t_store) {
      // a later part of a split frame, at the end of its warm-up
#pragma unroll
      for (int r = 0; r < R; ++r) cx.v_start[64 * r + cx.lane] = (int32_t)W.pm[r];
      if (cx.lane == 0) *cx.m_start = cx.offset;
    }
  }
  wave_sync();
  constexpr int P0 = (32 * BI) % KM1;
  if (n == 32) {
    T q[kPrefetch][R];
    prefetch_first<KM1, DT, R, NP, P0, 0>(q, bmt, pat);
    stages_full<KM1, DT, R, NP, P0, 0>(W, bmt, pat, q);
  } else {
#pragma unroll 1
    for (int k = 0; k < n; ++k) stage_dyn<KM1, DT, R, NP, 0>(W, bmt + k * NP, pat, (P0 + k) % KM1);
  }
  // this block's decisions: stored at the next block's start, or after the
  // last block
  cx.pend_dst = nullptr;
  if (tb >= cx.t_store) {
    cx.pend_dst = (uint8_t*)sv + (int64_t)(tb >> 3) * (1 << KM1) + cx.pos0 + cx.lane;
#pragma unroll
    for (int r = 0; r < R; ++r) W.pend[r] = n == 32 ? W.acc[r] : W.acc[r] << (32 - n);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) W.acc[r] = 0;
  wave_sync();
}

template <int KM1, int DT, int BETA, int BI, int NB, int R>
__device__ __forceinline__ void super_block(Wave<DT, R>& W, Ctx& cx, typename Ty<DT>::T* bmt,
                                            const typename Ty<DT>::In* llr,
                                            typename Ty<DT>::T (&lv)[BETA],
                                            const int (&pat)[KM1][R], uint64_t* sv, int t0) {
  if constexpr (BI < NB) {
    const int tb = t0 + 32 * BI;
    if (tb < cx.S) {
      one_block<KM1, DT, BETA, BI, R>(W, cx, bmt, llr, lv, pat, sv, tb);
      super_block<KM1, DT, BETA, BI + 1, NB, R>(W, cx, bmt, llr, lv, pat, sv, t0);
    }
  }
}

constexpr int kWideWaves = 4;  // independent wavefronts (frames) per workgroup

}  // namespace wide

// One wavefront per unit: a whole item (frame or chunk window), or, for
// int8 soft values, one part of a frame split in time (kind 0), or a repair
// of one (kind 1, unit count read from the device).  A part after the first
// runs `warm` stages from all-zero metrics before it_begin and keeps no
// decisions from them; a part before the last leaves its end metrics in a
// boundary record, the last part its own metric, which the check completes.
//
// WPF = 2 or 4 (float metrics, whole frames only): WPF wavefronts per
// frame, a workgroup each, wavefront w holding positions 64 (R w + r) +
// lane with R = 2^(K-1) / (64 WPF); the stages whose phase is a wavefront
// bit exchange the metrics through LDS, the others run as with one
// wavefront.  A lone long frame runs its stages with 1/WPF of the
// instructions per wavefront.
template <int KM1, int DT, int BETA, int WPF>
__global__ __launch_bounds__(64 * wide::kWideWaves, 3) void k_fwd_wide(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ units, int n_units, const int32_t* dev_count, int kind,
    WideBound* bounds, int64_t* last_m, const int64_t* rep_m0,
    const void* __restrict__ llr_v, uint64_t* __restrict__ surv, void* metric,
    int32_t* end_out, int32_t* item_end) {
  using namespace wide;
  using T = typename Ty<DT>::T;
  using In = typename Ty<DT>::In;
  static_assert(WPF == 1 || ((WPF == 2 || WPF == 4) && !Ty<DT>::kInt && (1 << (KM1 - 6)) >= WPF),
                "several wavefronts per frame: float metrics, at least one register each");
  constexpr int R = (1 << (KM1 - 6)) / WPF, NS = 1 << KM1, NP = 1 << BETA;
  constexpr int FPB = WPF == 1 ? kWideWaves : 1;  // frames per workgroup
  constexpr int SUPER = 32 * KM1 / gcd_c(32, KM1);  // lcm(32, K-1)
  __shared__ T bmt_all[kWideWaves][32 * NP];
  __shared__ T xpm_all[FPB][NS];
  __shared__ T xch_all[WPF > 1 ? 2 * WPF * 64 * R : 1];
  __shared__ T red_v[WPF];
  __shared__ int red_s[WPF];
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int fw = WPF == 1 ? 0 : wid;  // wavefront within the frame
  if (dev_count) n_units = min(n_units, __builtin_amdgcn_readfirstlane(*dev_count));
  const int u = WPF == 1 ? blockIdx.x * kWideWaves + wid : blockIdx.x;
  // every wavefront of a frame leaves together: the barriers are per frame
  if (u >= n_units) return;
  const SplitUnit U = units[u];
  const Item it = items[U.first];
  const DevCode c = codes[it.code];
  const In* llr = (const In*)llr_v + it.llr_off;
  uint64_t* sv = surv + it.surv_off;
  T* bmt = bmt_all[wid];
  T* xpm = xpm_all[WPF == 1 ? wid : 0];
  const bool first_part = kind == 0 && U.part == 0;
  const bool split = U.n_parts > 1;
  const int s0 = U.it_begin - U.warm;  // a multiple of SUPER: phases start at 0

  // table offset (pattern) of position 64 (R w + r) + lane at each phase: the
  // even previous state's branch into the state held there after the stage
  int pat[KM1][R];
#pragma unroll
  for (int q = 0; q < KM1; ++q) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // the new state at position p, and the previous state whose branch
      // the stage's metric table entry gives: the even one, or in
      // own/partner form the one at p (odd when bit q of p is set)
      const int j = rotr(64 * (R * fw + r) + lane, (q + 1) % KM1, KM1);
      const bool op = (q == 2 || q == 3) && !Ty<DT>::kInt;
      const int own = op ? ((lane >> q) & 1) : 0;
      pat[q][r] = branch_out(c, ((j << 1) | own) & (NS - 1), j >> (KM1 - 1));
    }
  }
  Wave<DT, R> W;
  W.xch = xch_all;
  W.nw = WPF;
  W.fw = fw;
  W.xb = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (first_part)
      W.pm[r] = (it.start_known && (R * fw + r != 0 || lane != 0)) ? Ty<DT>::unreachable()
                                                                   : (T)0;
    else if (kind == 0)
      W.pm[r] = (T)0;  // a later part: all-zero metrics (unknown start)
    else
      W.pm[r] = Ty<DT>::from(bounds[U.bnd + U.part - 1].v_end[64 * r + lane]);  // repair
    W.acc[r] = 0;
  }
  Ctx cx{0, U.it_end, lane, U.it_begin, nullptr, nullptr, nullptr, 64 * R * fw};
  if (kind == 0 && U.part > 0) {
    cx.v_start = bounds[U.bnd + U.part - 1].v_start;
    cx.m_start = &bounds[U.bnd + U.part - 1].m_start;
  }
  T lv[BETA];
  {
    const bool ok = lane < 32 && s0 + lane < cx.S;
#pragma unroll
    for (int b = 0; b < BETA; ++b) lv[b] = ok ? (T)llr[(int64_t)(s0 + lane) * BETA + b] : (T)0;
  }
  for (int t0 = s0; t0 < cx.S; t0 += SUPER)
    super_block<KM1, DT, BETA, 0, SUPER / 32, R>(W, cx, bmt, llr, lv, pat, sv, t0);
  if (cx.pend_dst) store_block<KM1, R>(cx.pend_dst, W.pend);

  if constexpr (Ty<DT>::kInt) {
    if (kind == 0 && split && U.part < U.n_parts - 1) {
      // the end of a part before the last: range control as at a block
      // start, then the boundary record
      const T ref = __builtin_amdgcn_readfirstlane(W.pm[0]);
      WideBound& B = bounds[U.bnd + U.part];
#pragma unroll
      for (int r = 0; r < R; ++r) B.v_end[64 * r + lane] = (int32_t)(W.pm[r] - ref);
      if (lane == 0) B.m_end = cx.offset + ref;
      return;
    }
  }

  // final metrics: position p holds state rotr(p, S mod (K-1)); best state
  // with ties to the lowest index
  const int S = cx.S;
  T bv = Ty<DT>::unreachable();
  int bs = NS;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int s = rotr(64 * (R * fw + r) + lane, S % KM1, KM1);
    xpm[s] = W.pm[r];
    if (W.pm[r] > bv || (W.pm[r] == bv && s < bs)) {
      bv = W.pm[r];
      bs = s;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T ov = Ty<DT>::from(__shfl_xor(Ty<DT>::bits(bv), o));
    const int os = __shfl_xor(bs, o);
    if (ov > bv || (ov == bv && os < bs)) {
      bv = ov;
      bs = os;
    }
  }
  if constexpr (WPF > 1) {
    // the best of the wavefronts' best states, ties to the lower index
    if (lane == 0) {
      red_v[fw] = bv;
      red_s[fw] = bs;
    }
    frame_sync<(WPF > 1)>();
#pragma unroll
    for (int k = 0; k < WPF; ++k) {
      const T ov = red_v[k];
      const int os = red_s[k];
      if (ov > bv || (ov == bv && os < bs)) {
        bv = ov;
        bs = os;
      }
    }
  } else {
    frame_sync<(WPF > 1)>();
  }
  if (lane == 0 && fw == 0) {
    const int js = it.end_state >= 0 ? it.end_state : bs;
    const T vj = xpm[js];
    item_end[it.slot] = js;
    if (it.frame >= 0 && end_out) end_out[it.frame] = js;
    if constexpr (Ty<DT>::kInt) {
      const int64_t local = (int64_t)vj + cx.offset;
      if (kind == 0 && split)
        last_m[it.slot] = local;  // completed by the check
      else if (it.frame >= 0 && metric)
        ((int64_t*)metric)[it.frame] = local + (kind == 1 ? rep_m0[it.slot] : 0);
    } else {
      if (it.frame >= 0 && metric) ((float*)metric)[it.frame] = vj;
    }
  }
}

namespace wide {

// Packed 16-bit form of the int8 kernel (variant 8): two positions per
// VGPR, p = 64 (v + V h) + lane in half h of VGPR v, V = 2^(K-1) / 128.
//
// A half holds c = 2 (PM - base) + tag, the metric doubled with the tie tag
// of the stage's winner in its low bit.  Branch metrics enter biased by
// 128 beta so that every candidate is an addition: the even previous state
// adds 2 (bm + bias) + 1, the odd one 2 (-bm + bias) (its branch has the
// opposite value, the corollary of §IV).  Every path gains the bias once
// per stage, which the metric offset takes back.  The larger sum wins
// (v_pk_max_u16); among equal metrics the even state's tag 1 wins, which is
// the strict comparison with ties to the lower index, and the winner's tag
// is 1 - d.  After the add-compare-select the tag is moved into the decision
// word and cleared.
//
// Range: the metrics of a frame's states differ by at most
// 2 (K-1) 128 beta (the spread bound of integer Viterbi metrics), and every
// kPkRenorm stages the metric of state 0 is moved to `off`; in between the
// halves grow by at most 4 bias per stage.  Unreachable start states begin
// at 0, below state 0's 2 off, and lose to it within K - 1 stages.
constexpr int kPkRenorm = 16;
template <int KM1, int BETA>
struct Pk {
  static constexpr int bias = 128 * BETA;
  static constexpr int spread = 2 * KM1 * BETA * 128;
  static constexpr int off = spread + 1024;
  static_assert(2 * (off + spread) + kPkRenorm * 4 * bias + 1 < 65536, "16-bit range");
  static_assert(2 * off > KM1 * 4 * bias, "unreachable start states must lose");
};

template <int V>
struct PkWave {
  uint32_t pm[V];      // the two halves' doubled metrics, tags clear
  uint32_t acc[V];     // decisions of the current group of 8 stages (bits 0-7, 16-23)
  uint32_t blk[2][V];  // the block's finished groups, low and high halves
  uint32_t pend[2 * V];  // the previous block's decision words (positions 64 r + lane)
  int64_t off64;       // PM = c / 2 + off64
};

__device__ __forceinline__ uint32_t pk_max16(uint32_t a, uint32_t b) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_add16(uint32_t a, uint32_t b) {  // per half, mod 2^16
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}

// One stage at phase Q on candidates e + we, o + wo of every VGPR; the sums
// stay below 2^16 in each half, so 32-bit adds (which take DPP operands)
// cannot carry across.
template <int KM1, int V, int Q>
__device__ __forceinline__ void pk_stage(PkWave<V>& W, const uint32_t (&we)[V],
                                         const uint32_t (&wo)[V]) {
  uint32_t m[V];
  if constexpr (Q < 6) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      int e, o;
      pair_fetch<Q, 1>((int)W.pm[v], e, o);
      m[v] = pk_max16((uint32_t)e + we[v], (uint32_t)o + wo[v]);
    }
  } else if constexpr (Q < KM1 - 1) {
    constexpr int vb = 1 << (Q - 6);  // a VGPR bit: both previous states in the lane
#pragma unroll
    for (int v = 0; v < V; ++v) m[v] = pk_max16(W.pm[v & ~vb] + we[v], W.pm[v | vb] + wo[v]);
  } else {
    // the half bit: the low half holds the even previous state, the high
    // half the odd one, for both new states of the VGPR
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint32_t e = __builtin_amdgcn_perm(W.pm[v], W.pm[v], 0x01000100u);
      const uint32_t o = __builtin_amdgcn_perm(W.pm[v], W.pm[v], 0x03020302u);
      m[v] = pk_max16(e + we[v], o + wo[v]);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t t = m[v] & 0x00010001u;
    W.pm[v] = m[v] ^ t;
    W.acc[v] = (W.acc[v] << 1) | t;
  }
}

// A finished group of 8 stages: its byte goes below the earlier groups of
// the block (low half: acc byte 0, high half: acc byte 2).
template <int V>
__device__ __forceinline__ void pk_group(PkWave<V>& W) {
#pragma unroll
  for (int v = 0; v < V; ++v) {
    W.blk[0][v] = __builtin_amdgcn_perm(W.blk[0][v], W.acc[v], 0x06050400u);
    W.blk[1][v] = __builtin_amdgcn_perm(W.blk[1][v], W.acc[v], 0x06050402u);
    W.acc[v] = 0;
  }
}

// Range control: state 0 (low half of VGPR 0, lane 0) to 2 off.
template <int KM1, int BETA, int V>
__device__ __forceinline__ void pk_renorm(PkWave<V>& W) {
  const uint32_t ref = __builtin_amdgcn_readfirstlane(W.pm[0]) & 0xFFFFu;
  const uint32_t k = (uint32_t)(2 * Pk<KM1, BETA>::off - (int)ref) & 0xFFFFu;
#pragma unroll
  for (int v = 0; v < V; ++v) W.pm[v] = pk_add16(W.pm[v], k * 0x10001u);
  W.off64 += (int64_t)(ref >> 1) - Pk<KM1, BETA>::off;
}

template <int KM1, int BETA, int V, int P0, int K>
__device__ __forceinline__ void pk_fetch(uint32_t (&we)[V], uint32_t (&wo)[V],
                                         const uint32_t* tbl, const int (&pat)[KM1][V]) {
  constexpr int Q = (P0 + K) % KM1, NP = 1 << BETA;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    we[v] = tbl[K * 2 * NP + pat[Q][v]];
    wo[v] = tbl[K * 2 * NP + NP + pat[Q][v]];
  }
}

template <int KM1, int BETA, int V, int P0, int K0>
__device__ __forceinline__ void pk_stages_full(PkWave<V>& W, const uint32_t* tbl,
                                               const int (&pat)[KM1][V],
                                               uint32_t (&qe)[kPrefetch][V],
                                               uint32_t (&qo)[kPrefetch][V]) {
  if constexpr (K0 < 32) {
    constexpr int Q = (P0 + K0) % KM1;
    uint32_t we[V], wo[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      we[v] = qe[K0 % kPrefetch][v];
      wo[v] = qo[K0 % kPrefetch][v];
    }
    if constexpr (K0 + kPrefetch < 32)
      pk_fetch<KM1, BETA, V, P0, K0 + kPrefetch>(qe[K0 % kPrefetch], qo[K0 % kPrefetch], tbl, pat);
    pk_stage<KM1, V, Q>(W, we, wo);
    if constexpr (K0 % 8 == 7) pk_group<V>(W);
    if constexpr (K0 + 1 == kPkRenorm) pk_renorm<KM1, BETA, V>(W);
    __builtin_amdgcn_sched_barrier(0);
    pk_stages_full<KM1, BETA, V, P0, K0 + 1>(W, tbl, pat, qe, qo);
  }
}

template <int KM1, int BETA, int V, int P0, int K>
__device__ __forceinline__ void pk_prefetch(uint32_t (&qe)[kPrefetch][V],
                                            uint32_t (&qo)[kPrefetch][V], const uint32_t* tbl,
                                            const int (&pat)[KM1][V]) {
  if constexpr (K < kPrefetch) {
    pk_fetch<KM1, BETA, V, P0, K>(qe[K], qo[K], tbl, pat);
    pk_prefetch<KM1, BETA, V, P0, K + 1>(qe, qo, tbl, pat);
  }
}

template <int KM1, int BETA, int V, int Q>
__device__ __forceinline__ void pk_stage_dyn(PkWave<V>& W, const uint32_t* row,
                                             const int (&pat)[KM1][V], int q) {
  if constexpr (Q < KM1) {
    if (q == Q) {
      constexpr int NP = 1 << BETA;
      uint32_t we[V], wo[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        we[v] = row[pat[Q][v]];
        wo[v] = row[NP + pat[Q][v]];
      }
      pk_stage<KM1, V, Q>(W, we, wo);
    } else {
      pk_stage_dyn<KM1, BETA, V, Q + 1>(W, row, pat, q);
    }
  }
}

struct PkCtx {
  int S, lane, t_store;
  int32_t* v_start;  // split part after the first: boundary record to fill at t_store
  int64_t* m_start;
  uint8_t* pend_dst;
  const DevCode* code;
};

// One block of up to 32 stages starting at tb (BI: its index in the period
// of the phase pattern); lv holds this lane's soft values of stage tb + lane
// (lanes < 32) and is replaced by those of the next block.
template <int KM1, int BETA, int BI, int V>
__device__ __forceinline__ void pk_block(PkWave<V>& W, PkCtx& cx, uint32_t* tbl,
                                         const int8_t* llr, int (&lv)[BETA],
                                         const int (&pat)[KM1][V], uint64_t* sv, int tb) {
  constexpr int NP = 1 << BETA, NS = 1 << KM1, bias = Pk<KM1, BETA>::bias;
  constexpr int P0 = (32 * BI) % KM1;
  const int n = min(32, cx.S - tb);
  if (cx.lane < 32) {
    // stage tb + lane: its phase, and the pattern difference between the
    // two halves of a VGPR there (the half bit of the position flips one
    // bit b of the new state j, so bit b + 1 of the encoder register j << 1)
    const int q = (P0 + cx.lane) % KM1;
    const int b = (2 * KM1 - 2 - q) % KM1 + 1;
    int dx = 0;
#pragma unroll
    for (int i = 0; i < BETA; ++i) dx |= (int)((cx.code->gen[i] >> b) & 1u) << i;
    // bm[x] of pattern x, bh[x] of pattern x ^ dx (the soft values whose
    // bit is set in dx enter with the other sign)
    int bm[NP], bh[NP];
#pragma unroll
    for (int x = 0; x < NP / 2; ++x) {
      int sum = 0, sum_h = 0;
#pragma unroll
      for (int i = 0; i < BETA; ++i) {
        const int l = ((x >> i) & 1) ? -lv[i] : lv[i];
        sum += l;
        sum_h += ((dx >> i) & 1) ? -l : l;
      }
      bm[x] = sum;
      bm[NP - 1 - x] = -sum;
      bh[x] = sum_h;
      bh[NP - 1 - x] = -sum_h;
    }
    uint32_t* row = tbl + cx.lane * 2 * NP;
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      row[x] = (uint32_t)(2 * (bm[x] + bias) + 1) | ((uint32_t)(2 * (bh[x] + bias) + 1) << 16);
      row[NP + x] = (uint32_t)(2 * (bias - bm[x])) | ((uint32_t)(2 * (bias - bh[x])) << 16);
    }
  }
  {
    const int t = tb + 32 + cx.lane;
    const bool ok = cx.lane < 32 && t < cx.S;
#pragma unroll
    for (int i = 0; i < BETA; ++i) lv[i] = ok ? (int)llr[(int64_t)t * BETA + i] : 0;
  }
  if (cx.pend_dst) store_block<KM1, 2 * V>(cx.pend_dst, W.pend);
  if (tb > 0) pk_renorm<KM1, BETA, V>(W);
  if (cx.v_start && tb == cx.t_store) {
    // a later part of a split frame, at the end of its warm-up
#pragma unroll
    for (int v = 0; v < V; ++v) {
      cx.v_start[64 * v + cx.lane] = (int32_t)(W.pm[v] & 0xFFFFu) / 2 - Pk<KM1, BETA>::off;
      cx.v_start[64 * (v + V) + cx.lane] = (int32_t)(W.pm[v] >> 16) / 2 - Pk<KM1, BETA>::off;
    }
    if (cx.lane == 0) *cx.m_start = W.off64 + Pk<KM1, BETA>::off;
  }
  // every candidate carries the bias once per stage: the block's total
  W.off64 -= (int64_t)bias * n;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    W.acc[v] = 0;
    W.blk[0][v] = 0;
    W.blk[1][v] = 0;
  }
  wave_sync();
  if (n == 32) {
    uint32_t qe[kPrefetch][V], qo[kPrefetch][V];
    pk_prefetch<KM1, BETA, V, P0, 0>(qe, qo, tbl, pat);
    pk_stages_full<KM1, BETA, V, P0, 0>(W, tbl, pat, qe, qo);
  } else {
#pragma unroll 1
    for (int k = 0; k < n; ++k) {
      pk_stage_dyn<KM1, BETA, V, 0>(W, tbl + k * 2 * NP, pat, (P0 + k) % KM1);
      if ((k & 7) == 7) pk_group<V>(W);
      if (k + 1 == kPkRenorm && n > kPkRenorm) pk_renorm<KM1, BETA, V>(W);
    }
    if (n & 7) {
      // the last, partial group: its first stage to bit 7 of the byte
      const int sh = 8 - (n & 7);
#pragma unroll
      for (int v = 0; v < V; ++v) W.acc[v] <<= sh;
      pk_group<V>(W);
    }
  }
  // this block's decision words, group g in byte 3 - g, the tags inverted
  // into decisions, stages past the block's end zero; stored at the next
  // block's start or after the last block
  cx.pend_dst = nullptr;
  if (tb >= cx.t_store) {
    const int groups = (n + 7) >> 3;
    const uint32_t valid = n == 32 ? 0xFFFFFFFFu : ~(0xFFFFFFFFu >> n);
    cx.pend_dst = (uint8_t*)sv + (int64_t)(tb >> 3) * NS + cx.lane;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const uint32_t w = groups == 4 ? W.blk[h][v] : W.blk[h][v] << (8 * (4 - groups));
        W.pend[V * h + v] = ~w & valid;
      }
    }
  }
  wave_sync();
}

template <int KM1, int BETA, int BI, int NB, int V>
__device__ __forceinline__ void pk_super(PkWave<V>& W, PkCtx& cx, uint32_t* tbl,
                                         const int8_t* llr, int (&lv)[BETA],
                                         const int (&pat)[KM1][V], uint64_t* sv, int t0) {
  if constexpr (BI < NB) {
    const int tb = t0 + 32 * BI;
    if (tb < cx.S) {
      pk_block<KM1, BETA, BI, V>(W, cx, tbl, llr, lv, pat, sv, tb);
      pk_super<KM1, BETA, BI + 1, NB, V>(W, cx, tbl, llr, lv, pat, sv, t0);
    }
  }
}

}  // namespace wide

// The packed form of the int8 kernel for kind 0 units (whole items or parts
// of split frames; repairs run the 32-bit kernel, whose decisions and
// records are the same).  Outputs as k_fwd_wide's.
template <int KM1, int BETA>
__global__ __launch_bounds__(64 * wide::kWideWaves, 3) void k_fwd_wpk(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ units, int n_units, WideBound* bounds, int64_t* last_m,
    const int8_t* __restrict__ llr_all, uint64_t* __restrict__ surv, int64_t* metric,
    int32_t* end_out, int32_t* item_end) {
  using namespace wide;
  using P = Pk<KM1, BETA>;
  constexpr int V = (1 << (KM1 - 6)) / 2, NS = 1 << KM1, NP = 1 << BETA;
  constexpr int SUPER = 32 * KM1 / gcd_c(32, KM1);  // lcm(32, K-1)
  static_assert(SUPER % kPkRenorm == 0, "range control at fixed stages of the period");
  __shared__ uint32_t tbl_all[kWideWaves][32 * 2 * NP];
  __shared__ int32_t xpm_all[kWideWaves][NS];
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int u = blockIdx.x * kWideWaves + wid;
  if (u >= n_units) return;  // no workgroup barriers: safe to leave
  const SplitUnit U = units[u];
  const Item it = items[U.first];
  const DevCode c = codes[it.code];
  const int8_t* llr = llr_all + it.llr_off;
  uint64_t* sv = surv + it.surv_off;
  uint32_t* tbl = tbl_all[wid];
  int32_t* xpm = xpm_all[wid];
  const bool split = U.n_parts > 1;
  const int s0 = U.it_begin - U.warm;  // a multiple of SUPER: phases start at 0

  // table offset (pattern) of the low position 64 v + lane of each VGPR at
  // each phase: the even previous state's branch into the new state there
  int pat[KM1][V];
#pragma unroll
  for (int q = 0; q < KM1; ++q) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = rotr(64 * v + lane, (q + 1) % KM1, KM1);
      pat[q][v] = branch_out(c, (j << 1) & (NS - 1), j >> (KM1 - 1));
    }
  }
  PkWave<V> W;
  const uint32_t all = (uint32_t)(2 * P::off) * 0x10001u;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    // a known start: state 0 (low half of VGPR 0, lane 0) at 2 off, the
    // others unreachable at 0; else (and for later parts) all at 2 off
    W.pm[v] = (U.part == 0 && it.start_known) ? ((v == 0 && lane == 0) ? (uint32_t)(2 * P::off) : 0u)
                                               : all;
  }
  W.off64 = -(int64_t)P::off;
  PkCtx cx{U.it_end, lane, U.it_begin, nullptr, nullptr, nullptr, &c};
  if (U.part > 0) {
    cx.v_start = bounds[U.bnd + U.part - 1].v_start;
    cx.m_start = &bounds[U.bnd + U.part - 1].m_start;
  }
  int lv[BETA];
  {
    const bool ok = lane < 32 && s0 + lane < cx.S;
#pragma unroll
    for (int i = 0; i < BETA; ++i) lv[i] = ok ? (int)llr[(int64_t)(s0 + lane) * BETA + i] : 0;
  }
  for (int t0 = s0; t0 < cx.S; t0 += SUPER)
    pk_super<KM1, BETA, 0, SUPER / 32, V>(W, cx, tbl, llr, lv, pat, sv, t0);
  if (cx.pend_dst) store_block<KM1, 2 * V>(cx.pend_dst, W.pend);

  if (split && U.part < U.n_parts - 1) {
    // the end of a part before the last: range control relative to state 0,
    // then the boundary record
    const int32_t ref = (int32_t)(__builtin_amdgcn_readfirstlane(W.pm[0]) & 0xFFFFu) / 2;
    WideBound& B = bounds[U.bnd + U.part];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      B.v_end[64 * v + lane] = (int32_t)(W.pm[v] & 0xFFFFu) / 2 - ref;
      B.v_end[64 * (v + V) + lane] = (int32_t)(W.pm[v] >> 16) / 2 - ref;
    }
    if (lane == 0) B.m_end = W.off64 + ref;
    return;
  }

  // final metrics: position p holds state rotr(p, S mod (K-1)); best state
  // with ties to the lowest index
  const int S = cx.S;
  int bv = -(1 << 30);
  int bs = NS;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int s = rotr(64 * (v + V * h) + lane, S % KM1, KM1);
      const int val = (int)((h ? W.pm[v] >> 16 : W.pm[v] & 0xFFFFu) >> 1) - P::off;
      xpm[s] = val;
      if (val > bv || (val == bv && s < bs)) {
        bv = val;
        bs = s;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int ov = __shfl_xor(bv, o);
    const int os = __shfl_xor(bs, o);
    if (ov > bv || (ov == bv && os < bs)) {
      bv = ov;
      bs = os;
    }
  }
  wave_sync();
  if (lane == 0) {
    const int js = it.end_state >= 0 ? it.end_state : bs;
    item_end[it.slot] = js;
    if (it.frame >= 0 && end_out) end_out[it.frame] = js;
    const int64_t local = (int64_t)xpm[js] + W.off64 + P::off;
    if (split)
      last_m[it.slot] = local;  // completed by the check
    else if (it.frame >= 0 && metric)
      metric[it.frame] = local;
  }
}

// The check after a split forward pass of the K = 8, 9 kernel, one wavefront
// per split frame (its part-0 unit): boundary k is exact when part k's
// range-controlled metrics at its end equal part k+1's after its warm-up at
// every position; then the metric is the last part's plus the accumulated
// constants, else a repair unit restarts the frame at the first inexact
// boundary from the true metrics.
__global__ __launch_bounds__(64 * wide::kWideWaves) void k_wide_check(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ split, int n_split,
    const WideBound* __restrict__ bounds, const int64_t* __restrict__ last_m, int64_t* rep_m0,
    SplitUnit* rep_units, int32_t* rep_count, int64_t* metric) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * wide::kWideWaves + (threadIdx.x >> 6);
  if (e >= n_split) return;
  const SplitUnit U = split[e];
  const Item it = items[U.first];
  const int NS = 1 << (codes[it.code].K - 1);  // positions compared
  const int n_b = U.n_parts - 1;
  int64_t T = bounds[U.bnd].m_end;  // part 0 is exact
  int64_t D = 0;
  int fail = -1;
  for (int b = 0; b < n_b; ++b) {
    const WideBound& B = bounds[U.bnd + b];
    bool diff = false;
    for (int p = lane; p < NS; p += 64) diff = diff || (B.v_end[p] != B.v_start[p]);
    if (__ballot(diff) != 0) {
      fail = b;
      break;
    }
    D = T - B.m_start;
    if (b + 1 < n_b) T = bounds[U.bnd + b + 1].m_end + D;
  }
  if (lane != 0) return;
  if (fail < 0) {
    if (metric && it.frame >= 0) metric[it.frame] = last_m[it.slot] + D;
    return;
  }
  rep_m0[it.slot] = T;
  SplitUnit R = U;
  R.it_begin = bounds[U.bnd + fail].it_at;
  R.it_end = it.n_stages;
  R.warm = 0;
  R.part = fail + 1;
  rep_units[atomicAdd(rep_count, 1)] = R;
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st);

hipError_t launch_fwd_wide(int K, int beta, int dt, int wpf, bool packed, const DevCode* codes,
                           const Item* items,
                           const SplitUnit* units, int n_units, const void* llr, uint64_t* surv,
                           void* metric, int32_t* end_out, int32_t* item_end, WideBound* bounds,
                           int64_t* last_m, const SplitUnit* split, int n_split, int64_t* rep_m0,
                           SplitUnit* rep_units, int32_t* rep_count, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  if (n_split > 0 && dt != 1) return hipErrorInvalidValue;  // split frames: int8 only
  if (wpf != 1 && ((wpf != 2 && !(wpf == 4 && K == 9)) || dt != 0)) return hipErrorInvalidValue;
  if (packed && (dt != 1 || wpf != 1 || beta > 3)) return hipErrorInvalidValue;
  const dim3 block(64 * wide::kWideWaves);
  const dim3 grid((n_units + wide::kWideWaves - 1) / wide::kWideWaves);
  if (wpf > 1) {  // float32 whole frames: a workgroup of wpf wavefronts per frame
#define MV_WIDE2(KM1, B, W)                                                                      \
  hipLaunchKernelGGL((k_fwd_wide<KM1, 0, B, W>), dim3(n_units), dim3(64 * W), 0, st, codes,      \
                     items, units, n_units, (const int32_t*)nullptr, 0, bounds, last_m,          \
                     (const int64_t*)nullptr, llr, surv, metric, end_out, item_end);             \
  return hipGetLastError()
    switch (K * 64 + beta * 8 + wpf) {
      case 8 * 64 + 2 * 8 + 2: MV_WIDE2(7, 2, 2);
      case 8 * 64 + 3 * 8 + 2: MV_WIDE2(7, 3, 2);
      case 8 * 64 + 4 * 8 + 2: MV_WIDE2(7, 4, 2);
      case 9 * 64 + 2 * 8 + 2: MV_WIDE2(8, 2, 2);
      case 9 * 64 + 3 * 8 + 2: MV_WIDE2(8, 3, 2);
      case 9 * 64 + 4 * 8 + 2: MV_WIDE2(8, 4, 2);
      case 9 * 64 + 2 * 8 + 4: MV_WIDE2(8, 2, 4);
      case 9 * 64 + 3 * 8 + 4: MV_WIDE2(8, 3, 4);
      case 9 * 64 + 4 * 8 + 4: MV_WIDE2(8, 4, 4);
      default: return hipErrorInvalidValue;
    }
#undef MV_WIDE2
  }
  const dim3 grid_rep((n_split + wide::kWideWaves - 1) / wide::kWideWaves);
  hipError_t e = hipSuccess;
#define MV_WIDE(KM1, D, B)                                                                       \
  do {                                                                                           \
    if constexpr (D == 1 && B <= 3) {                                                             \
      if (packed)                                                                                 \
        hipLaunchKernelGGL((k_fwd_wpk<KM1, B>), grid, block, 0, st, codes, items, units, n_units, \
                           bounds, last_m, (const int8_t*)llr, surv, (int64_t*)metric, end_out,    \
                           item_end);                                                             \
    }                                                                                             \
    if (!packed)                                                                                  \
      hipLaunchKernelGGL((k_fwd_wide<KM1, D, B, 1>), grid, block, 0, st, codes, items, units,     \
                         n_units, (const int32_t*)nullptr, 0, bounds, last_m,                     \
                         (const int64_t*)nullptr, llr,                                            \
                         surv, metric, end_out, item_end);                                        \
    e = hipGetLastError();                                                                        \
    if (e != hipSuccess || n_split <= 0) return e;                                                \
    e = launch_zero_i32(rep_count, 1, st);                                                        \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL(k_wide_check, grid_rep, block, 0, st, codes, items, split, n_split,        \
                       (const WideBound*)bounds, (const int64_t*)last_m, rep_m0, rep_units,       \
                       rep_count, (int64_t*)metric);                                              \
    e = hipGetLastError();                                                                        \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL((k_fwd_wide<KM1, D, B, 1>), grid_rep, block, 0, st, codes, items,         \
                       (const SplitUnit*)rep_units, n_split, (const int32_t*)rep_count, 1, bounds,\
                       last_m, (const int64_t*)rep_m0, llr, surv, metric, end_out, item_end);     \
    return hipGetLastError();                                                                     \
  } while (0)
#define MV_WIDE_B(KM1, D)             \
  switch (beta) {                     \
    case 2: MV_WIDE(KM1, D, 2);       \
    case 3: MV_WIDE(KM1, D, 3);       \
    case 4: MV_WIDE(KM1, D, 4);       \
    default: return hipErrorInvalidValue; \
  }
#define MV_WIDE_D(KM1)                \
  switch (dt) {                       \
    case 0: MV_WIDE_B(KM1, 0);        \
    case 1: MV_WIDE_B(KM1, 1);        \
    case 2: MV_WIDE_B(KM1, 2);        \
    default: return hipErrorInvalidValue; \
  }
  switch (K) {
    case 8: MV_WIDE_D(7);
    case 9: MV_WIDE_D(8);
    default: return hipErrorInvalidValue;
  }
#undef MV_WIDE_D
#undef MV_WIDE_B
#undef MV_WIDE
}

}  // namespace mivit
