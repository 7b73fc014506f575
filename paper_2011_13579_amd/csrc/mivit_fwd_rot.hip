// Radix-2 forward procedure for K <= 7 with a rotating state-to-lane map.
//
// Eq. (radix2:S) pairs the previous states 2f and 2f+1 (differing in their
// LSB) into the states f and f + 2^(K-2) (differing in their MSB).  With n =
// K-1 state bits, let the state s live in lane rotl_n(s, t mod n) at time t.
// Then at stage t both previous states of the state in lane l sit in lanes
// l with bit (t mod n) cleared and set, and the new state stays in lane l: a
// butterfly is an exchange between two lanes that differ in one lane bit, and
// no data moves otherwise.  Lane bits 0 and 1 are exchanged with DPP
// quad permutations fused into the adds, bits 2..4 with ds_swizzle, bit 5
// with ds_bpermute.
//
// Branch metrics: by the corollary of §IV (MSB and LSB taps set) the two
// branches into a state carry opposite metrics, delta(2f+1 -> j) =
// -delta(2f -> j), so each lane reads one value per stage from a per-frame
// LDS table of Eq. (BM) over the 2^beta output patterns.
//
// Decisions: d = 1 when the odd previous state wins (strict comparison, so a
// tie keeps the even, lower-index one).  Each lane shifts its decision into a
// 32-bit word (bit 31 - (t mod 32) holds stage t); every 32 stages the words
// of a frame's lanes are stored together, word index = lane.
//
// One wavefront runs 64/2^(K-1) frames of equal length side by side.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mivit_device.h"

namespace mivit {

namespace rot {

__device__ __forceinline__ int parity(uint32_t x) { return __popc(x) & 1; }

__device__ __forceinline__ int branch_out(const DevCode& c, int i, int u) {
  uint32_t reg = ((uint32_t)u << (c.K - 1)) | (uint32_t)i;
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

// Soft-value type DT (0: float32, 1: int8, 2: float16) and the metric
// arithmetic it runs in: float32 for both float types (a float16 value
// converts to float32 exactly), exact int32 with renormalisation for int8.
template <int DT>
struct Ty;
template <>
struct Ty<0> {
  static constexpr bool kInt = false;
  using T = float;
  using In = float;
  __device__ static float neg_unreachable() { return -__builtin_inff(); }
  __device__ static int bits(float x) { return __builtin_bit_cast(int, x); }
  __device__ static float from(int x) { return __builtin_bit_cast(float, x); }
};
template <>
struct Ty<1> {
  static constexpr bool kInt = true;
  using T = int;
  using In = int8_t;
  __device__ static int neg_unreachable() { return -(1 << 29); }
  __device__ static int bits(int x) { return x; }
  __device__ static int from(int x) { return x; }
};
template <>
struct Ty<2> : Ty<0> {
  using In = _Float16;
};

// Fetch the metrics of the even and odd previous states for lane bit Q.
template <int Q, int DT>
__device__ __forceinline__ void pair_fetch(typename Ty<DT>::T x, int addr_e, int addr_o,
                                           typename Ty<DT>::T& e, typename Ty<DT>::T& o) {
  const int xi = Ty<DT>::bits(x);
  int ei, oi;
  if constexpr (Q == 0) {
    ei = __builtin_amdgcn_mov_dpp(xi, 0xA0, 0xF, 0xF, true);  // quad_perm [0,0,2,2]
    oi = __builtin_amdgcn_mov_dpp(xi, 0xF5, 0xF, 0xF, true);  // quad_perm [1,1,3,3]
  } else if constexpr (Q == 1) {
    ei = __builtin_amdgcn_mov_dpp(xi, 0x44, 0xF, 0xF, true);  // quad_perm [0,1,0,1]
    oi = __builtin_amdgcn_mov_dpp(xi, 0xEE, 0xF, 0xF, true);  // quad_perm [2,3,2,3]
  } else if constexpr (Q <= 4) {
    // ds_swizzle bit-mask mode within 32 lanes: lane' = (lane & and) | or
    ei = __builtin_amdgcn_ds_swizzle(xi, 0x1F & ~(1 << Q));
    oi = __builtin_amdgcn_ds_swizzle(xi, 0x1F | ((1 << Q) << 5));
  } else {
    ei = __builtin_amdgcn_ds_bpermute(addr_e, xi);
    oi = __builtin_amdgcn_ds_bpermute(addr_o, xi);
  }
  e = Ty<DT>::from(ei);
  o = Ty<DT>::from(oi);
}

// Fetch the metric of the partner lane (lane XOR 2^Q).  XOR 1, 2 and 8 are
// single DPP patterns (fused by the compiler into the consuming subtract).
template <int Q, int DT>
__device__ __forceinline__ typename Ty<DT>::T partner_fetch(typename Ty<DT>::T x, int addr_p) {
  const int xi = Ty<DT>::bits(x);
  int pi;
  if constexpr (Q == 0) {
    pi = __builtin_amdgcn_mov_dpp(xi, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
  } else if constexpr (Q == 1) {
    pi = __builtin_amdgcn_mov_dpp(xi, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
  } else if constexpr (Q == 3) {
    pi = __builtin_amdgcn_mov_dpp(xi, 0x128, 0xF, 0xF, true);  // row_ror:8
  } else if constexpr (Q == 2 || Q == 4) {
    pi = __builtin_amdgcn_ds_swizzle(xi, 0x1F | ((1 << Q) << 10));  // xor mode
  } else {
    pi = __builtin_amdgcn_ds_bpermute(addr_p, xi);
  }
  return Ty<DT>::from(pi);
}

template <int KM1, int DT, int NP, int MODE>
struct Frame {
  using T = typename Ty<DT>::T;
  T pm;
  uint32_t acc;
  int pat_off[KM1];  // LDS word offset of this lane's pattern, per phase
  int addr_e, addr_o, addr_p;
  uint64_t bmask[KM1];  // lanes whose bit q is set, per phase q
};

// Mode 2 picks, per lane bit, the cheapest exchange that stays in the VALU:
//   bits 0, 1  both previous-state metrics by DPP quad permutations (fixed roles)
//   bit 2      partner (lane ^ 4) = quad reverse of the row half-mirror (two DPPs)
//   bit 3      partner (lane ^ 8) = DPP row rotate by 8
//   bits 4, 5  v_permlane16_swap / v_permlane32_swap of the metric and a copy:
//              one register receives the even rows (halves), the other the odd
template <int Q>
struct Mode2 {
  static constexpr bool fixed_roles = (Q == 0 || Q == 1 || Q == 4 || Q == 5);
};

template <int Q, int DT>
__device__ __forceinline__ void pair_fetch_valu(typename Ty<DT>::T x, typename Ty<DT>::T& e,
                                                typename Ty<DT>::T& o) {
  const int xi = Ty<DT>::bits(x);
  int ei, oi;
  if constexpr (Q == 0) {
    ei = __builtin_amdgcn_mov_dpp(xi, 0xA0, 0xF, 0xF, true);
    oi = __builtin_amdgcn_mov_dpp(xi, 0xF5, 0xF, 0xF, true);
  } else if constexpr (Q == 1) {
    ei = __builtin_amdgcn_mov_dpp(xi, 0x44, 0xF, 0xF, true);
    oi = __builtin_amdgcn_mov_dpp(xi, 0xEE, 0xF, 0xF, true);
  } else if constexpr (Q == 4) {
    auto r = __builtin_amdgcn_permlane16_swap(xi, xi, false, false);
    ei = r[0];
    oi = r[1];
  } else {
    auto r = __builtin_amdgcn_permlane32_swap(xi, xi, false, false);
    ei = r[0];
    oi = r[1];
  }
  e = Ty<DT>::from(ei);
  o = Ty<DT>::from(oi);
}

template <int Q, int DT>
__device__ __forceinline__ typename Ty<DT>::T partner_fetch_valu(typename Ty<DT>::T x) {
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

template <typename T>
__device__ __forceinline__ T tmax(T a, T b) {
  return a > b ? a : b;
}

// One stage at phase Q, own/partner form.  The lane keeps its own previous
// state's metric and fetches its partner's.  With m0 the Eq. (BM) value of
// the even previous state on input 0, the candidate through the lane's own
// previous state is own + m0 and through the partner's is partner - m0, in
// every lane (the corollary flips the sign once for the odd state and once
// for input 1).  The new metric is the larger one; the decision "the odd
// previous state won" is partner > own where the lane's bit Q is 0 (partner
// odd) and own > partner where it is 1 (own odd), strict either way, so a tie
// keeps the even state.
template <int KM1, int DT, int NP, int MODE, int Q>
__device__ __forceinline__ void stage_op(Frame<KM1, DT, NP, MODE>& F, typename Ty<DT>::T m0) {
  using T = typename Ty<DT>::T;
  const T cp = partner_fetch<Q, DT>(F.pm, F.addr_p) - m0;
  const T co = F.pm + m0;
  F.pm = tmax(co, cp);
  const uint64_t g1 = __builtin_amdgcn_ballot_w64(cp > co);
  const uint64_t g2 = __builtin_amdgcn_ballot_w64(co > cp);
  const uint64_t d = (g1 & ~F.bmask[Q]) | (g2 & F.bmask[Q]);
  F.acc = push_decision(F.acc, d);
}

// One stage at phase Q: add, compare, select, record.
template <int KM1, int DT, int NP, int MODE, int Q>
__device__ __forceinline__ void stage(Frame<KM1, DT, NP, MODE>& F, typename Ty<DT>::T bm) {
  using T = typename Ty<DT>::T;
  T e, o;
  pair_fetch<Q, DT>(F.pm, F.addr_e, F.addr_o, e, o);
  const T ce = e + bm;  // even previous state, Eq. (PM) candidate
  const T co = o - bm;  // odd previous state: opposite branch metric
  const bool d = co > ce;
  F.pm = d ? co : ce;
  F.acc = push_decision(F.acc, __builtin_amdgcn_ballot_w64(d));
}

// Mode 2 stage: fixed roles (both metrics fetched) or own/partner.
template <int KM1, int DT, int NP, int MODE, int Q>
__device__ __forceinline__ void stage_m2(Frame<KM1, DT, NP, MODE>& F, typename Ty<DT>::T bm) {
  using T = typename Ty<DT>::T;
  if constexpr (Mode2<Q>::fixed_roles) {
    T e, o;
    pair_fetch_valu<Q, DT>(F.pm, e, o);
    const T ce = e + bm;
    const T co = o - bm;
    const bool d = co > ce;
    F.pm = d ? co : ce;
    F.acc = push_decision(F.acc, __builtin_amdgcn_ballot_w64(d));
  } else {
    const T cp = partner_fetch_valu<Q, DT>(F.pm) - bm;
    const T co = F.pm + bm;
    F.pm = tmax(co, cp);
    const uint64_t g1 = __builtin_amdgcn_ballot_w64(cp > co);
    const uint64_t g2 = __builtin_amdgcn_ballot_w64(co > cp);
    const uint64_t d = (g1 & ~F.bmask[Q]) | (g2 & F.bmask[Q]);
    F.acc = push_decision(F.acc, d);
  }
}

template <int KM1, int DT, int NP, int MODE, int Q>
__device__ __forceinline__ void stage_any(Frame<KM1, DT, NP, MODE>& F, typename Ty<DT>::T bm) {
  if constexpr (MODE == 2)
    stage_m2<KM1, DT, NP, MODE, Q>(F, bm);
  else if constexpr (MODE == 1)
    stage_op<KM1, DT, NP, MODE, Q>(F, bm);
  else
    stage<KM1, DT, NP, MODE, Q>(F, bm);
}

template <int KM1, int DT, int NP, int MODE, int P0, int K0>
__device__ __forceinline__ void stages_full(Frame<KM1, DT, NP, MODE>& F,
                                            const typename Ty<DT>::T* bmv) {
  if constexpr (K0 < 32) {
    stage_any<KM1, DT, NP, MODE, (P0 + K0) % KM1>(F, bmv[K0]);
    stages_full<KM1, DT, NP, MODE, P0, K0 + 1>(F, bmv);
  }
}

// A stage whose phase is only known at run time (the last, partial block).
template <int KM1, int DT, int NP, int MODE, int Q>
__device__ __forceinline__ void stage_dyn(Frame<KM1, DT, NP, MODE>& F, const typename Ty<DT>::T* bmrow,
                                          int q) {
  if constexpr (Q < KM1) {
    if (q == Q) {
      stage_any<KM1, DT, NP, MODE, Q>(F, bmrow[F.pat_off[Q]]);
    } else {
      stage_dyn<KM1, DT, NP, MODE, Q + 1>(F, bmrow, q);
    }
  }
}

template <int KM1, int DT, int NP, int MODE, int P0>
__device__ __forceinline__ void block(Frame<KM1, DT, NP, MODE>& F, const typename Ty<DT>::T* bmt,
                                      int n) {
  using T = typename Ty<DT>::T;
  if (n == 32) {
    // this lane's branch metric of every stage of the block, read up front
    T bmv[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) bmv[k] = bmt[k * NP + F.pat_off[(P0 + k) % KM1]];
    stages_full<KM1, DT, NP, MODE, P0, 0>(F, bmv);
  } else {
#pragma unroll 1
    for (int k = 0; k < n; ++k) stage_dyn<KM1, DT, NP, MODE, 0>(F, bmt + k * NP, (P0 + k) % KM1);
  }
}

// Order LDS traffic between the lanes of one wavefront.  LDS instructions of
// a wavefront execute in order, so a compiler-level fence at wavefront scope
// is enough; unlike a workgroup barrier it does not wait for the outstanding
// global loads that prefetch the next block.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Soft values of the stages a lane tabulates in one block: stages
// sl + k*2^(K-1) for k < max(1, 32/2^(K-1)).
template <int KM1, int DT, int BETA>
struct LlrRegs {
  static constexpr int NS = 1 << KM1;
  static constexpr int NSTG = NS >= 32 ? 1 : 32 / NS;
  typename Ty<DT>::T v[NSTG][BETA];
  __device__ __forceinline__ void load(const typename Ty<DT>::In* llr, int tb, int S, int sl,
                                       bool valid) {
#pragma unroll
    for (int k = 0; k < NSTG; ++k) {
      const int t = tb + sl + k * NS;
      const bool ok = valid && sl + k * NS < 32 && t < S;
#pragma unroll
      for (int b = 0; b < BETA; ++b)
        v[k][b] = ok ? (typename Ty<DT>::T)llr[(int64_t)t * BETA + b] : (typename Ty<DT>::T)0;
    }
  }
};

// State shared by the blocks of one wavefront.
template <int KM1, int DT, int BETA, int MODE>
struct BlockCtx {
  Frame<KM1, DT, (1 << BETA), MODE>* F;
  typename Ty<DT>::T* bmt;
  const typename Ty<DT>::In* llr;
  uint32_t* sv;
  int64_t* offset;
  int* blk;
  int S, sl, lane;
  bool valid;
  LlrRegs<KM1, DT, BETA> lr;  // soft values of the current block, loaded a block ahead
};

// One block of up to 32 stages starting at tb, phase (32*BI) mod (K-1).
template <int KM1, int DT, int BETA, int MODE, int BI>
__device__ __forceinline__ void one_block(BlockCtx<KM1, DT, BETA, MODE>& bc, int tb) {
  using T = typename Ty<DT>::T;
  constexpr int NS = 1 << KM1, NP = 1 << BETA;
  constexpr int NSTG = LlrRegs<KM1, DT, BETA>::NSTG;
  const int n = min(32, bc.S - tb);
  // branch-metric table of this block: Eq. (BM) for every output pattern
#pragma unroll
  for (int k = 0; k < NSTG; ++k) {
    const int tt = bc.sl + k * NS;
    if (tt < 32) {
#pragma unroll
      for (int p = 0; p < NP / 2; ++p) {
        T v = (T)0;
#pragma unroll
        for (int b = 0; b < BETA; ++b) v += ((p >> b) & 1) ? -bc.lr.v[k][b] : bc.lr.v[k][b];
        bc.bmt[tt * NP + p] = v;
        bc.bmt[tt * NP + (NP - 1 - p)] = -v;
      }
    }
  }
  // the next block's soft values are read while this block runs
  bc.lr.load(bc.llr, tb + 32, bc.S, bc.sl, bc.valid);
  if constexpr (Ty<DT>::kInt) {
    if (tb > 0) {
      // renormalise by the metric of state 0 (always in the frame's lane 0)
      const T ref = __builtin_amdgcn_ds_bpermute((bc.lane & ~(NS - 1)) << 2, bc.F->pm);
      bc.F->pm -= ref;
      *bc.offset += ref;
    }
  }
  wave_sync();
  block<KM1, DT, NP, MODE, (32 * BI) % KM1>(*bc.F, bc.bmt, n);
  if (bc.valid) bc.sv[(int64_t)(*bc.blk) * NS + bc.sl] = bc.F->acc << (32 - n);
  bc.F->acc = 0;
  ++*bc.blk;
  wave_sync();
}

template <int KM1, int DT, int BETA, int MODE, int BI, int NB>
__device__ __forceinline__ void super_block(BlockCtx<KM1, DT, BETA, MODE>& bc, int t0) {
  if constexpr (BI < NB) {
    const int tb = t0 + 32 * BI;
    if (tb < bc.S) {
      one_block<KM1, DT, BETA, MODE, BI>(bc, tb);
      super_block<KM1, DT, BETA, MODE, BI + 1, NB>(bc, t0);
    }
  }
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

}  // namespace rot

// Wavefronts per workgroup: four, one per SIMD, so that every SIMD of a CU
// receives the same number of frames (the wavefronts share nothing).
constexpr int kRotWaves = 4;

// The frames of wave-table entry 'wave', on one wavefront.
template <int KM1, int DT, int BETA, int MODE>
__device__ __forceinline__ void fwd_rot_wave(const DevCode* __restrict__ codes,
                                             const Item* __restrict__ items,
                                             const int2* __restrict__ waves, int wave,
                                             const void* __restrict__ llr_v,
                                             uint64_t* __restrict__ surv, void* metric,
                                             int32_t* end_out, int32_t* item_end,
                                             typename rot::Ty<DT>::T (*bmt)[32 << BETA],
                                             typename rot::Ty<DT>::T* xpm, int lane) {
  using namespace rot;
  using T = typename Ty<DT>::T;
  using In = typename Ty<DT>::In;
  constexpr int NS = 1 << KM1;
  constexpr int NP = 1 << BETA;
  constexpr int SUPER = 32 * KM1 / gcd_c(32, KM1);  // lcm(32, K-1)
  const int fr = lane / NS, sl = lane % NS;
  // this wave's frames: waves[w] = (first item, count), all of equal length
  const int2 wv = waves[wave];
  const bool valid = fr < wv.y;
  const Item it = items[wv.x + (valid ? fr : 0)];
  const DevCode c = codes[it.code];
  const int S = __builtin_amdgcn_readfirstlane(it.n_stages);  // equal within the wave
  const In* llr = (const In*)llr_v + it.llr_off;
  uint32_t* sv = (uint32_t*)(surv + it.surv_off);

  Frame<KM1, DT, NP, MODE> F;
#pragma unroll
  for (int q = 0; q < KM1; ++q) {
    const int j = rotr(sl, (q + 1) % KM1, KM1);  // state held after a phase-q stage
    const int ie = (j << 1) & (NS - 1);
    const int u = j >> (KM1 - 1);
    // fixed roles: the even previous state's branch into j; own/partner
    // stages: its branch on input 0
    const bool fixed = MODE == 0 || (MODE == 2 && (q == 0 || q == 1 || q == 4 || q == 5));
    F.pat_off[q] = branch_out(c, ie, fixed ? u : 0);
    uint64_t bm = 0;
    for (int l = 0; l < 64; ++l)
      if ((l >> q) & 1) bm |= 1ull << l;
    F.bmask[q] = bm;
  }
  F.addr_e = (lane & ~32) << 2;
  F.addr_o = (lane | 32) << 2;
  F.addr_p = (lane ^ 32) << 2;
  F.pm = (it.start_known && sl != 0) ? Ty<DT>::neg_unreachable() : (T)0;
  F.acc = 0;
  int64_t offset = 0;
  T* my_bmt = &bmt[fr][0];

  int blk = 0;
  BlockCtx<KM1, DT, BETA, MODE> bc{&F, my_bmt, llr, sv, &offset, &blk, S, sl, lane, valid, {}};
  bc.lr.load(llr, 0, S, sl, valid);
  for (int t0 = 0; t0 < S; t0 += SUPER) super_block<KM1, DT, BETA, MODE, 0, SUPER / 32>(bc, t0);
  // final metrics: lane sl holds state rotr(sl, S mod (K-1))
  const int st = rotr(sl, S % KM1, KM1);
  xpm[fr * NS + st] = F.pm;
  wave_sync();
  if (sl == 0 && valid) {
    int js = it.end_state;
    if (js < 0) {
      js = 0;
      for (int j = 1; j < NS; ++j)
        if (xpm[fr * NS + j] > xpm[fr * NS + js]) js = j;
    }
    item_end[it.slot] = js;
    if (it.frame >= 0) {
      if (end_out) end_out[it.frame] = js;
      if (metric) {
        if constexpr (Ty<DT>::kInt)
          ((int64_t*)metric)[it.frame] = (int64_t)xpm[fr * NS + js] + offset;
        else
          ((float*)metric)[it.frame] = xpm[fr * NS + js];
      }
    }
  }
}

// One wavefront per wave-table entry, or (counter != nullptr) a persistent
// grid whose wavefronts take entries in table order (longest frames first)
// from a device counter that starts at zero, until the table is exhausted.
template <int KM1, int DT, int BETA, int MODE>
__global__ __launch_bounds__(64 * kRotWaves) void k_fwd_rot(const DevCode* __restrict__ codes,
                                                const Item* __restrict__ items,
                                                const int2* __restrict__ waves, int n_waves,
                                                const void* __restrict__ llr_v,
                                                uint64_t* __restrict__ surv, void* metric,
                                                int32_t* end_out, int32_t* item_end,
                                                int32_t* counter) {
  using T = typename rot::Ty<DT>::T;
  constexpr int FPW = 64 >> KM1;
  __shared__ T bmt_all[kRotWaves][FPW][32 << BETA];
  __shared__ T xpm_all[kRotWaves][64];
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (counter == nullptr) {
    const int wave = blockIdx.x * kRotWaves + wid;
    if (wave >= n_waves) return;  // no workgroup barriers: safe to leave
    fwd_rot_wave<KM1, DT, BETA, MODE>(codes, items, waves, wave, llr_v, surv, metric, end_out,
                                       item_end, bmt_all[wid], xpm_all[wid], lane);
    return;
  }
  for (;;) {
    int w = 0;
    if (lane == 0) w = atomicAdd(counter, 1);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= n_waves) break;
    fwd_rot_wave<KM1, DT, BETA, MODE>(codes, items, waves, w, llr_v, surv, metric, end_out,
                                       item_end, bmt_all[wid], xpm_all[wid], lane);
  }
}

hipError_t launch_fwd_rot(int K, int beta, int dt, int mode, const DevCode* codes,
                          const Item* items, const int2* waves, int n_waves, const void* llr,
                          uint64_t* surv, void* metric, int32_t* end_out, int32_t* item_end,
                          int32_t* counter, int grid_limit, hipStream_t st) {
  if (n_waves <= 0) return hipSuccess;
  const int threads = 64 * kRotWaves;
  auto go = [&](auto kernel) -> hipError_t {
    int nb = (n_waves + kRotWaves - 1) / kRotWaves;
    if (counter) {
      const int lim = grid_limit > 0 ? grid_limit : resident_workgroups(kernel, threads);
      if (lim > 0 && nb > lim) nb = lim;
    }
    hipLaunchKernelGGL(kernel, dim3(nb), dim3(threads), 0, st, codes, items, waves, n_waves, llr,
                       surv, metric, end_out, item_end, counter);
    return hipGetLastError();
  };
  // float16 soft values: the all-VALU exchange scheme (MODE 2) only
  if (dt == 2 && mode != 2) return hipErrorInvalidValue;
#define MV_ROT(KM1, I, B)                                                   \
  if constexpr (I == 2) return go(k_fwd_rot<KM1, I, B, 2>);                \
  else return mode == 2 ? go(k_fwd_rot<KM1, I, B, 2>)                      \
              : mode == 1 ? go(k_fwd_rot<KM1, I, B, 1>)                    \
                          : go(k_fwd_rot<KM1, I, B, 0>)
#define MV_ROT_B(KM1, I)              \
  switch (beta) {                     \
    case 2: MV_ROT(KM1, I, 2);        \
    case 3: MV_ROT(KM1, I, 3);        \
    case 4: MV_ROT(KM1, I, 4);        \
    default: return hipErrorInvalidValue; \
  }
#define MV_ROT_K(I)                   \
  switch (K) {                        \
    case 3: MV_ROT_B(2, I);           \
    case 4: MV_ROT_B(3, I);           \
    case 5: MV_ROT_B(4, I);           \
    case 6: MV_ROT_B(5, I);           \
    case 7: MV_ROT_B(6, I);           \
    default: return hipErrorInvalidValue; \
  }
  switch (dt) {
    case 0: MV_ROT_K(0);
    case 1: MV_ROT_K(1);
    case 2: MV_ROT_K(2);
    default: return hipErrorInvalidValue;
  }
#undef MV_ROT_K
#undef MV_ROT_B
#undef MV_ROT
}

}  // namespace mivit
