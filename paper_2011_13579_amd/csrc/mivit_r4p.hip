// Radix-4 forward procedure and traceback for int8 soft values, rate 1/2,
// K = 5 or 7, with two frames packed in the 16-bit halves of every register.
//
// Trellis (§VIII-A, Eq. (radix4:S)).  Write a state of n = K-1 bits as n/2
// base-4 digits.  One radix-4 iteration (two stages) maps the left state
// i = 4f + y to the right state j = f + 2^(n-2) u, u = 2 u2 + u1 the two new
// input bits: the lowest digit y of i is consumed, the others move down one
// place and u enters on top.  A dragonfly group is the four left states that
// differ in y and the four right states that differ in u.
//
// Rotating digit map.  At iteration it (phase ph = it mod n/2) the left state
// i lives in lane rotl_n(i, 2 ph): its lowest digit sits in lane-digit slot
// ph.  The right state j then lives in lane rotl_n(j, 2 (ph + 1)), which puts
// its new top digit u in slot ph as well and leaves every other digit where
// it was.  A dragonfly group is therefore the four lanes that differ only in
// slot ph, and the right states stay in place: slot 0 (lane bits 0-1) is a
// DPP quad broadcast, slot 1 (bits 2-3) a DPP row rotation by 4, 8, 12 (the
// adds take these as DPP operands), and slot 2 (bits 4-5, the rows of 16
// lanes) a 4 x 4 transpose of candidates that every lane forms for its four
// successors: two v_permlane32_swap and two v_permlane16_swap.
//
// Packed metrics.  Path metrics are unsigned 16-bit numbers, frame A in the
// low and frame B in the high half of a VGPR.  A metric is stored as
// 4 * (PM + offset) with offsets chosen so that every value stays in
// [0, 65535]; adding two such words with one 32-bit add then never carries
// between the halves, and v_pk_max_u16 compares both frames at once.  The
// two low bits carry the tie tag 3 - y of the left state a candidate came
// from: among equal metrics the larger tag, i.e. the smaller y, wins, which
// is the lowest-index previous state of the paper's strict comparison, and
// the winner's tag is the 2-bit decision.
//
// Branch metrics (Eq. (radix4:BM)).  For each iteration the 16 super-branch
// metrics of a frame are the dot products of its four int8 soft values with
// the +-1 sign rows of the 16 output patterns (v_dot4_i32_i8, signs scaled by
// 4, bias 2048 so entries are >= 0); both frames share one LDS word per
// pattern.  Every lane reads the four entries its candidates need.
//
// Range control.  Every 8 iterations the metric of state 0 (always lane 0 of
// its lane group) is brought back to 16384 by a subtraction common to all
// states of the frame; the subtracted amounts are accumulated exactly in
// 64 bits and added back to the final metric.  With |l| <= 128 the spread of
// reachable metrics is at most 2 (K-1) 2 128 (any state reaches any other in
// K-1 stages), so values stay within [4093, 61443].
//
// Odd stage counts: stage 0 is a radix-2 stage evaluated in closed form
// (the start metrics are either all zero or zero at state 0 only).  Its
// decisions are never needed: the traceback emits stage 0's bit from the
// state at time 1.
//
// Survivor layout of a frame pair (lane group of NS lanes): for each group
// of 8 iterations, NS words; word G*NS + R holds the tags the state in lane R
// won in iterations 8G..8G+7: iteration 8G+k, frame h (0 = A, 1 = B) in bits
// 16 (k & 1) + 8 h + 2 (k >> 1) and the bit above.  Two consecutive
// iterations are gathered by one byte permutation of their max results.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mivit_device.h"

namespace mivit {

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st);

namespace r4p {

constexpr uint32_t kBase = 16384;
constexpr uint32_t kBase2 = kBase | (kBase << 16);
constexpr uint32_t kStrip = 0xFFFCFFFCu;
constexpr uint32_t kTagBytes = 0x03030303u;
constexpr int kBias = 2048;   // 4 * max |super-branch metric| for |l| <= 128
constexpr int kLeadOff = 256;  // max |branch metric| of one stage

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(us2, a),
                                                                __builtin_bit_cast(us2, b)));
}

__device__ __forceinline__ int parity(uint32_t x) { return __popc(x) & 1; }

// beta = 2 output bits of the branch leaving state i on input u (§II-A).
__device__ __forceinline__ int branch_out2(const DevCode& c, int i, int u) {
  const uint32_t reg = ((uint32_t)u << (c.K - 1)) | (uint32_t)i;
  return parity(c.gen[0] & reg) | (parity(c.gen[1] & reg) << 1);
}

__device__ __forceinline__ int rotl_n(int x, int r, int n) {
  return r == 0 ? x : (((x << r) | (x >> (n - r))) & ((1 << n) - 1));
}
__device__ __forceinline__ int rotr_n(int x, int r, int n) { return rotl_n(x, (n - r) % n, n); }

// The four metrics a lane combines at phase PH, from the lanes that differ
// from it in lane-digit slot PH.  Applied to lane ids it names those lanes.
template <int PH>
__device__ __forceinline__ void fetch4(uint32_t x, uint32_t (&o)[4]) {
  if constexpr (PH == 0) {
    o[0] = __builtin_amdgcn_mov_dpp((int)x, 0x00, 0xF, 0xF, true);  // quad_perm [0,0,0,0]
    o[1] = __builtin_amdgcn_mov_dpp((int)x, 0x55, 0xF, 0xF, true);  // quad_perm [1,1,1,1]
    o[2] = __builtin_amdgcn_mov_dpp((int)x, 0xAA, 0xF, 0xF, true);  // quad_perm [2,2,2,2]
    o[3] = __builtin_amdgcn_mov_dpp((int)x, 0xFF, 0xF, 0xF, true);  // quad_perm [3,3,3,3]
  } else if constexpr (PH == 1) {
    o[0] = x;
    o[1] = __builtin_amdgcn_mov_dpp((int)x, 0x124, 0xF, 0xF, true);  // row_ror:4
    o[2] = __builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);  // row_ror:8
    o[3] = __builtin_amdgcn_mov_dpp((int)x, 0x12C, 0xF, 0xF, true);  // row_ror:12
  } else {
    // rows (r0 r1 r2 r3) -> (r0 r1 r0 r1), (r2 r3 r2 r3) -> each row everywhere
    const auto h = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    const auto a = __builtin_amdgcn_permlane16_swap(h[0], h[0], false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(h[1], h[1], false, false);
    o[0] = a[0];
    o[1] = a[1];
    o[2] = b[0];
    o[3] = b[1];
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Four int8 soft values of one iteration; any alignment.
__device__ __forceinline__ uint32_t load_llr4(const int8_t* p) {
  uint32_t w;
  __builtin_memcpy(&w, p, 4);
  return w;
}

template <int ND>
struct Fwd {
  static constexpr int KM1 = 2 * ND;
  static constexpr int NS = 1 << KM1;
  static constexpr int PPL = 256 / NS;  // table entries a lane fills per block

  const uint32_t* tp[ND][4];  // LDS table entry of candidate k at phase ph (block row 0)
  uint32_t tag[ND];           // tie tag of the state a lane holds entering phase ph
  int32_t sgn[PPL];           // sign rows (+-4 per soft value) of this lane's patterns
  uint32_t* tbl;              // this lane group's table: 16 rows x 16 patterns
  int ib;                     // table row this lane fills
  const int8_t* l0;           // soft values of iteration 0, frame A / B
  const int8_t* l1;
  uint32_t w0, w1;            // soft values of this lane's row, current block
  uint32_t V;                 // packed metrics, tagged for the next iteration
  uint32_t acc;               // decisions of the current group of 8 iterations
  uint32_t vs;                // max result of the last even iteration (its tags)
  uint32_t* sv;               // survivor words of the lane group
  int r, n_it;                // n_it: one past the last iteration this unit runs
  int it_store;               // first iteration whose decisions are stored
  bool store;
  uint64_t off0, off1;        // accumulated renormalisation amounts
};

// One iteration; returns the max result, whose low two bits per half are
// the winners' tags (the decisions).
template <int ND, int PH>
__device__ __forceinline__ uint32_t iterate(Fwd<ND>& F, int row) {
  uint32_t v;
  if constexpr (PH == 2) {
    // slot 2 is the row of 16 lanes: each lane adds the branch metrics of
    // its four successors (in the same lane of rows 0..3) to its own metric,
    // and a 4 x 4 transpose across the rows (two 32-lane and two 16-lane
    // swaps, no copies) hands every lane its four candidates
    const uint32_t c0 = F.V + F.tp[2][0][row * 16];
    const uint32_t c1 = F.V + F.tp[2][1][row * 16];
    const uint32_t c2 = F.V + F.tp[2][2][row * 16];
    const uint32_t c3 = F.V + F.tp[2][3][row * 16];
    const auto s02 = __builtin_amdgcn_permlane32_swap(c0, c2, false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(c1, c3, false, false);
    const auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
    const auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
    v = pk_max(pk_max(s01[0], s01[1]), pk_max(s23[0], s23[1]));
  } else {
    uint32_t o[4];
    fetch4<PH>(F.V, o);
    const uint32_t c0 = o[0] + F.tp[PH][0][row * 16];
    const uint32_t c1 = o[1] + F.tp[PH][1][row * 16];
    const uint32_t c2 = o[2] + F.tp[PH][2][row * 16];
    const uint32_t c3 = o[3] + F.tp[PH][3][row * 16];
    v = pk_max(pk_max(c0, c1), pk_max(c2, c3));
  }
  F.V = (v & kStrip) | F.tag[(PH + 1) % ND];
  return v;
}

// Decisions of iteration K8 (static) of a group: bytes 0 and 2 of the even
// and the odd iteration's max results in one permutation, then one mask.
template <int ND, int K8>
__device__ __forceinline__ void collect(Fwd<ND>& F, uint32_t v) {
  if constexpr ((K8 & 1) == 0) {
    F.vs = v;
  } else {
    const uint32_t t = __builtin_amdgcn_perm(v, F.vs, 0x06040200u) & kTagBytes;
    F.acc = K8 == 1 ? t : (F.acc | (t << (K8 - 1)));
  }
}

// The same for a runtime iteration index k (the last, partial block).
template <int ND>
__device__ __forceinline__ void iterate_dyn(Fwd<ND>& F, int row, int ph, int k) {
  uint32_t v;
  if (ph == 0) {
    v = iterate<ND, 0>(F, row);
  } else if (ph == 1) {
    v = iterate<ND, 1 % ND>(F, row);
  } else {
    v = iterate<ND, 2 % ND>(F, row);
  }
  const uint32_t sel = (k & 1) ? 0x02000C0Cu : 0x0C0C0200u;  // 0x0C: a zero byte
  F.acc |= (__builtin_amdgcn_perm(v, v, sel) & kTagBytes) << (2 * ((k & 7) >> 1));
}

// End of a group of iterations ending at iteration `last`.
template <int ND>
__device__ __forceinline__ void group_end(Fwd<ND>& F, int last) {
  constexpr int NS = Fwd<ND>::NS;
  const int n = (last & 7) + 1;
  if (F.store && last >= F.it_store) F.sv[(last >> 3) * NS + F.r] = F.acc;
  F.acc = 0;
  if (n == 8) {
    // bring state 0 (lane 0 of the group) back to kBase in both halves
    if constexpr (NS == 64) {
      const uint32_t ref = __builtin_amdgcn_readfirstlane(F.V);  // lane 0
      const uint32_t d = (ref & kStrip) - kBase2;
      F.V -= d;
      F.off0 += d & 0xFFFFu;
      F.off1 += d >> 16;
    } else {
      const int src = (int)((threadIdx.x & 63) & ~(NS - 1)) << 2;
      const uint32_t ref = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)F.V);
      const uint32_t d = (ref & kStrip) - kBase2;
      F.V -= d;
      F.off0 += d & 0xFFFFu;
      F.off1 += d >> 16;
    }
  }
}

// Iterations Q..15 of a full block (straight-line code, static phases).
template <int ND, int P0, int Q>
__device__ __forceinline__ void iterate_full(Fwd<ND>& F, int it0) {
  if constexpr (Q < 16) {
    collect<ND, Q & 7>(F, iterate<ND, (P0 + Q) % ND>(F, Q));
    if constexpr ((Q & 7) == 7) group_end<ND>(F, it0 + Q);
    iterate_full<ND, P0, Q + 1>(F, it0);
  }
}

// One block of up to 16 iterations from it0; P0 = phase of it0.
template <int ND, int P0>
__device__ __forceinline__ void block(Fwd<ND>& F, int it0) {
  constexpr int PPL = Fwd<ND>::PPL;
  // super-branch metric table of the block
  {
    uint32_t t[PPL];
#pragma unroll
    for (int e = 0; e < PPL; ++e) {
      const uint32_t a = (uint32_t)__builtin_amdgcn_sdot4((int)F.w0, F.sgn[e], kBias, false);
      const uint32_t b = (uint32_t)__builtin_amdgcn_sdot4((int)F.w1, F.sgn[e], kBias, false);
      t[e] = a | (b << 16);
    }
    uint4* dst = (uint4*)(F.tbl + F.ib * 16 + (F.r % (16 / PPL)) * PPL);
#pragma unroll
    for (int e = 0; e < PPL / 4; ++e) dst[e] = make_uint4(t[4 * e], t[4 * e + 1], t[4 * e + 2], t[4 * e + 3]);
  }
  // soft values of the next block
  {
    const int itn = it0 + 16 + F.ib;
    const bool ok = itn < F.n_it;
    F.w0 = ok ? load_llr4(F.l0 + 4 * (int64_t)itn) : 0u;
    F.w1 = ok ? load_llr4(F.l1 + 4 * (int64_t)itn) : 0u;
  }
  wave_sync();
  const int n = min(16, F.n_it - it0);
  if (n == 16) {
    iterate_full<ND, P0, 0>(F, it0);
  } else {
#pragma unroll 1
    for (int q = 0; q < n; ++q) {
      iterate_dyn<ND>(F, q, (P0 + q) % ND, q);
      if ((q & 7) == 7 || q == n - 1) group_end<ND>(F, it0 + q);
    }
  }
  wave_sync();
}

template <int ND, int B, int NB>
__device__ __forceinline__ void super_block(Fwd<ND>& F, int it0) {
  if constexpr (B < NB) {
    const int itb = it0 + 16 * B;
    if (itb < F.n_it) {
      block<ND, (16 * B) % ND>(F, itb);
      super_block<ND, B + 1, NB>(F, it0);
    }
  }
}

template <int ND, int PH>
__device__ __forceinline__ void lane_consts(Fwd<ND>& F, const DevCode& c, int lane, int r) {
  constexpr int KM1 = Fwd<ND>::KM1, NS = Fwd<ND>::NS;
  if constexpr (PH == 2 && ND == 3) {
    // source side: the branch from this lane's left state to the right
    // state held by the same lane of row u after the iteration
    const int i = rotr_n(r, (2 * PH) % KM1, KM1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = rotr_n((r & 15) | (u << 4), (2 * (PH + 1)) % KM1, KM1);
      const int un = j >> (KM1 - 2);  // = u: slot 2 holds the new digit
      const int mid = ((un & 1) << (KM1 - 1)) | (i >> 1);
      const int p = branch_out2(c, i, un & 1) | (branch_out2(c, mid, un >> 1) << 2);
      F.tp[PH][u] = F.tbl + p;
    }
  } else if constexpr (PH < ND) {
    uint32_t src[4];
    fetch4<PH>((uint32_t)lane, src);
    const int j = rotr_n(r, (2 * (PH + 1)) % KM1, KM1);  // right state held after the iteration
    const int u = j >> (KM1 - 2);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = rotr_n((int)src[k] & (NS - 1), (2 * PH) % KM1, KM1);  // left state in that lane
      const int mid = ((u & 1) << (KM1 - 1)) | (i >> 1);
      const int p = branch_out2(c, i, u & 1) | (branch_out2(c, mid, u >> 1) << 2);
      F.tp[PH][k] = F.tbl + p;
    }
  }
  if constexpr (PH < ND) {
    const int s = rotr_n(r, (2 * PH) % KM1, KM1);  // left state held entering the iteration
    F.tag[PH] = (uint32_t)(3 - (s & 3)) * 0x10001u;
    lane_consts<ND, PH + 1>(F, c, lane, r);
  }
}

constexpr int kR4Waves = 4;

}  // namespace r4p

// One wavefront decodes up to 2 * 64 / 2^(K-1) frames of equal length:
// lane group m (2^(K-1) lanes) holds frames 2m (low halves) and 2m+1 (high).
// It runs the iterations of one unit (whole frames, one part of frames split
// in time, or a repair, kind 1).  Split units that are not last leave their
// end metrics in a boundary record; the last part reports the end state and
// its own metric, which the check completes.
template <int ND>
__device__ __forceinline__ void fwd_r4p_wave(const DevCode* __restrict__ codes,
                                             const Item* __restrict__ items, const SplitUnit U,
                                             int kind, R4Bound* bounds, int64_t* last_m,
                                             const int64_t* rep_m0,
                                             const int8_t* __restrict__ llr,
                                             uint64_t* __restrict__ surv, int64_t* metric,
                                             int32_t* end_out, int32_t* item_end,
                                             uint32_t (*tbl_w)[16 * 16], int lane) {
  using namespace r4p;
  constexpr int KM1 = 2 * ND, NS = 1 << KM1, PPL = 256 / NS;
  const int m = lane / NS, r = lane % NS;
  const bool va = 2 * m < U.count, vb = 2 * m + 1 < U.count;
  const int ia = U.first + (va ? 2 * m : 0);
  const int ib_ = vb ? ia + 1 : ia;  // a missing frame B repeats frame A
  const Item ita = items[ia], itb = items[ib_];
  const DevCode c = codes[ita.code];
  const int S = __builtin_amdgcn_readfirstlane(ita.n_stages);  // equal within the wave
  const int lead = S & 1;
  // iterations: warm-up from s0, decisions kept from it_b, last one it_e - 1
  const int it_b = U.it_begin, it_e = U.it_end, s0 = U.it_begin - U.warm;
  const bool first_part = kind == 0 && U.part == 0;
  const bool split = U.n_parts > 1;

  Fwd<ND> F;
  F.tbl = &tbl_w[m][0];
  F.r = r;
  F.n_it = it_e;
  F.it_store = it_b;
  // lanes 4k .. 4k+3 (K = 7) fill row k, so one 16-byte store per lane
  // covers the table contiguously (no LDS bank conflicts)
  F.ib = r / (16 / PPL);
  F.store = va;
  F.sv = (uint32_t*)(surv + ita.surv_off);
  F.l0 = llr + ita.llr_off + 2 * lead;
  F.l1 = llr + itb.llr_off + 2 * lead;
  F.off0 = F.off1 = 0;
  F.acc = 0;
#pragma unroll
  for (int e = 0; e < PPL; ++e) {
    const int p = (r % (16 / PPL)) * PPL + e;
    uint32_t s = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) s |= (((p >> b) & 1) ? 0xFCu : 0x04u) << (8 * b);
    F.sgn[e] = (int32_t)s;
  }
  lane_consts<ND, 0>(F, c, lane, r);

  // metrics entering iteration s0 (lane r holds state r: s0 is a multiple of
  // the digit count, so the map is the identity there)
  if (first_part) {
    const int j = r;
    uint32_t v[2];
    const Item* its[2] = {&ita, &itb};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool known = its[h]->start_known != 0;
      if (lead) {
        const int8_t* p = llr + its[h]->llr_off;
        const int i0 = (j << 1) & (NS - 1);
        const int w = branch_out2(c, i0, j >> (KM1 - 1));
        const int bm = ((w & 1) ? -(int)p[0] : (int)p[0]) + ((w & 2) ? -(int)p[1] : (int)p[1]);
        int pm;
        bool reach = true;
        if (known) {
          reach = i0 == 0;
          pm = bm;
        } else {
          pm = bm < 0 ? -bm : bm;  // max(bm, -bm): the two branches into j
        }
        v[h] = reach ? kBase + 4u * (uint32_t)(pm + kLeadOff) : 0u;
      } else {
        v[h] = (!known || j == 0) ? kBase : 0u;
      }
    }
    F.V = v[0] | (v[1] << 16) | F.tag[0];
  } else if (kind == 0) {
    F.V = kBase2 | F.tag[0];  // a later part: all-zero metrics (unknown start)
  } else {
    F.V = (bounds[U.bnd + U.part - 1].v_end[lane] & kStrip) | F.tag[0];  // repair
  }
  {
    const int itn = s0 + F.ib;
    const bool ok = itn < it_e;
    F.w0 = ok ? load_llr4(F.l0 + 4 * (int64_t)itn) : 0u;
    F.w1 = ok ? load_llr4(F.l1 + 4 * (int64_t)itn) : 0u;
  }
  // metric of state 0 from this unit's origin, per half, at iteration x
  // (range control has just brought state 0 back to kBase there)
  auto m0_at = [&](int x, int h) -> int64_t {
    const int64_t o = (int64_t)(h ? F.off1 : F.off0);
    return o / 4 - (int64_t)(kBias / 4) * (x - s0) - (first_part ? (int64_t)kLeadOff * lead : 0);
  };
  constexpr int SUPER = (ND == 3) ? 3 : 1;  // blocks per period of the phase pattern
  for (int it0 = s0; it0 < it_e; it0 += 16 * SUPER) {
    if (kind == 0 && U.part > 0 && it0 == it_b) {
      R4Bound& B = bounds[U.bnd + U.part - 1];
      B.v_start[lane] = F.V & kStrip;
      if (r == 0) {
        B.m_start[2 * m] = m0_at(it_b, 0);
        B.m_start[2 * m + 1] = m0_at(it_b, 1);
      }
    }
    super_block<ND, 0, SUPER>(F, it0);
  }
  if (kind == 0 && split && U.part < U.n_parts - 1) {
    R4Bound& B = bounds[U.bnd + U.part];
    B.v_end[lane] = F.V & kStrip;
    if (r == 0) {
      B.m_end[2 * m] = m0_at(it_e, 0);
      B.m_end[2 * m + 1] = m0_at(it_e, 1);
    }
    return;
  }

  // final metrics: lane r holds state rotr(r, 2 (it_e mod ND))
  const int js_lane = rotr_n(r, (2 * (it_e % ND)) % KM1, KM1);
  const uint32_t vs = F.V & kStrip;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const Item& it = h ? itb : ita;
    const bool valid = h ? vb : va;
    const uint32_t val = (vs >> (16 * h)) & 0xFFFFu;
    uint32_t key = (val << 8) | (uint32_t)(255 - js_lane);
#pragma unroll
    for (int o = 1; o < NS; o <<= 1) {
      const uint32_t other = (uint32_t)__shfl_xor((int)key, o);
      key = other > key ? other : key;
    }
    const bool fixed = it.end_state >= 0;
    const int js = fixed ? it.end_state : 255 - (int)(key & 255);
    const int src = m * NS + rotl_n(js & (NS - 1), (2 * (it_e % ND)) % KM1, KM1);
    const uint32_t vfix = (uint32_t)__shfl((int)val, src);
    const uint32_t vbest = fixed ? vfix : key >> 8;
    if (r == 0 && valid) {
      item_end[it.slot] = js;
      const int64_t o = (int64_t)(h ? F.off1 : F.off0);
      const int64_t local = ((int64_t)vbest - (int64_t)kBase + o) / 4 -
                            (int64_t)(kBias / 4) * (it_e - s0) -
                            (first_part ? (int64_t)kLeadOff * lead : 0);
      if (kind == 0 && split) {
        last_m[it.slot] = local;  // completed by the check
      } else if (it.frame >= 0) {
        if (end_out) end_out[it.frame] = js;
        if (metric) metric[it.frame] = local + (kind == 1 ? rep_m0[it.slot] : 0);
      }
      if (kind == 0 && split && it.frame >= 0 && end_out) end_out[it.frame] = js;
    }
  }
}

// ---------------------------------------------------------------------------
// Traceback of a frame pair (Algorithm 2), 32 segments per frame.
//
// Lanes g and g+32 trace segment g of frames A and B; both frames of a pair
// share their survivor words, so the two lanes share each staged block of 64
// words: lane g streams its 16-byte chunks 0, 2, .., 14 and lane g+32 chunks
// 1, 3, .., 15 into LDS (global_load_lds).  Word w of the block then sits at
// byte ((w & 3) << 2) | ((w & ~3) << 7) + 16 g of the buffer.  The chase
// keeps its state as that byte offset (for the word of its lane in the
// current group), so taking a step only replaces one 2-bit field: the digit
// slot the iteration consumed.  Segment boundaries, speculation and repair as
// in the radix-2 traceback: lane g starts `warm` stages above its segment
// from state 0, and a lane whose state at its upper boundary disagrees with
// the (exact) lane above traces again from that lane's state.
// ---------------------------------------------------------------------------
namespace r4p {

typedef __attribute__((address_space(3))) void* lds_ptr_t;

template <int ND>
struct Tb {
  static constexpr int KM1 = 2 * ND, NS = 1 << KM1;
  static constexpr int IPB = 512 / NS;  // iterations per staged block
};

__device__ __forceinline__ uint32_t addr_of(int R) {
  return (uint32_t)(((R & 3) << 2) | ((R & ~3) << 7));
}
__device__ __forceinline__ int lane_of(uint32_t A) {
  return (int)(((A >> 2) & 3) | ((A >> 7) & ~3));
}
// byte position of lane-digit slot s in the offset form
__device__ __forceinline__ int slot_pos(int s) { return s == 0 ? 2 : (s == 1 ? 9 : 11); }

struct Chase {
  int hi, lo;       // iterations hi-1 down to lo are traced (lo >= 0)
  int a, b;         // stages [a, b) are emitted
  int PX, PY;       // iteration tops (time lead + 2P) where X and Y are taken
  uint32_t A;       // current state (offset form) at time lead + 2*(current top)
  uint32_t X, Y;
  bool emit;
};

template <int ND>
__device__ __forceinline__ void fetch_half(const uint32_t* blk, uint32_t* buf, int hb) {
#pragma unroll
  for (int c = 0; c < 8; ++c)
    __builtin_amdgcn_global_load_lds((const void*)(blk + 4 * (2 * c + hb)), (lds_ptr_t)(buf + c * 256),
                                     16, 0, 0);
}

// All lanes whose pair has work chase their range in lockstep rounds; lanes
// with go set update c and emit.  The stage-0 bit of an odd stage count is
// the top bit of the state at time 1, where the chase of iteration 0 ends.
template <int ND>
__device__ __forceinline__ void chase_all(Chase& c, bool go, bool pair_go, const uint32_t* sv,
                                          uint32_t* lds, int lead, int h, int g, int ob,
                                          uint32_t* bits, int64_t bit_off) {
  constexpr int KM1 = Tb<ND>::KM1, NS = Tb<ND>::NS, IPB = Tb<ND>::IPB;
  const int lane = threadIdx.x & 63;
  GroupEmitter em;
  const bool any = pair_go && c.hi > c.lo;
  const int B0 = any ? (c.hi - 1) / IPB : 0;
  const int nb = any ? B0 - c.lo / IPB + 1 : 0;
  int P = c.hi;
  uint32_t A = go ? c.A : 0u;
  if (go && P == c.PY) c.Y = A;
  if (go && P == c.PX) c.X = A;
  const int hb = lane >> 5;
  if (nb > 0) fetch_half<ND>(sv + (int64_t)B0 * 64, lds, hb);
  for (int rd = 0;; ++rd) {
    if (__ballot(rd < nb) == 0) break;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    wave_sync();
    const uint32_t base = (uint32_t)((rd & 1) * 8192 + g * 16);
    uint32_t* nxt = lds + ((rd + 1) & 1) * 2048;
    if (rd + 1 < nb) fetch_half<ND>(sv + (int64_t)(B0 - rd - 1) * 64, nxt, hb);
    if (rd < nb) {
      const int B = B0 - rd;
      const int lo = max(c.lo, B * IPB);
      for (; P > lo; --P) {
        const int it = P - 1;
        const int pos = slot_pos(it % ND);
        const uint32_t goff = (uint32_t)(((it >> 3) & (64 / NS - 1)) << 11);
        const uint32_t word = *(const uint32_t*)((const char*)lds + base + goff + A);
        const uint32_t tag = (word >> (16 * (it & 1) + 8 * h + 2 * ((it & 7) >> 1))) & 3u;
        const uint32_t u = (A >> pos) & 3u;
        A = (A | (3u << pos)) - (tag << pos);
        if (go && c.emit) {
          const int s1 = lead + 2 * it + 1, s0 = s1 - 1;
          if (s1 >= c.a && s1 < c.b) em.put(s1 - ob, u >> 1, bits, bit_off);
          if (s0 >= c.a && s0 < c.b) em.put(s0 - ob, u & 1u, bits, bit_off);
        }
        if (go && it == c.PY) c.Y = A;
        if (go && it == c.PX) c.X = A;
      }
    }
    wave_sync();
  }
  if (go) {
    c.A = A;
    // time 1 holds state lane_of(A) (the phase-0 map is the identity)
    if (c.emit && lead && c.lo == 0 && c.a <= 0 && c.b > 0)
      em.put(-ob, (uint32_t)(lane_of(A) >> (KM1 - 1)), bits, bit_off);
  }
  em.flush(bits);
}

}  // namespace r4p

template <int ND>
__global__ __launch_bounds__(64) void k_tb_r4p(const Item* __restrict__ items,
                                               const int2* __restrict__ pairs,
                                               const uint64_t* __restrict__ surv,
                                               const int32_t* __restrict__ item_end,
                                               uint32_t* __restrict__ bits, int warm) {
  using namespace r4p;
  constexpr int KM1 = 2 * ND;
  __shared__ uint32_t lds[2 * 2048];
  const int lane = threadIdx.x;
  const int h = lane >> 5, g = lane & 31;
  const int2 pr = pairs[blockIdx.x];
  const bool have = h < pr.y;
  const Item it = items[pr.x + (have ? h : 0)];
  const int S = it.n_stages, ob = it.out_begin, n = it.n_out;
  if (n <= 0) return;  // equal within the pair: the whole wavefront leaves
  const int lead = S & 1, n_it = S >> 1;
  const uint32_t* sv = (const uint32_t*)(surv + it.surv_off);
  // segments of L stages (L a multiple of 32), at most 32 per frame
  int G = min(32, (n + 31) / 32);
  const int L = (((n + G - 1) / G) + 31) & ~31;
  G = (n + L - 1) / L;
  const bool active = g < G;
  const int a = ob + g * L;
  const int b = min(ob + (g + 1) * L, ob + n);
  // pair-aligned times at or above a time t: lead + 2P
  auto top_of = [&](int t) { return (t - lead + 1) >> 1; };  // smallest P with lead + 2P >= t
  // lanes whose warm-up reaches the frame end start from the known end state
  const int P_top = (g == G - 1) ? n_it : min(n_it, top_of(b + warm));
  const bool exact = active && P_top == n_it;
  Chase c;
  c.hi = active ? P_top : 0;
  c.lo = max(0, (a - lead) >> 1);  // the iteration holding stage a (0: stage 0 of odd S)
  c.a = a;
  c.b = b;
  c.PX = top_of(a);
  c.PY = top_of(b);
  c.emit = have;
  c.X = c.Y = 0xFFFFFFFFu;
  if (exact) {
    const int js = item_end[it.slot];
    c.A = addr_of(rotl_n(js, (2 * (n_it % ND)) % KM1, KM1));
  } else {
    c.A = 0;
  }
  // a frame of one stage has no iteration: only stage 0's bit is emitted
  const bool go = active && (c.hi > c.lo || (lead && c.lo == 0 && a <= 0));
  // the shuffle runs on every lane: inside a short-circuit it would run only
  // where the left side is false and read nothing from the other lanes
  const int go_partner = __shfl_xor((int)go, 32);
  const bool pair_go = go | (go_partner != 0);
  chase_all<ND>(c, go, pair_go, sv, lds, lead, h, g, ob, bits, it.bit_off);
  // repair: lane g is right when its state at its upper boundary equals the
  // state lane g+1 reached at its lower boundary (the same time)
  bool checked = exact;
  constexpr uint32_t kStateBits = (uint32_t)((3 << 2) | (((1 << (2 * ND)) - 4) << 7));
  for (int round = 0; round <= G; ++round) {
    const uint32_t x_up = (uint32_t)__shfl_down((int)c.X, 1) & kStateBits;
    const bool bad = active && !checked && g < G - 1 && c.Y != x_up;
    if (__ballot(bad) == 0) break;
    const int bad_partner = __shfl_xor((int)bad, 32);
    const bool pbad = bad | (bad_partner != 0);
    Chase rc = c;
    rc.hi = c.PY;
    rc.A = x_up;
    rc.Y = c.Y;
    chase_all<ND>(rc, bad, pbad, sv, lds, lead, h, g, ob, bits, it.bit_off);
    if (bad) {
      c.A = rc.A;
      c.X = rc.X;
      c.Y = x_up;
    }
  }
}

// One wavefront per unit, or (counter != nullptr) a persistent grid whose
// wavefronts take units in table order from a device counter that starts at
// zero, until the table is exhausted.  Repair launches (kind 1) read their
// unit count from the device (dev_count).
template <int ND>
__global__ __launch_bounds__(64 * r4p::kR4Waves) void k_fwd_r4p(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ units, int n_units, const int32_t* dev_count, int kind,
    R4Bound* bounds, int64_t* last_m, const int64_t* rep_m0, const int8_t* __restrict__ llr,
    uint64_t* __restrict__ surv, int64_t* metric, int32_t* end_out, int32_t* item_end,
    int32_t* counter) {
  constexpr int FPG = 64 >> (2 * ND);
  __shared__ uint32_t tbl_all[r4p::kR4Waves][FPG][16 * 16];
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (dev_count) n_units = min(n_units, __builtin_amdgcn_readfirstlane(*dev_count));
  if (counter == nullptr) {
    const int u = blockIdx.x * r4p::kR4Waves + wid;
    if (u >= n_units) return;  // no workgroup barriers: safe to leave
    fwd_r4p_wave<ND>(codes, items, units[u], kind, bounds, last_m, rep_m0, llr, surv, metric,
                     end_out, item_end, tbl_all[wid], lane);
    return;
  }
  for (;;) {
    int w = 0;
    if (lane == 0) w = atomicAdd(counter, 1);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= n_units) break;
    fwd_r4p_wave<ND>(codes, items, units[w], kind, bounds, last_m, rep_m0, llr, surv, metric,
                     end_out, item_end, tbl_all[wid], lane);
  }
}

// The check after a split forward pass, one wavefront per split entry (its
// part-0 unit): boundary k is exact when part k's metrics at its end equal
// part k+1's after its warm-up at every position (both are range-controlled
// to state 0 there, so equal words mean metric vectors that differ by a
// constant).  Every boundary of the entry is loaded at once.  Lane k
// follows frame k of the entry: T = the true metric of state 0 at the first
// inexact boundary, D = the constant the last part's metrics lack when all
// are exact.
struct EntryCheck {
  int fail;  // first inexact boundary, or -1
  int64_t T, D;
};

template <int NV>
__device__ __forceinline__ EntryCheck check_entry(const SplitUnit& U,
                                                  const R4Bound* __restrict__ bounds, int lane) {
  const int n_b = U.n_parts - 1;
  const int k = lane < U.count ? lane : 0;
  uint32_t bad = 0;
#pragma unroll
  for (int b = 0; b < kMaxSplitParts - 1; ++b) {
    if (b < n_b) {
      const R4Bound& B = bounds[U.bnd + b];
      bool diff = false;
#pragma unroll
      for (int x = 0; x < NV / 64; ++x) diff = diff || B.v_end[64 * x + lane] != B.v_start[64 * x + lane];
      if (__ballot(diff) != 0) bad |= 1u << b;
    }
  }
  EntryCheck r;
  r.fail = bad ? (int)__builtin_ctz(bad) : -1;
  const int last = r.fail < 0 ? n_b : r.fail;
  int64_t T = bounds[U.bnd].m_end[k], D = 0;  // part 0 is exact
  for (int b = 0; b < last; ++b) {
    D = T - bounds[U.bnd + b].m_start[k];
    if (b + 1 < n_b) T = bounds[U.bnd + b + 1].m_end[k] + D;
  }
  r.T = T;
  r.D = D;
  return r;
}

// The repair unit of an entry whose boundary `fail` is inexact: the frames
// from that boundary to their end, from the metrics part `fail` left there.
__device__ __forceinline__ SplitUnit repair_unit(const SplitUnit& U, const R4Bound* bounds,
                                                 int fail, int n_stages) {
  SplitUnit R = U;
  R.it_begin = bounds[U.bnd + fail].it_at;
  R.it_end = n_stages >> 1;
  R.warm = 0;
  R.part = fail + 1;
  return R;
}

// Check of the one-state kernel's split entries; an entry with an inexact
// boundary is repaired by the same wavefront, right here.
template <int ND>
__global__ __launch_bounds__(64 * r4p::kR4Waves) void k_r4p_check(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ split, int n_split, R4Bound* bounds,
    const int64_t* __restrict__ last_m, int64_t* rep_m0, const int8_t* __restrict__ llr,
    uint64_t* __restrict__ surv, int64_t* metric, int32_t* end_out, int32_t* item_end) {
  constexpr int FPG = 64 >> (2 * ND);
  __shared__ uint32_t tbl_all[r4p::kR4Waves][FPG][16 * 16];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = blockIdx.x * r4p::kR4Waves + wid;
  if (e >= n_split) return;  // no workgroup barriers: safe to leave
  const SplitUnit U = split[e];
  const EntryCheck c = check_entry<64>(U, bounds, lane);
  const bool mine = lane < U.count;
  const Item it = items[U.first + (mine ? lane : 0)];
  if (c.fail < 0) {
    if (mine && metric && it.frame >= 0) metric[it.frame] = last_m[it.slot] + c.D;
    return;
  }
  if (mine) rep_m0[it.slot] = c.T;
  __threadfence();
  fwd_r4p_wave<ND>(codes, items, repair_unit(U, bounds, c.fail, items[U.first].n_stages), 1,
                   bounds, const_cast<int64_t*>(last_m), rep_m0, llr, surv, metric, end_out,
                   item_end, tbl_all[wid], lane);
}

// ---------------------------------------------------------------------------
// Packed radix 4 with four states per lane (K = 7).
//
// The same trellis, digit map, packed tagged metrics, tables and survivor
// words as above, laid out differently: a frame pair occupies one row of 16
// lanes (up to four pairs, eight frames, per wavefront) and lane-digit slot
// 2 becomes the register index, so position p = l + 16 q holds, in register
// q of lane l of the pair's row, what lane p holds in the one-state kernel.
// Phases 0 and 1 are the DPP exchanges above applied to each register; the
// dragonfly groups of phase 2 differ only in the register index, so that
// phase is evaluated inside every lane with no exchange (the 4 x 4 transpose
// of the one-state kernel, four permlane swaps, disappears), and the four
// registers are independent dependency chains.
//
// Scheduling.  Every lane fills one table row of its pair per 16-iteration
// block; three blocks of tables rotate in LDS, so a block's table is written
// one block before it is read, and rows are padded (20 words) and pairs
// offset (16 banks) so neither the 16-byte table stores nor the lookups
// conflict on LDS banks.  Each iteration loads the table entries of the next
// one (the last iteration of a block those of the next block's first), and
// a block is branch-free: pairs beyond the entry's frame count repeat pair 0
// exactly (they store the same words to the same places), and the warm-up
// iterations of a split unit, whose decisions are not kept, run a copy of
// the loop without stores.
//
// Table addresses.  The output pattern of a two-stage branch is linear over
// GF(2) in the left state and the two inputs (the code is a convolution), so
// a lane's 48 candidate patterns are the XOR of a part that depends on its
// lane, one that depends on the register only and one of the inputs.
//
// The survivor word of position p is word G*64 + p as above, so the same
// traceback reads it.
// ---------------------------------------------------------------------------
namespace r4q {

using namespace r4p;

constexpr int kRow = 20;                   // words per table row (16 used)
constexpr int kPairTbl = 16 * kRow + 16;   // words per pair table: pairs 16 banks apart
constexpr int kBufWords = 4 * kPairTbl;    // one block's tables of a wavefront
constexpr int kWaves = 2;                  // wavefronts per workgroup

// +-4 sign row of output pattern p (bit b set: soft value b enters negated)
__host__ __device__ constexpr int32_t sign_row(int p) {
  return (int32_t)(((p & 1) ? 0xFCu : 0x04u) | (((p & 2) ? 0xFCu : 0x04u) << 8) |
                   (((p & 4) ? 0xFCu : 0x04u) << 16) | (((p & 8) ? 0xFCu : 0x04u) << 24));
}

// Output pattern (4 bits: stage 2t's two output bits, then stage 2t+1's) of
// the two-stage branch from left state i on inputs u (u & 1 first), K = 7.
__device__ __forceinline__ int pattern(const DevCode& c, int i, int u) {
  const int mid = ((u & 1) << 5) | (i >> 1);
  return branch_out2(c, i, u & 1) | (branch_out2(c, mid, u >> 1) << 2);
}

struct Fq {
  const uint32_t* tp[3][4][4];  // table entry (buffer 0, row 0) of candidate k of register q at phase ph
  uint32_t tag0, tag1;          // tie tags entering phases 0 and 1
  uint32_t tag2[4];             // entering phase 2: 3 - q (held in registers, so the
                                // retag is one v_and_or with the strip mask)
  int32_t sg[8];                // sign rows of patterns 0..7 (scalar registers)
  uint32_t bias;                // 2048 in both halves
  uint32_t* trow;               // this lane's row in its pair table (buffer 0)
  const int8_t* l0;             // soft values of iteration 0, frames A / B of the pair
  const int8_t* l1;
  uint32_t w0, w1;              // soft values of this lane's row, block after the current one
  uint32_t V[4];                // packed metrics of positions l + 16 q, tagged
  uint32_t cur[16];             // table entries of the next iteration
  uint32_t acc[4], vs[4];       // decisions of the current group; last even iteration's max
  uint32_t hi[4];               // decisions of iterations 4..5 of the group
  uint32_t* sv;                 // survivor words of the pair, plus the lane's position l
  int n_it;
  uint64_t off0, off1;          // accumulated renormalisation amounts of the pair
};

// Orders this wavefront's table stores before its later table loads (and
// its earlier loads before the stores), without waiting for either.
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Table of one block (buffer nb) from this lane's soft values: its row.
// Pattern p ^ 15 negates every soft value of pattern p, so its entry is
// 2 * 2048 - (entry of p) in each half.
__device__ __forceinline__ void q_table(Fq& F, int nb) {
  uint4* dst = (uint4*)(F.trow + nb * kBufWords);
  uint32_t t[16];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    // frame A's entry + 2048 in the low half, frame B's + 2048 in the high
    // (the second product accumulates into the shifted first, in place)
    const uint32_t b = (uint32_t)__builtin_amdgcn_sdot4((int)F.w1, F.sg[p], 0, false);
    t[p] = (uint32_t)__builtin_amdgcn_sdot4((int)F.w0, F.sg[p], (int)((b << 16) + F.bias), false);
    t[p ^ 15] = (uint32_t)(2 * kBias) * 0x10001u - t[p];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) dst[e] = make_uint4(t[4 * e], t[4 * e + 1], t[4 * e + 2], t[4 * e + 3]);
}

// Soft values of iteration itn (0 past the unit's last iteration); n_it >= 1.
__device__ __forceinline__ void q_load(Fq& F, int itn) {
  const int64_t x = 4 * (int64_t)min(itn, F.n_it - 1);
  const uint32_t a = load_llr4(F.l0 + x), b = load_llr4(F.l1 + x);
  const bool ok = itn < F.n_it;
  F.w0 = ok ? a : 0u;
  F.w1 = ok ? b : 0u;
}

// Table entries of an iteration at phase PH, word offset o (buffer, row).
template <int PH>
__device__ __forceinline__ void q_fetch(const Fq& F, int o, uint32_t (&t)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int k = 0; k < 4; ++k) t[4 * q + k] = F.tp[PH][q][k][o];
}

// One iteration at phase PH with table entries t; v receives the max
// results (tags = decisions) of the four registers.
template <int PH>
__device__ __forceinline__ void q_step(Fq& F, const uint32_t (&t)[16], uint32_t (&v)[4]) {
  if constexpr (PH == 2) {
    // the right state of register u takes the best of the left states in
    // registers y = 0..3 of the same lane (entry 4u + y)
    uint32_t c[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int y = 0; y < 4; ++y) c[u][y] = F.V[y] + t[4 * u + y];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = pk_max(pk_max(c[u][0], c[u][1]), pk_max(c[u][2], c[u][3]));
#pragma unroll
    for (int q = 0; q < 4; ++q) F.V[q] = (v[q] & kStrip) | F.tag0;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t x[4];
      fetch4<PH>(F.V[q], x);
      const uint32_t c0 = x[0] + t[4 * q];
      const uint32_t c1 = x[1] + t[4 * q + 1];
      const uint32_t c2 = x[2] + t[4 * q + 2];
      const uint32_t c3 = x[3] + t[4 * q + 3];
      v[q] = pk_max(pk_max(c0, c1), pk_max(c2, c3));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) F.V[q] = (v[q] & kStrip) | (PH == 0 ? F.tag1 : F.tag2[q]);
  }
}

// Decisions of iteration K8 (static) of a group, per register.
template <int K8>
__device__ __forceinline__ void q_collect(Fq& F, const uint32_t (&v)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr ((K8 & 1) == 0) {
      F.vs[q] = v[q];
    } else {
      // pairs of iterations combined as a tree: one shift-or each
      const uint32_t t = __builtin_amdgcn_perm(v[q], F.vs[q], 0x06040200u) & kTagBytes;
      if constexpr (K8 == 1) F.acc[q] = t;
      if constexpr (K8 == 3) F.acc[q] |= t << 2;
      if constexpr (K8 == 5) F.hi[q] = t;
      if constexpr (K8 == 7) F.acc[q] |= (F.hi[q] | (t << 2)) << 4;
    }
  }
}

__device__ __forceinline__ void q_renorm(Fq& F) {
  // bring state 0 (register 0 of the row's lane 0) back to kBase
  const uint32_t ref = (uint32_t)__builtin_amdgcn_mov_dpp((int)F.V[0], 0x150, 0xF, 0xF, false);
  const uint32_t d = (ref & kStrip) - kBase2;
#pragma unroll
  for (int q = 0; q < 4; ++q) F.V[q] -= d;
  F.off0 += d & 0xFFFFu;
  F.off1 += d >> 16;
}

// End of a whole group of 8 iterations ending at iteration `last`.
template <bool STORE>
__device__ __forceinline__ void q_group_end(Fq& F, int last) {
  if constexpr (STORE) {
#pragma unroll
    for (int q = 0; q < 4; ++q) F.sv[(last >> 3) * 64 + 16 * q] = F.acc[q];
  }
  q_renorm(F);
}

template <int P0, int Q, bool STORE>
__device__ __forceinline__ void q_iterate_full(Fq& F, int it0, int ob, int ob_next) {
  if constexpr (Q < 16) {
    uint32_t t[16], v[4];
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = F.cur[e];
    if constexpr (Q < 15)
      q_fetch<(P0 + Q + 1) % 3>(F, ob + (Q + 1) * kRow, F.cur);
    else
      q_fetch<(P0 + 1) % 3>(F, ob_next, F.cur);  // the next block's first row
    q_step<(P0 + Q) % 3>(F, t, v);
    q_collect<Q & 7>(F, v);
    if constexpr ((Q & 7) == 7) q_group_end<STORE>(F, it0 + Q);
    // keep each iteration's loads one iteration ahead of their use
    __builtin_amdgcn_sched_barrier(0);
    q_iterate_full<P0, Q + 1, STORE>(F, it0, ob, ob_next);
  }
}

// Block B (0, 1, 2) of a 48-iteration period from it0: its table is buffer
// B (and its first row's entries are in F.cur); it writes buffer B+1 for the
// next block and loads the soft values of the block after that.
template <int B, bool STORE>
__device__ __forceinline__ void q_block(Fq& F, int it0) {
  constexpr int P0 = (16 * B) % 3;
  q_table(F, (B + 1) % 3);
  q_load(F, it0 + 32 + (int)(threadIdx.x & 15));
  wave_fence();
  const int n = min(16, F.n_it - it0);
  if (n == 16) {
    q_iterate_full<P0, 0, STORE>(F, it0, B * kBufWords, ((B + 1) % 3) * kBufWords);
  } else {
    // the unit's last, partial block (stores: the warm-up is whole periods);
    // the static groups leave their decisions in acc
#pragma unroll
    for (int r = 0; r < 4; ++r) F.acc[r] = 0;
#pragma unroll 1
    for (int q = 0; q < n; ++q) {
      uint32_t t[16], v[4];
      const int o = B * kBufWords + q * kRow;
      const int ph = (P0 + q) % 3;
      if (ph == 0) {
        q_fetch<0>(F, o, t);
        q_step<0>(F, t, v);
      } else if (ph == 1) {
        q_fetch<1>(F, o, t);
        q_step<1>(F, t, v);
      } else {
        q_fetch<2>(F, o, t);
        q_step<2>(F, t, v);
      }
      const uint32_t sel = (q & 1) ? 0x02000C0Cu : 0x0C0C0200u;  // 0x0C: a zero byte
#pragma unroll
      for (int r = 0; r < 4; ++r)
        F.acc[r] |= (__builtin_amdgcn_perm(v[r], v[r], sel) & kTagBytes) << (2 * ((q & 7) >> 1));
      if ((q & 7) == 7 || q == n - 1) {
        const int last = it0 + q;
#pragma unroll
        for (int r = 0; r < 4; ++r) F.sv[(last >> 3) * 64 + 16 * r] = F.acc[r];
#pragma unroll
        for (int r = 0; r < 4; ++r) F.acc[r] = 0;
        if ((q & 7) == 7) q_renorm(F);
      }
    }
  }
}

template <int B, bool STORE>
__device__ __forceinline__ void q_period(Fq& F, int it0) {
  if constexpr (B < 3) {
    const int itb = it0 + 16 * B;
    if (itb < F.n_it) {
      q_block<B, STORE>(F, itb);
      q_period<B + 1, STORE>(F, it0);
    }
  }
}

}  // namespace r4q

// One wavefront decodes up to 8 frames of equal length: the row of lanes
// 16m .. 16m+15 holds frames 2m (low halves) and 2m+1 (high).  Units, split
// boundaries and repairs as in fwd_r4p_wave; boundary records hold position
// p = l + 16 q of pair m at index 64 q + 16 m + l.
__device__ __forceinline__ void fwd_r4q_wave(const DevCode* __restrict__ codes,
                                             const Item* __restrict__ items, const SplitUnit U,
                                             int kind, R4Bound* bounds, int64_t* last_m,
                                             const int64_t* rep_m0,
                                             const int8_t* __restrict__ llr,
                                             uint64_t* __restrict__ surv, int64_t* metric,
                                             int32_t* end_out, int32_t* item_end,
                                             uint32_t* tbl, int lane) {
  using namespace r4q;
  constexpr int KM1 = 6;
  const int m = lane >> 4, l = lane & 15;
  const bool va = 2 * m < U.count, vb = 2 * m + 1 < U.count;
  // a pair beyond the frame count repeats pair 0 (same inputs, same stores)
  const int ia = U.first + (va ? 2 * m : 0);
  const int ib_ = va ? (vb ? ia + 1 : ia) : U.first + (U.count > 1 ? 1 : 0);
  const Item ita = items[ia], itb = items[ib_];
  const DevCode c = codes[__builtin_amdgcn_readfirstlane(ita.code)];  // one code per part
  const int S = __builtin_amdgcn_readfirstlane(ita.n_stages);  // equal within the wave
  const int lead = S & 1;
  const int it_b = U.it_begin, it_e = U.it_end, s0 = U.it_begin - U.warm;
  const bool first_part = kind == 0 && U.part == 0;
  const bool split = U.n_parts > 1;

  Fq F;
  F.trow = tbl + m * kPairTbl + l * kRow;
  F.n_it = it_e;
  F.sv = (uint32_t*)(surv + ita.surv_off) + l;
  F.l0 = llr + ita.llr_off + 2 * lead;
  F.l1 = llr + itb.llr_off + 2 * lead;
  F.off0 = F.off1 = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) F.acc[q] = F.vs[q] = 0;
  // table entries of every candidate (the digit map of lane_consts):
  // pattern(i, u) = pattern(i_lane, 0) ^ pattern(i_reg, 0) ^ pattern(0, u)
  {
    const uint32_t* pt = tbl + m * kPairTbl;
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      uint32_t src[4];
      if (ph == 0)
        fetch4<0>((uint32_t)lane, src);
      else
        fetch4<1>((uint32_t)lane, src);
      // the right state's new digit u sits in slot ph of the lane: l's digit ph
      const int zu = pattern(c, 0, (l >> (2 * ph)) & 3);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int xk = pattern(c, rotr_n((int)(src[k] & 15), 2 * ph, KM1), 0) ^ zu;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          F.tp[ph][q][k] = pt + (xk ^ pattern(c, rotr_n(16 * q, 2 * ph, KM1), 0));
      }
    }
    // phase 2: right state l + 16 u from the left states of registers y
    const int d = pattern(c, rotr_n(l, 4, KM1), 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int y = 0; y < 4; ++y)
        F.tp[2][u][y] = pt + (d ^ pattern(c, rotr_n(16 * y, 4, KM1), u));
  }
  F.tag0 = (uint32_t)(3 - (l & 3)) * 0x10001u;
  F.tag1 = (uint32_t)(3 - ((l >> 2) & 3)) * 0x10001u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // a register copy the compiler does not fold back into two literals
    asm volatile("v_mov_b32 %0, %1" : "=v"(F.tag2[q]) : "n"((3 - q) * 0x10001));
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    // in scalar registers (not literals), so the products can read them directly
    asm volatile("s_mov_b32 %0, %1" : "=s"(F.sg[p]) : "n"(sign_row(p)));
  }
  F.bias = (uint32_t)((kBias << 16) | kBias);

  // metrics entering iteration s0 (a multiple of 3: position p holds state p)
  if (first_part) {
    const Item* its[2] = {&ita, &itb};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = l + 16 * q;
      uint32_t v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool known = its[h]->start_known != 0;
        if (lead) {
          const int8_t* p = llr + its[h]->llr_off;
          const int i0 = (j << 1) & 63;
          const int w = branch_out2(c, i0, j >> (KM1 - 1));
          const int bm = ((w & 1) ? -(int)p[0] : (int)p[0]) + ((w & 2) ? -(int)p[1] : (int)p[1]);
          int pm;
          bool reach = true;
          if (known) {
            reach = i0 == 0;
            pm = bm;
          } else {
            pm = bm < 0 ? -bm : bm;
          }
          v[h] = reach ? kBase + 4u * (uint32_t)(pm + kLeadOff) : 0u;
        } else {
          v[h] = (!known || j == 0) ? kBase : 0u;
        }
      }
      F.V[q] = v[0] | (v[1] << 16) | F.tag0;
    }
  } else if (kind == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) F.V[q] = kBase2 | F.tag0;  // later part: unknown start
  } else {
    const R4Bound& B = bounds[U.bnd + U.part - 1];
#pragma unroll
    for (int q = 0; q < 4; ++q) F.V[q] = (B.v_end[64 * q + lane] & kStrip) | F.tag0;  // repair
  }
  auto m0_at = [&](int x, int h) -> int64_t {
    const int64_t o = (int64_t)(h ? F.off1 : F.off0);
    return o / 4 - (int64_t)(kBias / 4) * (x - s0) - (first_part ? (int64_t)kLeadOff * lead : 0);
  };
  if (it_e > s0) {
    // tables of the first block, its first row, soft values of the second
    q_load(F, s0 + l);
    q_table(F, 0);
    q_load(F, s0 + 16 + l);
    wave_fence();
    q_fetch<0>(F, 0, F.cur);
    int it0 = s0;
    for (; it0 < it_b; it0 += 48) q_period<0, false>(F, it0);  // warm-up: no stores
    if (kind == 0 && U.part > 0) {
      R4Bound& B = bounds[U.bnd + U.part - 1];
#pragma unroll
      for (int q = 0; q < 4; ++q) B.v_start[64 * q + lane] = F.V[q] & kStrip;
      if (l == 0) {
        B.m_start[2 * m] = m0_at(it_b, 0);
        B.m_start[2 * m + 1] = m0_at(it_b, 1);
      }
    }
    for (; it0 < it_e; it0 += 48) q_period<0, true>(F, it0);
  }
  if (kind == 0 && split && U.part < U.n_parts - 1) {
    R4Bound& B = bounds[U.bnd + U.part];
#pragma unroll
    for (int q = 0; q < 4; ++q) B.v_end[64 * q + lane] = F.V[q] & kStrip;
    if (l == 0) {
      B.m_end[2 * m] = m0_at(it_e, 0);
      B.m_end[2 * m + 1] = m0_at(it_e, 1);
    }
    return;
  }

  // final metrics: position p holds state rotr(p, 2 (it_e mod 3))
  const int rot = (2 * (it_e % 3)) % KM1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const Item& it = h ? itb : ita;
    const bool valid = h ? vb : va;
    uint32_t val[4];
    uint32_t key = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      val[q] = ((F.V[q] & kStrip) >> (16 * h)) & 0xFFFFu;
      const int js_q = rotr_n(l + 16 * q, rot, KM1);
      const uint32_t kq = (val[q] << 8) | (uint32_t)(255 - js_q);
      key = kq > key ? kq : key;
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const uint32_t other = (uint32_t)__shfl_xor((int)key, o);
      key = other > key ? other : key;
    }
    const bool fixed = it.end_state >= 0;
    const int js = fixed ? it.end_state : 255 - (int)(key & 255);
    const int pos = rotl_n(js & 63, rot, KM1);
    const int src = 16 * m + (pos & 15);
    uint32_t vfix = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t x = (uint32_t)__shfl((int)val[q], src);
      vfix = (pos >> 4) == q ? x : vfix;
    }
    const uint32_t vbest = fixed ? vfix : key >> 8;
    if (l == 0 && valid) {
      item_end[it.slot] = js;
      const int64_t o = (int64_t)(h ? F.off1 : F.off0);
      const int64_t local = ((int64_t)vbest - (int64_t)kBase + o) / 4 -
                            (int64_t)(kBias / 4) * (it_e - s0) -
                            (first_part ? (int64_t)kLeadOff * lead : 0);
      if (kind == 0 && split) {
        last_m[it.slot] = local;  // completed by the check
        if (it.frame >= 0 && end_out) end_out[it.frame] = js;
      } else if (it.frame >= 0) {
        if (end_out) end_out[it.frame] = js;
        if (metric) metric[it.frame] = local + (kind == 1 ? rep_m0[it.slot] : 0);
      }
    }
  }
}

__global__ __launch_bounds__(64 * r4q::kWaves, 2) void k_fwd_r4q(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ units, int n_units, const int32_t* dev_count, int kind,
    R4Bound* bounds, int64_t* last_m, const int64_t* rep_m0, const int8_t* __restrict__ llr,
    uint64_t* __restrict__ surv, int64_t* metric, int32_t* end_out, int32_t* item_end,
    int32_t* counter) {
  __shared__ __align__(16) uint32_t tbl_all[r4q::kWaves][3 * r4q::kBufWords];
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (dev_count) n_units = min(n_units, __builtin_amdgcn_readfirstlane(*dev_count));
  if (counter == nullptr) {
    const int u = blockIdx.x * r4q::kWaves + wid;
    if (u >= n_units) return;  // no workgroup barriers: safe to leave
    fwd_r4q_wave(codes, items, units[u], kind, bounds, last_m, rep_m0, llr, surv, metric,
                 end_out, item_end, tbl_all[wid], lane);
    return;
  }
  for (;;) {
    int w = 0;
    if (lane == 0) w = atomicAdd(counter, 1);
    w = __builtin_amdgcn_readfirstlane(w);
    if (w >= n_units) break;
    fwd_r4q_wave(codes, items, units[w], kind, bounds, last_m, rep_m0, llr, surv, metric,
                 end_out, item_end, tbl_all[wid], lane);
  }
}

// Check of the four-state kernel's split entries, with repairs in place.
__global__ __launch_bounds__(64 * r4q::kWaves, 2) void k_r4q_check(
    const DevCode* __restrict__ codes, const Item* __restrict__ items,
    const SplitUnit* __restrict__ split, int n_split, R4Bound* bounds,
    const int64_t* __restrict__ last_m, int64_t* rep_m0, const int8_t* __restrict__ llr,
    uint64_t* __restrict__ surv, int64_t* metric, int32_t* end_out, int32_t* item_end) {
  __shared__ __align__(16) uint32_t tbl_all[r4q::kWaves][3 * r4q::kBufWords];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = blockIdx.x * r4q::kWaves + wid;
  if (e >= n_split) return;  // no workgroup barriers: safe to leave
  const SplitUnit U = split[e];
  const EntryCheck c = check_entry<256>(U, bounds, lane);
  const bool mine = lane < U.count;
  const Item it = items[U.first + (mine ? lane : 0)];
  if (c.fail < 0) {
    if (mine && metric && it.frame >= 0) metric[it.frame] = last_m[it.slot] + c.D;
    return;
  }
  if (mine) rep_m0[it.slot] = c.T;
  __threadfence();
  fwd_r4q_wave(codes, items, repair_unit(U, bounds, c.fail, items[U.first].n_stages), 1, bounds,
               const_cast<int64_t*>(last_m), rep_m0, llr, surv, metric, end_out, item_end,
               tbl_all[wid], lane);
}

// Forward pass of a part; split entries are then checked (and repaired in
// place) by one more launch.
hipError_t launch_fwd_r4p(int K, const DevCode* codes, const Item* items, const SplitUnit* units,
                          int n_units, const int8_t* llr, uint64_t* surv, int64_t* metric,
                          int32_t* end_out, int32_t* item_end, int32_t* counter, int grid_limit,
                          R4Bound* bounds, int64_t* last_m, const SplitUnit* split, int n_split,
                          int64_t* rep_m0, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  if (K != 5 && K != 7) return hipErrorInvalidValue;
  auto kernel = K == 7 ? k_fwd_r4p<3> : k_fwd_r4p<2>;
  const int threads = 64 * r4p::kR4Waves;
  int nb = (n_units + r4p::kR4Waves - 1) / r4p::kR4Waves;
  if (counter) {
    const int lim = grid_limit > 0 ? grid_limit : resident_workgroups(kernel, threads);
    if (lim > 0 && nb > lim) nb = lim;
  }
  hipLaunchKernelGGL(kernel, dim3(nb), dim3(threads), 0, st, codes, items, units, n_units,
                     (const int32_t*)nullptr, 0, bounds, last_m, (const int64_t*)nullptr, llr,
                     surv, metric, end_out, item_end, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_split <= 0) return e;
  auto check = K == 7 ? k_r4p_check<3> : k_r4p_check<2>;
  const int ns = (n_split + r4p::kR4Waves - 1) / r4p::kR4Waves;
  hipLaunchKernelGGL(check, dim3(ns), dim3(threads), 0, st, codes, items, split, n_split, bounds,
                     (const int64_t*)last_m, rep_m0, llr, surv, metric, end_out, item_end);
  return hipGetLastError();
}

hipError_t launch_fwd_r4q(const DevCode* codes, const Item* items, const SplitUnit* units,
                          int n_units, const int8_t* llr, uint64_t* surv, int64_t* metric,
                          int32_t* end_out, int32_t* item_end, int32_t* counter, int grid_limit,
                          R4Bound* bounds, int64_t* last_m, const SplitUnit* split, int n_split,
                          int64_t* rep_m0, hipStream_t st) {
  if (n_units <= 0) return hipSuccess;
  const int threads = 64 * r4q::kWaves;
  int nb = (n_units + r4q::kWaves - 1) / r4q::kWaves;
  if (counter) {
    const int lim = grid_limit > 0 ? grid_limit : resident_workgroups(k_fwd_r4q, threads);
    if (lim > 0 && nb > lim) nb = lim;
  }
  hipLaunchKernelGGL(k_fwd_r4q, dim3(nb), dim3(threads), 0, st, codes, items, units, n_units,
                     (const int32_t*)nullptr, 0, bounds, last_m, (const int64_t*)nullptr, llr,
                     surv, metric, end_out, item_end, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_split <= 0) return e;
  const int ns = (n_split + r4q::kWaves - 1) / r4q::kWaves;
  hipLaunchKernelGGL(k_r4q_check, dim3(ns), dim3(threads), 0, st, codes, items, split, n_split,
                     bounds, (const int64_t*)last_m, rep_m0, llr, surv, metric, end_out,
                     item_end);
  return hipGetLastError();
}

hipError_t launch_tb_r4p(int K, const Item* items, const int2* pairs, int n_pairs,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits, int warm,
                         hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  if (K == 7)
    hipLaunchKernelGGL(k_tb_r4p<3>, dim3(n_pairs), dim3(64), 0, st, items, pairs, surv, item_end,
                       bits, warm);
  else if (K == 5)
    hipLaunchKernelGGL(k_tb_r4p<2>, dim3(n_pairs), dim3(64), 0, st, items, pairs, surv, item_end,
                       bits, warm);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mivit
