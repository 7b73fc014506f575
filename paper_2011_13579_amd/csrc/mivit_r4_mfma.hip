// Radix-4 forward procedure with the candidate additions of Eq. (radix4:PM)
// done by the int8 matrix cores: the tensor-core mapping of §V-A and §VIII-C
// with the dragonfly groups of §VIII-D-2, carried to gfx950's
// v_mfma_i32_16x16x32_i8.  K = 7, rate 1/2, int8 soft values, exact integers.
//
// One wavefront per frame.  Lane l holds state l (4 x its path metric, low
// two bits zero).  One iteration (two stages) is one 16 x 16 x 32 product
//   D = A * B + C,   D[(z, y'), f] = candidate of right state 16 z + f from
//                    left state 4 f + (y' ^ a_f), plus the tie tag 3 - y,
// where the columns are the 16 dragonflies f, the rows the 16 branches
// (z, y') of a dragonfly (z = 2 u2 + u1 the two new input bits, y' the
// permuted left index), and the inner dimension holds, per dragonfly group
// g, the four soft values of the iteration:
//   A[(z, y'), 4 g + b] = 4 (-1)^{bit b of the leader's super-branch output
//                         for (y', z)}        (Eq. (radix4:branchOutMat)),
//   A[(z, y'), 16 + t]  = [y' == t],
//   B[4 g + b, f]       = l_b if f belongs to group g, else 0,
//   B[16 + t, f]        = 3 - (t ^ a_f)         (the tie tag of row t),
//   C[(z, y'), f]       = 4 PM(4 f + (y' ^ a_f)).
// Dragonfly f's super-branch outputs equal those of its group's leader with
// the left index y replaced by y ^ a_f (§VIII-D-2: dragonflies of a group
// have the same matrix up to a permutation of their left states), so four
// leader matrices side by side in A serve all sixteen dragonflies.
//
// In the 16 x 16 result lane l holds rows 4 (l/16) .. 4 (l/16) + 3 of column
// l mod 16: the four candidates of right state l.  Their maximum (three
// compares) is the new metric with the winner's tag 3 - y in its low bits:
// among equal candidates the smallest y wins, the lower-index previous
// state of the paper's strict comparison.  The C operand of the next
// iteration is gathered with four ds_bpermute from lanes 4 f + (i ^ a_f).
//
// Decisions are written in the natural radix-4 layout of the generic
// kernels (one 64-bit word per stage: for the stage pair (t, t+1), word t
// holds bit 0 of y and word t+1 bit 1), so the segmented traceback reads
// them; an odd stage count ends with one radix-2 stage on the vector ALU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mivit_device.h"

namespace mivit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kUnreach = -(1 << 29);  // 4 x metric of unreachable states

__host__ __device__ inline int par(uint32_t x) { return __builtin_popcount(x) & 1; }

__host__ __device__ inline int out2(const int32_t K, const uint32_t* gen, int i, int u) {
  const uint32_t reg = ((uint32_t)u << (K - 1)) | (uint32_t)i;
  return par(gen[0] & reg) | (par(gen[1] & reg) << 1);
}

// 4-bit super-branch output (Eq. (radix4:BM)) of left state 4 f + y and the
// two inputs z = 2 u2 + u1: stage one's two bits, then stage two's.
__host__ __device__ inline int super_out(const int32_t K, const uint32_t* gen, int f, int y, int z) {
  const int i = 4 * f + y, u1 = z & 1, u2 = z >> 1;
  const int m = (u1 << (K - 2)) | (i >> 1);
  return out2(K, gen, i, u1) | (out2(K, gen, m, u2) << 2);
}

}  // namespace

bool mfma_groups(int K, int beta, const uint32_t* gen, MfmaGroups* G) {
  if (K != 7 || beta != 2) return false;
  int n = 0;
  for (int g = 0; g < 4; ++g) G->leader[g] = -1;
  for (int f = 0; f < 16; ++f) {
    bool found = false;
    for (int g = 0; g < n && !found; ++g)
      for (int a = 0; a < 4 && !found; ++a) {
        bool same = true;
        for (int y = 0; y < 4 && same; ++y)
          for (int z = 0; z < 4 && same; ++z)
            same = super_out(K, gen, f, y, z) == super_out(K, gen, G->leader[g], y ^ a, z);
        if (same) {
          G->group[f] = g;
          G->a[f] = a;
          found = true;
        }
      }
    if (!found) {
      if (n == 4) return false;
      G->leader[n] = f;
      G->group[f] = n;
      G->a[f] = 0;
      ++n;
    }
  }
  return true;
}

__global__ __launch_bounds__(64 * kWaves) void k_fwd_r4_mfma(
    const DevCode* __restrict__ codes, const Item* __restrict__ items, int n_items,
    const int8_t* __restrict__ llr, uint64_t* __restrict__ surv, int64_t* metric,
    int32_t* end_out, int32_t* item_end, MfmaGroups G) {
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (item >= n_items) return;  // whole wavefronts leave; no workgroup barriers follow
  const Item it = items[item];
  const DevCode c = codes[it.code];
  const int q = lane >> 4, col = lane & 15;
  // A: row lane mod 16 = (z, y'), inner slots 8q .. 8q+7
  uint64_t A = 0;
  {
    const int r = lane & 15, z = r >> 2, yp = r & 3;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * q + e;
      int v = 0;
      if (k < 16) {
        const int L = G.leader[k >> 2];
        if (L >= 0) v = ((super_out(c.K, c.gen, L, yp, z) >> (k & 3)) & 1) ? -4 : 4;
      } else if (k < 20) {
        v = (k - 16) == yp ? 1 : 0;
      }
      A |= (uint64_t)(uint8_t)(int8_t)v << (8 * e);
    }
  }
  // B: lanes q = 0, 1 take the soft values for groups 2q, 2q+1 of their
  // column's dragonfly; lanes q = 2 hold the tie tags; q = 3 zero
  const int gcol = G.group[col], acol = G.a[col];
  const bool sel_lo = q < 2 && gcol == 2 * q;
  const bool sel_hi = q < 2 && gcol == 2 * q + 1;
  uint32_t tags = 0;
  if (q == 2)
    for (int t = 0; t < 4; ++t) tags |= (uint32_t)(3 - (t ^ acol)) << (8 * t);
  int src[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) src[i] = (4 * col + (i ^ acol)) * 4;

  const bool odd = lane & 1;
  const int S = it.n_stages, n_pairs = S >> 1;
  const int8_t* l = llr + it.llr_off;
  uint64_t* sv = surv + it.surv_off;
  int P = (it.start_known && lane != 0) ? kUnreach : 0;
  int64_t off4 = 0;  // 4 x the amount subtracted by renormalisation
  for (int p0 = 0, t0 = 0; t0 < S; p0 += 32, t0 += 64) {
    if (t0 > 0) {  // state 0 (lane 0) back to zero; every state is reachable by now
      const int ref = __builtin_amdgcn_readfirstlane(P);
      P -= ref;
      off4 += ref;
    }
    uint32_t wreg = 0;  // soft values of pair p0 + lane
    if (lane < 32 && p0 + lane < n_pairs) __builtin_memcpy(&wreg, l + 4 * (int64_t)(p0 + lane), 4);
    uint32_t dlo = 0, dhi = 0;  // decision word of stage t0 + lane
    const int np = min(32, n_pairs - p0);
    for (int k = 0; k < np; ++k) {
      const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)wreg, k);
      const uint32_t blo = sel_lo ? w : tags;
      const uint32_t bhi = sel_hi ? w : 0u;
      const long B = (long)(((uint64_t)bhi << 32) | blo);
      v4i C;
#pragma unroll
      for (int i = 0; i < 4; ++i) C[i] = __builtin_amdgcn_ds_bpermute(src[i], P);
      const v4i D = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)A, B, C, 0, 0, 0);
      const int W = max(max(D[0], D[1]), max(D[2], D[3]));
      const uint64_t m0 = __ballot(!(W & 1));  // bit 0 of y = 3 - tag
      const uint64_t m1 = __ballot(!(W & 2));  // bit 1 of y
      // lanes 2k and 2k+1 keep the words of stages t0 + 2k and t0 + 2k + 1
      const uint64_t m = odd ? m1 : m0;
      const bool mine = (lane >> 1) == k;
      dlo = mine ? (uint32_t)m : dlo;
      dhi = mine ? (uint32_t)(m >> 32) : dhi;
      P = W & ~3;
    }
    if ((S & 1) && t0 + 64 >= S) {
      // the last stage of an odd count: one radix-2 stage (Eq. (PM))
      const int t = S - 1;
      const int l0 = l[2 * (int64_t)t], l1 = l[2 * (int64_t)t + 1];
      const int f2 = lane & 31, u = lane >> 5;
      const int o0 = out2(c.K, c.gen, 2 * f2, u), o1 = out2(c.K, c.gen, 2 * f2 + 1, u);
      const int b0 = ((o0 & 1) ? -l0 : l0) + ((o0 & 2) ? -l1 : l1);
      const int b1 = ((o1 & 1) ? -l0 : l0) + ((o1 & 2) ? -l1 : l1);
      const int c0 = __builtin_amdgcn_ds_bpermute(8 * f2, P) + 4 * b0;
      const int c1 = __builtin_amdgcn_ds_bpermute(8 * f2 + 4, P) + 4 * b1;
      const bool d = c1 > c0;  // strict: a tie keeps the lower previous state
      const uint64_t m = __ballot(d);
      if (lane == t - t0) {
        dlo = (uint32_t)m;
        dhi = (uint32_t)(m >> 32);
      }
      P = d ? c1 : c0;
    }
    if (t0 + lane < S) sv[t0 + lane] = ((uint64_t)dhi << 32) | dlo;
  }
  // final state: fixed, or the best (lowest index on ties)
  int js = it.end_state;
  if (js < 0) {
    int best = P;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) best = max(best, __shfl_xor(best, o));
    const uint64_t at = __ballot(P == best);
    js = (int)__builtin_ctzll(at);
  }
  const int Pjs = __shfl(P, js);
  if (lane == 0) {
    item_end[it.slot] = js;
    if (it.frame >= 0) {
      if (end_out) end_out[it.frame] = js;
      if (metric) metric[it.frame] = ((int64_t)Pjs + off4) / 4;
    }
  }
}

hipError_t launch_fwd_r4_mfma(const MfmaGroups& G, const DevCode* codes, const Item* items,
                              int n_items, const int8_t* llr, uint64_t* surv, int64_t* metric,
                              int32_t* end_out, int32_t* item_end, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const int nb = (n_items + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(k_fwd_r4_mfma, dim3(nb), dim3(64 * kWaves), 0, st, codes, items, n_items,
                     llr, surv, metric, end_out, item_end, G);
  return hipGetLastError();
}

}  // namespace mivit
