// C ABI of the Viterbi decoder library: argument validation, plan building
// (chunking of long frames into overlapping windows, §III), one part per code
// with its own kernel choice, work ordering, scheduling (concurrent parts on
// plan-owned streams, persistent work-queue launches, graph capture), the
// autotuner, device memory ownership and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mivit.h"
#include "mivit_device.h"

namespace mivit {
hipError_t launch_fwd(int radix, int nsl, int dt, const DevCode* codes, const Item* items,
                      int n_items, const void* llr, uint64_t* surv, void* metric,
                      int32_t* end_out, int32_t* item_end, hipStream_t st);
hipError_t launch_grad(const DevCode* codes, const GradFrame* frames, int n_frames,
                       int max_stages, const uint32_t* bits, const float* gm, float* grad,
                       hipStream_t st);
hipError_t launch_quant(const float* x, int8_t* q, int64_t n, float scale, hipStream_t st);
hipError_t launch_fwd_rot(int K, int beta, int dt, int mode, const DevCode* codes,
                          const Item* items, const int2* waves, int n_waves, const void* llr,
                          uint64_t* surv, void* metric, int32_t* end_out, int32_t* item_end,
                          int32_t* counter, int grid_limit, hipStream_t st);
hipError_t launch_fwd_wide(int K, int beta, int dt, int wpf, bool packed, const DevCode* codes,
                           const Item* items,
                           const SplitUnit* units, int n_units, const void* llr, uint64_t* surv,
                           void* metric, int32_t* end_out, int32_t* item_end, WideBound* bounds,
                           int64_t* last_m, const SplitUnit* split, int n_split, int64_t* rep_m0,
                           SplitUnit* rep_units, int32_t* rep_count, hipStream_t st);
hipError_t launch_tb_seg(int layout, const DevCode* codes, const Item* items, int n_items,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits,
                         int warm, hipStream_t st);
hipError_t launch_fwd_r4p(int K, const DevCode* codes, const Item* items, const SplitUnit* units,
                          int n_units, const int8_t* llr, uint64_t* surv, int64_t* metric,
                          int32_t* end_out, int32_t* item_end, int32_t* counter, int grid_limit,
                          R4Bound* bounds, int64_t* last_m, const SplitUnit* split, int n_split,
                          int64_t* rep_m0, hipStream_t st);
hipError_t launch_fwd_r4q(const DevCode* codes, const Item* items, const SplitUnit* units,
                          int n_units, const int8_t* llr, uint64_t* surv, int64_t* metric,
                          int32_t* end_out, int32_t* item_end, int32_t* counter, int grid_limit,
                          R4Bound* bounds, int64_t* last_m, const SplitUnit* split, int n_split,
                          int64_t* rep_m0, hipStream_t st);
hipError_t launch_tb_r4p(int K, const Item* items, const int2* pairs, int n_pairs,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits, int warm,
                         hipStream_t st);
hipError_t launch_fwd_r4_mfma(const MfmaGroups& G, const DevCode* codes, const Item* items,
                              int n_items, const int8_t* llr, uint64_t* surv, int64_t* metric,
                              int32_t* end_out, int32_t* item_end, hipStream_t st);
hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t st);
hipError_t launch_fill_random(void* p, int64_t n, int dt, uint32_t seed, hipStream_t st);
}  // namespace mivit

using namespace mivit;

// forward kernels and the survivor layouts they write
enum : int {
  kKernGeneric2 = 0,
  kKernGeneric4 = 1,
  kKernRot2 = 2,
  kKernRot4P = 3,
  kKernWide = 4,
  kKernGeneric8 = 5,
  kKernMfma4 = 6,  // radix 4, candidate additions on the int8 matrix cores
  kKernRot4Q = 7,  // packed radix 4 with four states per lane (K = 7)
};
enum : int {
  kLayoutNatR2 = 0,
  kLayoutNatR4 = 1,
  kLayoutRotR2 = 2,
  kLayoutRot4P = 3,
  kLayoutRotByte = 4,  // per 8 stages, 2^(K-1) bytes of positions (wide kernel)
  kLayoutNatR8 = 5,
};
constexpr int kWarmStages = 64;  // speculative traceback warm-up
// The packed radix-4 traceback runs one wavefront per frame pair, so one
// mis-started segment (whose boundary state disagrees with the exact lane
// above) re-chases a whole segment while the rest of the grid idles: a
// longer warm-up that makes repairs rare costs less than the repairs
// (4096 x 8192 K=7 frames at 3 dB: 64 stages 0.095 ms, 80 0.085, 96 0.073,
// 112 0.073, 128 0.076).  The radix-2 tracebacks measured best at 64.
constexpr int kWarmStagesR4P = 96;
// rotating forward kernel: its MODE template argument per plan variant.
// Variant 0 (MODE 2): all exchanges in the VALU (DPP, permlane swaps);
// variant 1 (MODE 0): both previous-state metrics via DPP/LDS swizzles;
// variant 2 (MODE 1): one partner metric via DPP/LDS swizzles.
constexpr int kRotMode[3] = {2, 0, 1};
constexpr int kMaxAux = 4;     // plan-owned streams for concurrent parts
constexpr int kMaxGraphs = 8;  // recorded decode graphs kept per plan

// Kernel choice of one part (all frames of one code).
struct Choice {
  int radix = 2;
  int variant = 0;
  bool persistent = false;
  bool split = true;  // packed radix 4: split long frame pairs in time
};

// Time split of the packed radix-4 forward: frame pairs are cut into parts
// of whole 48-iteration periods (the digit-map period times the table
// block), later parts warming up for kSplitWarm iterations (192 stages)
// from all-zero metrics.  Parts are added until the batch has about
// kSplitWavesPerSimd wavefronts per SIMD, each part at least kSplitMinIt
// iterations long.
constexpr int kSplitAlign = 48;
constexpr int kSplitWarm = 96;
constexpr int kSplitMinIt = 384;
constexpr int kSplitMaxParts = kMaxSplitParts;
constexpr int kSplitWavesPerSimd = 4;
// The four-states-per-lane kernel holds eight frames per wavefront and four
// independent chains per lane: it targets fewer wavefronts per SIMD.
constexpr int kSplitWavesPerSimdQ = 2;
// Time split of the K = 8, 9 radix-2 kernel (int8): a frame is cut into
// about S / len parts of whole lcm(32, K-1)-stage periods, len being the
// batch's stages per wavefront slot (at least kWideSplitLen), later parts
// warming up for at least kWideSplitWarm stages.
constexpr int kWideSplitLen = 1024;
constexpr int kWideSplitWarm = 192;

// Wavefronts per frame of the K = 8, 9 radix-2 kernel: variants 6 and 7
// spread a float32 frame's states over two or four wavefronts.
int waves_per_frame(const Choice& ch) { return ch.variant == 6 ? 2 : ch.variant == 7 ? 4 : 1; }

struct PlanGroup {
  int kern;   // forward kernel
  int layout; // survivor layout (selects the traceback)
  int nsl;    // generic kernels: states per lane
  int K, beta;
  int first;  // first item of the group
  int count;
  int wave_off;  // rotating kernels: first entry of the group in the wave table
  int n_waves;
  int pair_off;  // packed radix-4 kernel: first entry in the traceback pair table
  int n_pairs;
  int counter;   // persistent launch: index of the group's work counter, else -1
};

struct Part {
  int code = 0;
  Choice ch;
  std::vector<Item> items;
  std::vector<PlanGroup> groups;
  int64_t surv_words = 0;
  int64_t total_stages = 0;
  Item* d_items = nullptr;
  int32_t* d_item_end = nullptr;
  uint64_t* d_surv = nullptr;
  int2* d_waves = nullptr;  // rotating kernels: (first item, count) per wavefront
  int2* d_pairs = nullptr;  // packed radix-4 traceback: (first item, count) per frame pair
  int32_t* d_counters = nullptr;
  int n_counters = 0;
  // packed radix 4: work units (parts of entries), split entries' part-0
  // units, boundary records, last-part metrics, repair units and count
  SplitUnit* d_units = nullptr;
  int n_units = 0;
  SplitUnit* d_split = nullptr;
  int n_split = 0;
  R4Bound* d_bounds = nullptr;
  WideBound* d_wbounds = nullptr;  // K = 8, 9 radix-2 kernel
  int64_t* d_last_m = nullptr;
  int64_t* d_rep_m0 = nullptr;
  SplitUnit* d_rep_units = nullptr;
  int32_t* d_rep_count = nullptr;
  MfmaGroups mg{};  // dragonfly groups (matrix-core radix-4 kernel)
};

struct GraphEntry {
  const void* llr;
  uint32_t* bits;
  void* metric;
  int32_t* end;
  hipStream_t stream;
  hipGraphExec_t exec;
};

struct mivit_plan {
  int device = 0;
  int dtype = MIVIT_F32;
  uint32_t flags = 0;
  int n_frames = 0;
  int64_t llr_end = 0;   // soft values the frames address
  int64_t word_end = 0;  // output words the frames address
  bool grad_ok = false;
  int grad_max_stages = 0;
  DevCode* d_codes = nullptr;
  GradFrame* d_gframes = nullptr;
  std::vector<Part> parts;
  hipStream_t origin = nullptr;  // capture stream
  std::vector<hipStream_t> aux;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  std::vector<GraphEntry> graphs;
};

namespace {

// Kernel launches report failure through hipGetLastError, which would also
// return an unrelated earlier failure of the calling thread (another
// library's, say): every entry point that launches clears it first.
inline void clear_stale_error() { (void)hipGetLastError(); }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    clear_stale_error();
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

mivit_status check_code(const mivit_code& c) {
  if (c.K < 3 || c.K > kMaxK || c.beta < 2 || c.beta > 4) return MIVIT_EINVAL;
  for (int b = 0; b < c.beta; ++b) {
    if (c.gen[b] == 0 || c.gen[b] >= (1u << c.K)) return MIVIT_EINVAL;
    // premise of the branch-output corollary (§IV): MSB and LSB taps set
    if (!((c.gen[b] >> (c.K - 1)) & 1u) || !(c.gen[b] & 1u)) return MIVIT_EUNSUPPORTED;
  }
  return MIVIT_OK;
}

int nsl_of(int K) { return K <= 7 ? 1 : (1 << (K - 1)) / 64; }

bool packed_ok(const mivit_code& c) { return c.beta == 2 && (c.K == 5 || c.K == 7); }
bool quad_ok(const mivit_code& c) { return c.beta == 2 && c.K == 7; }

// The matrix-core radix-4 kernel: K = 7, rate 1/2, at most four dragonfly groups.
bool mfma_ok(const mivit_code& c) {
  MfmaGroups g;
  return mfma_groups(c.K, c.beta, c.gen, &g);
}

mivit_status hip_status(hipError_t e) {
  return e == hipSuccess ? MIVIT_OK : (e == hipErrorOutOfMemory ? MIVIT_ENOMEM : MIVIT_EHIP);
}

void free_part(Part& q) {
  (void)hipFree(q.d_items);
  (void)hipFree(q.d_item_end);
  (void)hipFree(q.d_surv);
  (void)hipFree(q.d_waves);
  (void)hipFree(q.d_pairs);
  (void)hipFree(q.d_counters);
  (void)hipFree(q.d_units);
  (void)hipFree(q.d_split);
  (void)hipFree(q.d_bounds);
  (void)hipFree(q.d_wbounds);
  (void)hipFree(q.d_last_m);
  (void)hipFree(q.d_rep_m0);
  (void)hipFree(q.d_rep_units);
  (void)hipFree(q.d_rep_count);
  q = Part();
}

void free_plan(mivit_plan* p) {
  if (!p) return;
  for (GraphEntry& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  for (Part& q : p->parts) free_part(q);
  (void)hipFree(p->d_codes);
  (void)hipFree(p->d_gframes);
  for (hipEvent_t e : p->ev_join) (void)hipEventDestroy(e);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  for (hipStream_t s : p->aux) (void)hipStreamDestroy(s);
  if (p->origin) (void)hipStreamDestroy(p->origin);
  delete p;
}

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n) {
  *dst = nullptr;
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

// Work items of the frames fidx (all of one code): whole frames, or the
// windows of §III for frames longer than the chunk.
void expand_items(const mivit_code* codes, const mivit_frame* frames, const std::vector<int>& fidx,
                  const mivit_opts& o, std::vector<Item>& items) {
  for (int f : fidx) {
    const mivit_frame& fr = frames[f];
    const mivit_code& c = codes[fr.code];
    const int S = fr.n_stages;
    if (o.chunk > 0 && S > o.chunk) {
      for (int c0 = 0; c0 < S; c0 += o.chunk) {
        const int c1 = std::min(S, c0 + o.chunk);
        const int w0 = std::max(0, c0 - o.overlap);
        const int w1 = std::min(S, c1 + o.overlap);
        const bool last = c1 == S;
        const int e1 = std::min(c1, fr.n_out);
        const int nout = e1 > c0 ? e1 - c0 : 0;
        if (nout == 0 && !last) continue;
        Item it;
        std::memset(&it, 0, sizeof it);
        it.llr_off = fr.llr_offset + (int64_t)w0 * c.beta;
        it.bit_off = fr.bit_offset + c0;
        it.n_stages = w1 - w0;
        it.out_begin = c0 - w0;
        it.n_out = nout;
        it.code = fr.code;
        it.start_known = (w0 == 0) && (fr.flags & MIVIT_START_KNOWN);
        it.end_state = (last && (fr.flags & MIVIT_END_ZERO)) ? 0 : -1;
        it.frame = last ? f : -1;
        items.push_back(it);
      }
    } else {
      Item it;
      std::memset(&it, 0, sizeof it);
      it.llr_off = fr.llr_offset;
      it.bit_off = fr.bit_offset;
      it.n_stages = S;
      it.out_begin = fr.out_begin;
      it.n_out = fr.n_out;
      it.code = fr.code;
      it.start_known = (fr.flags & MIVIT_START_KNOWN) ? 1 : 0;
      it.end_state = (fr.flags & MIVIT_END_ZERO) ? 0 : -1;
      it.frame = f;
      items.push_back(it);
    }
  }
}

// The four-state radix-4 kernel holds eight frames of one length per
// wavefront and, with its longer iterations, needs about two wavefronts per
// SIMD (after the time split) to hide latency; batches that fill fewer
// (few frames, or frames of many different lengths) run the one-state
// kernel faster.
bool quad_pays(const std::vector<Item>& items) {
  if (items.empty()) return false;
  std::map<int, int64_t> by_len;  // stages -> frames
  for (const Item& it : items) by_len[it.n_stages]++;
  int64_t entries = 0, waves = 0;
  for (const auto& kv : by_len) {
    const int64_t e = (kv.second + 7) / 8;
    entries += e;
    waves += e * std::max(1, std::min(kSplitMaxParts, (kv.first >> 1) / kSplitMinIt));
  }
  if (24 * entries > 4 * (int64_t)items.size()) return false;  // entries under 3/4 full
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  return waves >= 2 * 4 * (int64_t)cus;
}

// Build one part: kernel per item, groups, wave and pair tables, survivor
// memory, device copies.
mivit_status build_part(const mivit_code* codes, const mivit_frame* frames,
                        const std::vector<int>& fidx, const mivit_opts& o, int dtype, Choice ch,
                        int code, Part& q) {
  q = Part();
  q.code = code;
  q.ch = ch;
  std::vector<Item> items;
  expand_items(codes, frames, fidx, o, items);
  const mivit_code& c = codes[code];
  const bool i8 = dtype == MIVIT_I8;
  int kern;
  if (ch.radix == 8)
    kern = kKernGeneric8;
  else if (ch.radix == 4 && ch.variant == 3)
    kern = kKernMfma4;
  else if (ch.radix == 4 && ch.variant == 4)
    kern = kKernRot4P;  // packed, one state per lane (the K = 5 default)
  else if (ch.radix == 4 && ch.variant == 5)
    kern = kKernRot4Q;  // packed, four states per lane, whatever the batch
  else if (ch.radix == 4 && ch.variant == 0 && packed_ok(c) && i8)
    kern = quad_ok(c) && quad_pays(items) ? kKernRot4Q : kKernRot4P;
  else if (ch.radix == 4)
    kern = kKernGeneric4;
  else
    kern = c.K <= 7 ? kKernRot2
                    : ((ch.variant == 0 || ch.variant >= 6) ? kKernWide : kKernGeneric2);
  // longest first; items that can share a packed lane group next to each other
  std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
    if (a.n_stages != b.n_stages) return a.n_stages > b.n_stages;
    if (a.out_begin != b.out_begin) return a.out_begin < b.out_begin;
    return a.n_out < b.n_out;
  });
  PlanGroup g;
  g.kern = kern;
  g.layout = kern == kKernRot2      ? kLayoutRotR2
             : (kern == kKernRot4P || kern == kKernRot4Q) ? kLayoutRot4P
             : kern == kKernWide    ? kLayoutRotByte
             : (kern == kKernGeneric4 || kern == kKernMfma4) ? kLayoutNatR4
             : kern == kKernGeneric8 ? kLayoutNatR8
                                     : kLayoutNatR2;
  g.nsl = nsl_of(c.K);
  g.K = c.K;
  g.beta = c.beta;
  g.first = 0;
  g.count = (int)items.size();
  g.wave_off = g.n_waves = g.pair_off = g.n_pairs = 0;
  g.counter = -1;
  for (size_t k = 0; k < items.size(); ++k) {
    items[k].slot = (int32_t)k;
    q.total_stages += items[k].n_stages;
  }
  // rotating kernels: wavefronts of frames of equal length (radix 2: up to
  // 64/2^(K-1) frames; packed radix 4: up to 2*64/2^(K-1), where the two
  // frames of a lane group must also emit the same stages)
  std::vector<int2> waves, pairs;
  std::vector<SplitUnit> units, split;
  std::vector<R4Bound> bounds;
  std::vector<WideBound> wbounds;
  int n_bounds = 0;
  std::vector<char> pair_hi(items.size(), 0);
  if (kern == kKernRot2 || kern == kKernRot4P || kern == kKernRot4Q) {
    const bool packed = kern != kKernRot2;
    const int fpw = kern == kKernRot4Q ? 8 : (packed ? 2 : 1) * (64 >> (c.K - 1));
    for (int k = 0; k < (int)items.size(); ++k) {
      if (!waves.empty()) {
        int2& w = waves.back();
        const Item& prev = items[k - 1];
        bool fits = w.y < fpw && items[w.x].n_stages == items[k].n_stages;
        if (packed && (w.y & 1))
          fits = fits && prev.out_begin == items[k].out_begin && prev.n_out == items[k].n_out;
        if (fits) {
          if (packed) pair_hi[k] = (char)(w.y & 1);
          w.y++;
          continue;
        }
      }
      waves.push_back(make_int2(k, 1));
    }
    g.n_waves = (int)waves.size();
    if (packed) {
      for (const int2& w : waves)
        for (int s = 0; s < w.y; s += 2) pairs.push_back(make_int2(w.x + s, std::min(2, w.y - s)));
      g.n_pairs = (int)pairs.size();
      // work units: whole entries, or parts of entries in time.  The batch
      // is to fill about kSplitWavesPerSimd wavefronts per SIMD: with slots
      // such wavefront places and I iterations over all entries, an entry
      // of n iterations is cut into about n * slots / I parts, so in a
      // batch of mixed lengths the longest entries are cut the most (in a
      // batch of one length every entry gets the same number of parts).
      // Persistent launches keep frame pairs whole.
      int64_t slots = 0, total_it = 0;
      if (ch.split && !ch.persistent && !waves.empty()) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
          slots = (int64_t)cus * 4 * (kern == kKernRot4Q ? kSplitWavesPerSimdQ : kSplitWavesPerSimd);
        for (const int2& w : waves) total_it += items[w.x].n_stages >> 1;
      }
      for (const int2& w : waves) {
        const int n_it = items[w.x].n_stages >> 1;
        int64_t want = 1;
        if (slots > 0 && total_it > 0) want = ((int64_t)n_it * slots + total_it - 1) / total_it;
        const int P = (int)std::max<int64_t>(
            1, std::min<int64_t>(want, std::min(kSplitMaxParts, n_it / kSplitMinIt)));
        SplitUnit u;
        u.first = w.x;
        u.count = w.y;
        u.warm = 0;
        u.n_parts = P;
        u.bnd = P > 1 ? n_bounds : -1;
        // part 0 has no warm-up: it takes kSplitWarm more iterations than
        // the others, so every part runs about T iterations in all
        const int64_t T = ((int64_t)n_it + (int64_t)(P - 1) * kSplitWarm) / P;
        int prev = 0;
        for (int k = 0; k < P; ++k) {
          int end = n_it;
          if (k < P - 1) {
            const int64_t x = T + (int64_t)k * (T - kSplitWarm);  // nearest period boundary
            end = (int)((x + kSplitAlign / 2) / kSplitAlign * kSplitAlign);
            end = std::max(end, prev + kSplitAlign);
            end = std::min(end, n_it - kSplitAlign * (P - 1 - k));
          }
          u.part = k;
          u.it_begin = prev;
          u.it_end = end;
          u.warm = k == 0 ? 0 : std::min(kSplitWarm, prev);
          units.push_back(u);
          if (k == 0 && P > 1) split.push_back(u);
          if (k > 0) {
            R4Bound b;
            std::memset(&b, 0, sizeof b);
            b.it_at = prev;
            bounds.push_back(b);
          }
          prev = end;
        }
        if (P > 1) n_bounds += P - 1;
      }
    }
    if (ch.persistent) g.counter = q.n_counters++;
  }
  // K = 8, 9 radix-2 kernel: one unit per item, int8 frames much longer than
  // the batch's stages per wavefront slot split in time
  if (kern == kKernWide) {
    int64_t total = 0;
    for (const Item& it : items) total += it.n_stages;
    int slots = 4096;
    {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          cus > 0)
        slots = cus * 4 * kSplitWavesPerSimd;
    }
    const int64_t len = std::max<int64_t>(kWideSplitLen, total / slots);
    const int period = (c.K - 1) == 8 ? 32 : 32 * (c.K - 1);  // lcm(32, K-1) for K = 8, 9
    const int warm = (kWideSplitWarm + period - 1) / period * period;
    const bool can = ch.split && dtype == MIVIT_I8;
    for (int k = 0; k < (int)items.size(); ++k) {
      const int S = items[k].n_stages;
      int P = can ? (int)std::min<int64_t>(kSplitMaxParts, (S + len - 1) / len) : 1;
      if (S < 2 * period + warm) P = 1;
      SplitUnit u;
      u.first = k;
      u.count = 1;
      u.n_parts = P;
      u.bnd = P > 1 ? (int)wbounds.size() : -1;
      int prev = 0;
      for (int p = 0; p < P; ++p) {
        const int end = p == P - 1 ? S : (int)((int64_t)S * (p + 1) / P) / period * period;
        u.part = p;
        u.it_begin = prev;
        u.it_end = end;
        u.warm = p == 0 ? 0 : std::min(warm, prev);
        units.push_back(u);
        if (p == 0 && P > 1) split.push_back(u);
        if (p > 0) {
          WideBound b;
          std::memset(&b, 0, sizeof b);
          b.it_at = prev;
          wbounds.push_back(b);
        }
        prev = end;
      }
    }
  }
  // survivor memory, 16-byte aligned per item (per frame pair when packed)
  int64_t words_total = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    Item& it = items[k];
    if ((kern == kKernRot4P || kern == kKernRot4Q) && pair_hi[k]) {
      it.surv_off = items[k - 1].surv_off;
      continue;
    }
    it.surv_off = words_total;
    if (kern == kKernRot2 || kern == kKernWide)
      words_total += surv_words_blocks32(c.K, it.n_stages);
    else if (kern == kKernRot4P || kern == kKernRot4Q)
      words_total += surv_words_r4p(c.K, it.n_stages);
    else
      words_total += surv_words_natural(c.K, it.n_stages);
  }
  words_total += kSurvSlackWords;
  q.surv_words = words_total;
  if (kern == kKernMfma4 && !mfma_groups(c.K, c.beta, c.gen, &q.mg)) return MIVIT_EUNSUPPORTED;
  if (!items.empty()) q.groups.push_back(g);
  q.items = items;
  hipError_t e = upload(&q.d_items, items.data(), items.size());
  if (e == hipSuccess) e = upload(&q.d_waves, waves.data(), waves.size());
  if (e == hipSuccess) e = upload(&q.d_pairs, pairs.data(), pairs.size());
  if (e == hipSuccess && !items.empty())
    e = hipMalloc((void**)&q.d_item_end, items.size() * sizeof(int32_t));
  if (e == hipSuccess && !items.empty())
    e = hipMalloc((void**)&q.d_surv, (size_t)words_total * sizeof(uint64_t));
  if (e == hipSuccess && q.n_counters > 0)
    e = hipMalloc((void**)&q.d_counters, q.n_counters * sizeof(int32_t));
  q.n_units = (int)units.size();
  q.n_split = (int)split.size();
  if (e == hipSuccess) e = upload(&q.d_units, units.data(), units.size());
  if (e == hipSuccess) e = upload(&q.d_split, split.data(), split.size());
  if (e == hipSuccess) e = upload(&q.d_bounds, bounds.data(), bounds.size());
  if (e == hipSuccess) e = upload(&q.d_wbounds, wbounds.data(), wbounds.size());
  if (e == hipSuccess && q.n_split > 0) {
    e = hipMalloc((void**)&q.d_last_m, items.size() * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void**)&q.d_rep_m0, items.size() * sizeof(int64_t));
    if (e == hipSuccess) e = upload(&q.d_rep_units, split.data(), split.size());
    if (e == hipSuccess) e = hipMalloc((void**)&q.d_rep_count, sizeof(int32_t));
  }
  if (e != hipSuccess) {
    free_part(q);
    return hip_status(e);
  }
  return MIVIT_OK;
}

hipError_t part_forward(const mivit_plan* p, const Part& q, const void* llr, void* metric,
                        int32_t* end_state, hipStream_t st) {
  const int dt = p->dtype;  // the kernels number the soft-value types as mivit_dtype does
  for (const PlanGroup& g : q.groups) {
    hipError_t e;
    int32_t* counter = g.counter >= 0 ? q.d_counters + g.counter : nullptr;
    if (counter) {
      e = launch_zero_i32(counter, 1, st);
      if (e != hipSuccess) return e;
    }
    if (g.kern == kKernRot4P)
      e = launch_fwd_r4p(g.K, p->d_codes, q.d_items, q.d_units, q.n_units, (const int8_t*)llr,
                         q.d_surv, (int64_t*)metric, end_state, q.d_item_end, counter, 0,
                         q.d_bounds, q.d_last_m, q.d_split, q.n_split, q.d_rep_m0, st);
    else if (g.kern == kKernRot4Q)
      e = launch_fwd_r4q(p->d_codes, q.d_items, q.d_units, q.n_units, (const int8_t*)llr,
                         q.d_surv, (int64_t*)metric, end_state, q.d_item_end, counter, 0,
                         q.d_bounds, q.d_last_m, q.d_split, q.n_split, q.d_rep_m0, st);
    else if (g.kern == kKernMfma4)
      e = launch_fwd_r4_mfma(q.mg, p->d_codes, q.d_items + g.first, g.count, (const int8_t*)llr,
                             q.d_surv, (int64_t*)metric, end_state, q.d_item_end, st);
    else if (g.kern == kKernWide)
      e = launch_fwd_wide(g.K, g.beta, dt, waves_per_frame(q.ch), q.ch.variant == 8,
                          p->d_codes, q.d_items,
                          q.d_units, q.n_units, llr, q.d_surv, metric, end_state, q.d_item_end,
                          q.d_wbounds, q.d_last_m,
                          q.d_split, q.n_split, q.d_rep_m0, q.d_rep_units, q.d_rep_count, st);
    else if (g.kern == kKernRot2)
      e = launch_fwd_rot(g.K, g.beta, dt, kRotMode[q.ch.variant], p->d_codes, q.d_items,
                         q.d_waves + g.wave_off, g.n_waves, llr, q.d_surv, metric, end_state,
                         q.d_item_end, counter, 0, st);
    else
      e = launch_fwd(g.kern == kKernGeneric4 ? 4 : g.kern == kKernGeneric8 ? 8 : 2, g.nsl, dt,
                     p->d_codes,
                     q.d_items + g.first, g.count, llr, q.d_surv, metric, end_state,
                     q.d_item_end, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t part_traceback(const mivit_plan* p, const Part& q, uint32_t* bits, hipStream_t st) {
  for (const PlanGroup& g : q.groups) {
    hipError_t e =
        g.layout == kLayoutRot4P
            ? launch_tb_r4p(g.K, q.d_items, q.d_pairs + g.pair_off, g.n_pairs, q.d_surv,
                            q.d_item_end, bits, kWarmStagesR4P, st)
            : launch_tb_seg(g.layout, p->d_codes, q.d_items + g.first, g.count, q.d_surv,
                            q.d_item_end, bits, kWarmStages, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

enum : int { kPhaseForward = 1, kPhaseTraceback = 2 };

// Run the phases of every part on 'st'.  Two or more parts run concurrently
// on the plan's streams, forked from and joined back into 'st'.
hipError_t run_parts(mivit_plan* p, int phases, const void* llr, uint32_t* bits, void* metric,
                     int32_t* end_state, hipStream_t st) {
  auto one = [&](const Part& q, hipStream_t s) -> hipError_t {
    hipError_t e = hipSuccess;
    if (phases & kPhaseForward) e = part_forward(p, q, llr, metric, end_state, s);
    if (e == hipSuccess && (phases & kPhaseTraceback)) e = part_traceback(p, q, bits, s);
    return e;
  };
  if (p->parts.size() == 1) return one(p->parts[0], st);
  hipError_t e = hipEventRecord(p->ev_fork, st);
  for (size_t k = 0; k < p->parts.size() && e == hipSuccess; ++k) {
    hipStream_t s = p->aux[k % p->aux.size()];
    if (k < p->aux.size()) e = hipStreamWaitEvent(s, p->ev_fork, 0);
    if (e == hipSuccess) e = one(p->parts[k], s);
  }
  for (size_t k = 0; k < p->aux.size() && e == hipSuccess; ++k) {
    e = hipEventRecord(p->ev_join[k], p->aux[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, p->ev_join[k], 0);
  }
  return e;
}

// Candidate kernel choices of a part, for the autotuner.
std::vector<Choice> candidates(const mivit_code& c, int dtype, int radix) {
  std::vector<Choice> out;
  auto add = [&](int r, int v, bool pers, bool split = true) {
    Choice ch;
    ch.radix = r;
    ch.variant = v;
    ch.persistent = pers;
    ch.split = split;
    out.push_back(ch);
  };
  const bool i8 = dtype == MIVIT_I8;
  if (dtype == MIVIT_F16) {  // the default exchange scheme only
    add(2, 0, false);
    if (c.K <= 7) add(2, 0, true);
    return out;
  }
  // K >= 8: variant 0 holds the states in registers, 1 and 2 exchange through LDS
  if (radix == 0 || radix == 2) {
    if (c.K <= 7) {
      for (int v = 0; v < 3; ++v) add(2, v, false);
      add(2, 0, true);
    } else {
      add(2, 0, false);  // registers (wide kernel)
      add(2, 1, false);  // LDS exchanges (generic kernel)
      if (dtype == MIVIT_F32) add(2, 6, false);  // registers, two wavefronts per frame
      if (dtype == MIVIT_F32 && c.K == 9) add(2, 7, false);  // four wavefronts per frame
      if (i8 && c.beta <= 3) add(2, 8, false);  // two states per register, 16-bit
    }
  }
  if (i8 && (radix == 0 || radix == 4)) {
    if (packed_ok(c)) {
      add(4, 0, false);
      add(4, 0, true);
      add(4, 0, false, false);  // frame pairs not split in time
    }
    add(4, 1, false);
    if (mfma_ok(c)) add(4, 3, false);
    if (quad_ok(c)) {
      add(4, 4, false);  // one state per lane
      add(4, 5, false);  // four states per lane
    }
  }
  if (i8 && (radix == 0 || radix == 8) && c.K >= 4) add(8, 0, false);
  return out;
}

// Time one candidate: two decodes of synthetic soft values, the second
// timed.  Returns milliseconds, or a negative value on failure.
float time_part(mivit_plan* p, const Part& q, const void* llr, uint32_t* bits, void* metric,
                int32_t* end_state) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = -1.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  if (part_forward(p, q, llr, metric, end_state, p->origin) != hipSuccess) goto done;
  if (part_traceback(p, q, bits, p->origin) != hipSuccess) goto done;
  if (hipEventRecord(e0, p->origin) != hipSuccess) goto done;
  if (part_forward(p, q, llr, metric, end_state, p->origin) != hipSuccess) goto done;
  if (part_traceback(p, q, bits, p->origin) != hipSuccess) goto done;
  if (hipEventRecord(e1, p->origin) != hipSuccess) goto done;
  if (hipEventSynchronize(e1) != hipSuccess) goto done;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.0f;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return ms;
}

const char* kern_name(int kern) {
  switch (kern) {
    case kKernGeneric2: return "radix-2 generic";
    case kKernGeneric4: return "radix-4 generic";
    case kKernRot2: return "radix-2 rotating";
    case kKernWide: return "radix-2 rotating, states in registers";
    case kKernRot4P: return "radix-4 packed two-frame";
    case kKernRot4Q: return "radix-4 packed, four states per lane";
    case kKernGeneric8: return "radix-8 generic";
    case kKernMfma4: return "radix-4 matrix-core candidate additions";
  }
  return "?";
}

}  // namespace

extern "C" {

const char* mivit_strerror(mivit_status s) {
  switch (s) {
    case MIVIT_OK: return "ok";
    case MIVIT_EINVAL: return "invalid argument";
    case MIVIT_ENOMEM: return "out of memory";
    case MIVIT_EHIP: return "HIP runtime error";
    case MIVIT_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char* mivit_version(void) { return "mivit 0.2 (gfx950)"; }

mivit_status mivit_plan_create(mivit_plan** out, const mivit_code* codes, int32_t n_codes,
                               const mivit_frame* frames, int32_t n_frames,
                               const mivit_opts* opts) {
  if (!out) return MIVIT_EINVAL;
  *out = nullptr;
  if (!codes || n_codes <= 0 || n_codes > 32767 || n_frames < 0 || (n_frames > 0 && !frames))
    return MIVIT_EINVAL;
  clear_stale_error();
  mivit_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  if (o.dtype != MIVIT_F32 && o.dtype != MIVIT_I8 && o.dtype != MIVIT_F16) return MIVIT_EINVAL;
  if (o.radix != 0 && o.radix != 2 && o.radix != 4 && o.radix != 8) return MIVIT_EINVAL;
  if ((o.radix == 4 || o.radix == 8) && o.dtype != MIVIT_I8) return MIVIT_EINVAL;
  if (o.chunk < 0 || o.overlap < 0 || (o.chunk > 0 && o.chunk % 32 != 0)) return MIVIT_EINVAL;
  if (o.variant < 0 || o.variant > 8) return MIVIT_EINVAL;
  if (o.variant >= 3 && o.variant <= 5 && (o.radix != 4 || o.dtype != MIVIT_I8))
    return MIVIT_EUNSUPPORTED;
  if ((o.variant == 6 || o.variant == 7) &&
      ((o.radix != 0 && o.radix != 2) || o.dtype != MIVIT_F32))
    return MIVIT_EUNSUPPORTED;
  if (o.variant == 8 && ((o.radix != 0 && o.radix != 2) || o.dtype != MIVIT_I8))
    return MIVIT_EUNSUPPORTED;
  if (o.flags & ~(MIVIT_PLAN_GRAPH | MIVIT_PLAN_AUTOTUNE | MIVIT_PLAN_PERSISTENT |
                  MIVIT_PLAN_NO_SPLIT))
    return MIVIT_EINVAL;
  if (o.reserved[0] != 0 || o.reserved[1] != 0) return MIVIT_EINVAL;
  for (int c = 0; c < n_codes; ++c) {
    mivit_status s = check_code(codes[c]);
    if (s != MIVIT_OK) return s;
  }
  if (o.dtype == MIVIT_F16 && o.variant != 0) return MIVIT_EUNSUPPORTED;
  if (o.variant == 3)
    for (int c = 0; c < n_codes; ++c)
      if (!mfma_ok(codes[c])) return MIVIT_EUNSUPPORTED;
  if (o.variant == 4)
    for (int c = 0; c < n_codes; ++c)
      if (!packed_ok(codes[c])) return MIVIT_EUNSUPPORTED;
  if (o.variant == 5)
    for (int c = 0; c < n_codes; ++c)
      if (!quad_ok(codes[c])) return MIVIT_EUNSUPPORTED;
  if (o.variant == 6 || o.variant == 7)  // 2 or 4 wavefronts per frame: 128 or 256 states
    for (int c = 0; c < n_codes; ++c)
      if (codes[c].K < (o.variant == 6 ? 8 : 9)) return MIVIT_EUNSUPPORTED;
  if (o.variant == 8)  // two states per register, 16-bit metrics: K = 8, 9 and beta <= 3
    for (int c = 0; c < n_codes; ++c)
      if (codes[c].K < 8 || codes[c].beta > 3) return MIVIT_EUNSUPPORTED;
  if (o.radix == 8) {  // one kernel, and at least 8 states
    if (o.variant != 0) return MIVIT_EUNSUPPORTED;
    for (int c = 0; c < n_codes; ++c)
      if (codes[c].K < 4) return MIVIT_EUNSUPPORTED;
  }
  // frames: ranges and non-overlapping outputs
  std::vector<std::pair<int64_t, int64_t>> words;
  words.reserve(n_frames);
  int64_t llr_end = 0, word_end = 0;
  for (int f = 0; f < n_frames; ++f) {
    const mivit_frame& fr = frames[f];
    if (fr.code < 0 || fr.code >= n_codes) return MIVIT_EINVAL;
    if (fr.n_stages < 0 || fr.out_begin < 0 || fr.n_out < 0) return MIVIT_EINVAL;
    if ((int64_t)fr.out_begin + fr.n_out > fr.n_stages) return MIVIT_EINVAL;
    if (fr.llr_offset < 0 || fr.bit_offset < 0 || (fr.bit_offset & 31)) return MIVIT_EINVAL;
    if (fr.flags & ~(MIVIT_START_KNOWN | MIVIT_END_ZERO)) return MIVIT_EINVAL;
    if (o.chunk > 0 && fr.n_stages > o.chunk && fr.out_begin != 0) return MIVIT_EUNSUPPORTED;
    if (fr.n_out > 0) words.push_back({fr.bit_offset >> 5, (fr.bit_offset + fr.n_out + 31) >> 5});
    llr_end = std::max(llr_end, fr.llr_offset + (int64_t)fr.n_stages * codes[fr.code].beta);
    word_end = std::max(word_end, (fr.bit_offset + fr.n_out + 31) >> 5);
  }
  std::sort(words.begin(), words.end());
  for (size_t k = 1; k < words.size(); ++k)
    if (words[k].first < words[k - 1].second) return MIVIT_EINVAL;

  mivit_plan* p = nullptr;
  void* t_llr = nullptr;
  void* t_bits = nullptr;
  void* t_metric = nullptr;
  void* t_end = nullptr;
  mivit_status status = MIVIT_OK;
  try {
    p = new mivit_plan();
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return MIVIT_EHIP;
    }
    p->dtype = o.dtype;
    p->flags = o.flags;
    p->n_frames = n_frames;
    p->llr_end = llr_end;
    p->word_end = word_end;
    std::vector<DevCode> dc(n_codes);
    for (int c = 0; c < n_codes; ++c) {
      dc[c].K = codes[c].K;
      dc[c].beta = codes[c].beta;
      for (int b = 0; b < 4; ++b) dc[c].gen[b] = b < codes[c].beta ? codes[c].gen[b] : 0;
    }
    hipError_t e = upload(&p->d_codes, dc.data(), dc.size());
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->origin, hipStreamNonBlocking);
    if (e != hipSuccess) throw hip_status(e);
    // one part per code, largest work first
    std::vector<std::vector<int>> by_code(n_codes);
    std::vector<int64_t> work(n_codes, 0);
    for (int f = 0; f < n_frames; ++f) {
      by_code[frames[f].code].push_back(f);
      work[frames[f].code] += (int64_t)frames[f].n_stages << (codes[frames[f].code].K - 1);
    }
    std::vector<int> order;
    for (int c = 0; c < n_codes; ++c)
      if (!by_code[c].empty()) order.push_back(c);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    const bool tune = (o.flags & MIVIT_PLAN_AUTOTUNE) != 0;
    if (tune) {
      // synthetic soft values covering every frame, and scratch outputs
      const size_t esz = o.dtype == MIVIT_I8 ? 1 : o.dtype == MIVIT_F16 ? 2 : 4;
      e = hipMalloc(&t_llr, (size_t)std::max<int64_t>(llr_end, 1) * esz);
      if (e == hipSuccess) e = hipMalloc(&t_bits, (size_t)std::max<int64_t>(word_end, 1) * 4);
      if (e == hipSuccess) e = hipMalloc(&t_metric, (size_t)std::max(n_frames, 1) * 8);
      if (e == hipSuccess) e = hipMalloc(&t_end, (size_t)std::max(n_frames, 1) * 4);
      if (e == hipSuccess)
        e = launch_fill_random(t_llr, llr_end, o.dtype, 0x5eed1234u, p->origin);
      if (e != hipSuccess) throw hip_status(e);
    }
    for (int c : order) {
      Choice base;
      base.radix = o.radix == 0 ? 2 : o.radix;
      base.variant = o.variant;
      base.persistent = (o.flags & MIVIT_PLAN_PERSISTENT) != 0;
      base.split = (o.flags & MIVIT_PLAN_NO_SPLIT) == 0;
      std::vector<Choice> cand = tune ? candidates(codes[c], o.dtype, o.radix)
                                      : std::vector<Choice>{base};
      Part best;
      float best_ms = 0.0f;
      bool have = false;
      for (const Choice& ch : cand) {
        Part q;
        mivit_status s = build_part(codes, frames, by_code[c], o, o.dtype, ch, c, q);
        if (s != MIVIT_OK) throw s;
        const float ms =
            cand.size() > 1 ? time_part(p, q, t_llr, (uint32_t*)t_bits, t_metric, (int32_t*)t_end)
                            : 0.0f;
        if (cand.size() > 1 && ms < 0.0f) {
          free_part(q);
          throw MIVIT_EHIP;
        }
        if (!have || ms < best_ms) {
          if (have) free_part(best);
          best = q;
          best_ms = ms;
          have = true;
        } else {
          free_part(q);
        }
      }
      p->parts.push_back(best);
    }
    // streams and events for concurrent parts
    const int n_aux = std::min<int>(kMaxAux, (int)p->parts.size());
    if (p->parts.size() > 1) {
      e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
      for (int k = 0; k < n_aux && e == hipSuccess; ++k) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) p->aux.push_back(s);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) p->ev_join.push_back(ev);
      }
      if (e != hipSuccess) throw hip_status(e);
    }
    // gradient support: whole frames whose bits cover every stage but a zero tail
    bool grad = std::all_of(frames, frames + n_frames, [&](const mivit_frame& fr) {
      return o.chunk == 0 || fr.n_stages <= o.chunk;
    });
    std::vector<GradFrame> gf(n_frames);
    for (int f = 0; f < n_frames && grad; ++f) {
      const mivit_frame& fr = frames[f];
      const int K = codes[fr.code].K;
      const bool term = (fr.flags & MIVIT_END_ZERO) && (fr.flags & MIVIT_START_KNOWN);
      // the backward re-encodes the decoded bits from state 0: an unknown
      // start state would leave the first K-1 stages' outputs undetermined
      if (!(fr.flags & MIVIT_START_KNOWN)) grad = false;
      if (fr.out_begin != 0) grad = false;
      if (!(fr.n_out == fr.n_stages || (term && fr.n_out + K - 1 == fr.n_stages))) grad = false;
      gf[f].llr_off = fr.llr_offset;
      gf[f].bit_off = fr.bit_offset;
      gf[f].n_stages = fr.n_stages;
      gf[f].n_out = fr.n_out;
      gf[f].code = fr.code;
      gf[f].pad = 0;
      p->grad_max_stages = std::max(p->grad_max_stages, fr.n_stages);
    }
    if (grad && n_frames > 0) {
      e = upload(&p->d_gframes, gf.data(), gf.size());
      if (e != hipSuccess) throw hip_status(e);
      p->grad_ok = true;
    }
  } catch (mivit_status s) {
    status = s;
  } catch (const std::bad_alloc&) {
    status = MIVIT_ENOMEM;
  } catch (...) {
    status = MIVIT_EHIP;
  }
  if (p && p->origin) (void)hipStreamSynchronize(p->origin);
  (void)hipFree(t_llr);
  (void)hipFree(t_bits);
  (void)hipFree(t_metric);
  (void)hipFree(t_end);
  if (status != MIVIT_OK) {
    free_plan(p);
    return status;
  }
  *out = p;
  return MIVIT_OK;
}

mivit_status mivit_forward(mivit_plan* p, const void* llr, void* metric, int32_t* end_state,
                           void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (p->parts.empty()) return MIVIT_OK;
  if (!llr) return MIVIT_EINVAL;
  DeviceGuard guard(p->device);
  return hip_status(run_parts(p, kPhaseForward, llr, nullptr, metric, end_state,
                              (hipStream_t)stream));
}

mivit_status mivit_traceback(mivit_plan* p, uint32_t* bits, void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (p->parts.empty()) return MIVIT_OK;
  if (!bits) return MIVIT_EINVAL;
  DeviceGuard guard(p->device);
  return hip_status(run_parts(p, kPhaseTraceback, nullptr, bits, nullptr, nullptr,
                              (hipStream_t)stream));
}

mivit_status mivit_plan_create_on(mivit_plan** out, int32_t device, const mivit_code* codes,
                                  int32_t n_codes, const mivit_frame* frames, int32_t n_frames,
                                  const mivit_opts* opts) {
  if (!out) return MIVIT_EINVAL;
  *out = nullptr;
  if (device < 0) return mivit_plan_create(out, codes, n_codes, frames, n_frames, opts);
  clear_stale_error();
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    clear_stale_error();
    return MIVIT_EHIP;
  }
  if (device >= count) return MIVIT_EINVAL;
  // the plan is built, and records its device, with that device current;
  // the caller's current device is restored
  DeviceGuard guard(device);
  return mivit_plan_create(out, codes, n_codes, frames, n_frames, opts);
}

mivit_status mivit_decode(mivit_plan* p, const void* llr, uint32_t* bits, void* metric,
                          int32_t* end_state, void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (p->parts.empty()) return MIVIT_OK;
  if (!llr || !bits) return MIVIT_EINVAL;
  DeviceGuard guard(p->device);
  hipStream_t st = (hipStream_t)stream;
  const int both = kPhaseForward | kPhaseTraceback;
  if (!(p->flags & MIVIT_PLAN_GRAPH))
    return hip_status(run_parts(p, both, llr, bits, metric, end_state, st));
  for (const GraphEntry& g : p->graphs)
    if (g.llr == llr && g.bits == bits && g.metric == metric && g.end == end_state &&
        g.stream == st)
      return hip_status(hipGraphLaunch(g.exec, st));
  // record the launch sequence once on the plan's own stream, then replay
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(p->origin, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return MIVIT_EHIP;
  hipError_t er = run_parts(p, both, llr, bits, metric, end_state, p->origin);
  e = hipStreamEndCapture(p->origin, &graph);
  if (er != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return MIVIT_EHIP;
  }
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return MIVIT_EHIP;
  if (p->graphs.size() >= (size_t)kMaxGraphs) {
    (void)hipGraphExecDestroy(p->graphs.front().exec);
    p->graphs.erase(p->graphs.begin());
  }
  p->graphs.push_back(GraphEntry{llr, bits, metric, end_state, st, exec});
  return hip_status(hipGraphLaunch(exec, st));
}

mivit_status mivit_decode_grad(mivit_plan* p, const uint32_t* bits, const float* grad_metric,
                               float* grad_llr, void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (!p->grad_ok) return p->n_frames == 0 ? MIVIT_OK : MIVIT_EUNSUPPORTED;
  if (!bits || !grad_metric || !grad_llr) return MIVIT_EINVAL;
  DeviceGuard guard(p->device);
  hipError_t e = launch_grad(p->d_codes, p->d_gframes, p->n_frames, p->grad_max_stages, bits,
                             grad_metric, grad_llr, (hipStream_t)stream);
  return e == hipSuccess ? MIVIT_OK : MIVIT_EHIP;
}

mivit_status mivit_plan_destroy(mivit_plan* p) {
  if (!p) return MIVIT_EINVAL;
  {
    DeviceGuard guard(p->device);
    (void)hipDeviceSynchronize();
    free_plan(p);
  }
  return MIVIT_OK;
}

mivit_status mivit_plan_get_info(const mivit_plan* p, mivit_plan_info* info) {
  if (!p || !info) return MIVIT_EINVAL;
  std::memset(info, 0, sizeof *info);
  int64_t best = -1;
  for (const Part& q : p->parts) {
    info->n_items += (int64_t)q.items.size();
    info->survivor_bytes += q.surv_words * 8;
    info->total_stages += q.total_stages;
    if (q.total_stages > best) {
      best = q.total_stages;
      info->radix = q.ch.radix;
    }
  }
  if (best < 0) info->radix = 2;
  info->dtype = p->dtype;
  info->llr_elems = p->llr_end;
  info->bit_words = p->word_end;
  info->n_frames = p->n_frames;
  info->device = p->device;
  return MIVIT_OK;
}

mivit_status mivit_plan_describe(const mivit_plan* p, char* buf, int32_t len) {
  if (!p || !buf || len <= 0) return MIVIT_EINVAL;
  std::string s;
  for (const Part& q : p->parts) {
    char line[256];
    for (const PlanGroup& g : q.groups) {
      // the rotating kernels run a wave table; the others one wavefront per item
      const bool table = g.kern == kKernRot2 || g.kern == kKernRot4P || g.kern == kKernRot4Q;
      const int wpf = g.kern == kKernWide ? waves_per_frame(q.ch) : 1;
      const bool two16 = g.kern == kKernWide && q.ch.variant == 8;
      std::snprintf(line, sizeof line,
                    "%scode %d: K=%d beta=%d, %s forward, variant %d, %s, %d items, %d wavefronts",
                    s.empty() ? "" : "; ", q.code, g.K, g.beta, kern_name(g.kern), q.ch.variant,
                    g.counter >= 0 ? "persistent work queue"
                    : table        ? "one wavefront per table entry"
                    : wpf == 2     ? "two wavefronts per item"
                    : wpf == 4     ? "four wavefronts per item"
                    : two16        ? "one wavefront per item, two states per register"
                                   : "one wavefront per item",
                    g.count, table ? g.n_waves : wpf * g.count);
      s += line;
    }
  }
  std::snprintf(buf, (size_t)len, "%s", s.c_str());
  return MIVIT_OK;
}

mivit_status mivit_quantize_i8(const float* llr, int8_t* q, int64_t n, float scale,
                               void* stream) {
  if (n < 0 || (n > 0 && (!llr || !q))) return MIVIT_EINVAL;
  if (!(scale > 0.0f) || scale > 3.0e38f) return MIVIT_EINVAL;
  clear_stale_error();
  hipError_t e = launch_quant(llr, q, n, scale, (hipStream_t)stream);
  return e == hipSuccess ? MIVIT_OK : MIVIT_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// One-call decode of equal-length frames.  Plans are kept per (device,
// stream, code, dtype, shape): a plan owns its survivor memory, so calls on
// one stream reuse it in stream order and calls on different streams never
// share one.  The least recently used plan is released (after its stream
// has drained) when more than kUniformPlans are held.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kUniformPlans = 16;

struct UniformEntry {
  int device;
  void* stream;
  mivit_code code;
  int32_t dtype, n_frames, n_info, terminated;
  mivit_plan* plan;
  uint64_t last_use;
};

struct UniformCache {
  std::mutex mu;
  std::vector<UniformEntry> entries;
  uint64_t clock = 0;
};

UniformCache& uniform_cache() {
  static UniformCache* c = new UniformCache();  // never destroyed: HIP may be gone at exit
  return *c;
}

// Radix of the one-call entry points: the packed radix-4 kernel where it
// applies (int8, K = 5 or 7, beta = 2), radix 2 otherwise.
int uniform_radix(const mivit_code& code, int dtype) {
  return (dtype == MIVIT_I8 && packed_ok(code)) ? 4 : 2;
}

bool same_code(const mivit_code& a, const mivit_code& b) {
  if (a.K != b.K || a.beta != b.beta) return false;
  for (int k = 0; k < a.beta; ++k)
    if (a.gen[k] != b.gen[k]) return false;
  return true;
}

}  // namespace

extern "C" {

mivit_status mivit_decode_uniform(const void* llr, int32_t dtype, const mivit_code* code,
                                  int32_t n_frames, int32_t n_info, int32_t terminated,
                                  uint32_t* bits, void* metric, void* stream) {
  if (!code || n_frames < 0 || n_info < 0) return MIVIT_EINVAL;
  if (dtype != MIVIT_F32 && dtype != MIVIT_I8 && dtype != MIVIT_F16) return MIVIT_EINVAL;
  if (terminated != 0 && terminated != 1) return MIVIT_EINVAL;
  mivit_status cs = check_code(*code);
  if (cs != MIVIT_OK) return cs;
  const int64_t S = (int64_t)n_info + (terminated ? code->K - 1 : 0);
  const int64_t W = ((int64_t)n_info + 31) / 32;
  if (S > INT32_MAX || (int64_t)n_frames * W * 32 > ((int64_t)1 << 62)) return MIVIT_EINVAL;
  if (n_frames == 0 || S == 0) return MIVIT_OK;
  if (!llr || !bits) return MIVIT_EINVAL;
  int dev = 0;
  clear_stale_error();
  if (hipGetDevice(&dev) != hipSuccess) return MIVIT_EHIP;
  UniformCache& cache = uniform_cache();
  std::lock_guard<std::mutex> lock(cache.mu);
  mivit_plan* plan = nullptr;
  for (UniformEntry& e : cache.entries)
    if (e.device == dev && e.stream == stream && e.dtype == dtype && e.n_frames == n_frames &&
        e.n_info == n_info && e.terminated == terminated && same_code(e.code, *code)) {
      e.last_use = ++cache.clock;
      plan = e.plan;
      break;
    }
  if (!plan) {
    std::vector<mivit_frame> fr;
    try {
      fr.resize((size_t)n_frames);
    } catch (const std::bad_alloc&) {
      return MIVIT_ENOMEM;
    }
    for (int32_t f = 0; f < n_frames; ++f) {
      mivit_frame& x = fr[(size_t)f];
      x.llr_offset = (int64_t)f * S * code->beta;
      x.bit_offset = (int64_t)f * W * 32;
      x.n_stages = (int32_t)S;
      x.out_begin = 0;
      x.n_out = n_info;
      x.code = 0;
      x.flags = (uint16_t)(MIVIT_START_KNOWN | (terminated ? MIVIT_END_ZERO : 0));
    }
    mivit_opts o;
    std::memset(&o, 0, sizeof o);
    o.dtype = dtype;
    o.radix = uniform_radix(*code, dtype);
    mivit_status s = mivit_plan_create(&plan, code, 1, fr.data(), n_frames, &o);
    if (s != MIVIT_OK) return s;
    if (cache.entries.size() >= kUniformPlans) {
      auto old = std::min_element(cache.entries.begin(), cache.entries.end(),
                                  [](const UniformEntry& a, const UniformEntry& b) {
                                    return a.last_use < b.last_use;
                                  });
      {
        DeviceGuard guard(old->device);
        (void)hipStreamSynchronize((hipStream_t)old->stream);
        free_plan(old->plan);
      }
      cache.entries.erase(old);
    }
    UniformEntry e;
    e.device = dev;
    e.stream = stream;
    e.code = *code;
    e.dtype = dtype;
    e.n_frames = n_frames;
    e.n_info = n_info;
    e.terminated = terminated;
    e.plan = plan;
    e.last_use = ++cache.clock;
    cache.entries.push_back(e);
  }
  return mivit_decode(plan, llr, bits, metric, nullptr, stream);
}

}  // extern "C"
