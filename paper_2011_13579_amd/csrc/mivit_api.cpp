// C ABI of the Viterbi decoder library: argument validation, plan building
// (chunking of long frames into overlapping windows, §III), work ordering,
// device memory ownership and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mivit.h"
#include "mivit_device.h"

namespace mivit {
hipError_t launch_fwd(int radix, int nsl, bool is_int, const DevCode* codes, const Item* items,
                      int n_items, const void* llr, uint64_t* surv, void* metric,
                      int32_t* end_out, int32_t* item_end, hipStream_t st);
hipError_t launch_tb(int radix, const DevCode* codes, const Item* items, int n_items,
                     const uint64_t* surv, const int32_t* item_end, uint32_t* bits,
                     hipStream_t st);
hipError_t launch_grad(const DevCode* codes, const GradFrame* frames, int n_frames,
                       int max_stages, const uint32_t* bits, const float* gm, float* grad,
                       hipStream_t st);
hipError_t launch_quant(const float* x, int8_t* q, int64_t n, float scale, hipStream_t st);
hipError_t launch_fwd_rot(int K, int beta, bool is_int, int mode, const DevCode* codes,
                          const Item* items, const int2* waves, int n_waves, const void* llr,
                          uint64_t* surv, void* metric, int32_t* end_out, int32_t* item_end,
                          hipStream_t st);
hipError_t launch_tb_seg(int layout, const DevCode* codes, const Item* items, int n_items,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits,
                         int warm, hipStream_t st);
hipError_t launch_fwd_r4p(int K, const DevCode* codes, const Item* items, const int2* waves,
                          int n_waves, const int8_t* llr, uint64_t* surv, int64_t* metric,
                          int32_t* end_out, int32_t* item_end, hipStream_t st);
hipError_t launch_tb_r4p(int K, const Item* items, const int2* pairs, int n_pairs,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits, int warm,
                         hipStream_t st);
}  // namespace mivit

using namespace mivit;

// forward kernels and the survivor layouts they write
enum : int { kKernGeneric2 = 0, kKernGeneric4 = 1, kKernRot2 = 2, kKernRot4P = 3 };
enum : int { kLayoutNatR2 = 0, kLayoutNatR4 = 1, kLayoutRotR2 = 2, kLayoutRot4P = 3 };
constexpr int kWarmStages = 64;  // speculative traceback warm-up
// rotating forward kernel exchange scheme per plan variant:
// 0 all exchanges in the VALU (DPP, permlane swaps), 1 both previous-state
// metrics via DPP/LDS swizzles, 2 one partner metric via DPP/LDS swizzles
constexpr int kRotMode[3] = {2, 0, 1};

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
};

struct mivit_plan {
  int device = 0;
  int dtype = MIVIT_F32;
  int radix = 2;
  int variant = 0;  // kernel variant (0: default)
  int n_frames = 0;
  bool grad_ok = false;
  int grad_max_stages = 0;
  int64_t total_stages = 0;
  int64_t surv_words = 0;
  std::vector<Item> items;
  std::vector<PlanGroup> groups;
  std::vector<int> group_keys;
  DevCode* d_codes = nullptr;
  Item* d_items = nullptr;
  int32_t* d_item_end = nullptr;
  uint64_t* d_surv = nullptr;
  GradFrame* d_gframes = nullptr;
  int2* d_waves = nullptr;  // rotating kernels: (first item, count) per wavefront
  int2* d_pairs = nullptr;  // packed radix-4 traceback: (first item, count) per frame pair
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
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

void free_plan(mivit_plan* p) {
  if (!p) return;
  (void)hipFree(p->d_codes);
  (void)hipFree(p->d_items);
  (void)hipFree(p->d_item_end);
  (void)hipFree(p->d_surv);
  (void)hipFree(p->d_gframes);
  (void)hipFree(p->d_waves);
  (void)hipFree(p->d_pairs);
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

const char* mivit_version(void) { return "mivit 0.1 (gfx950)"; }

mivit_status mivit_plan_create(mivit_plan** out, const mivit_code* codes, int32_t n_codes,
                               const mivit_frame* frames, int32_t n_frames,
                               const mivit_opts* opts) {
  if (!out) return MIVIT_EINVAL;
  *out = nullptr;
  if (!codes || n_codes <= 0 || n_codes > 32767 || n_frames < 0 || (n_frames > 0 && !frames))
    return MIVIT_EINVAL;
  mivit_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  if (o.dtype != MIVIT_F32 && o.dtype != MIVIT_I8) return MIVIT_EINVAL;
  if (o.radix != 0 && o.radix != 2 && o.radix != 4) return MIVIT_EINVAL;
  if (o.radix == 4 && o.dtype != MIVIT_I8) return MIVIT_EINVAL;
  if (o.chunk < 0 || o.overlap < 0 || (o.chunk > 0 && o.chunk % 32 != 0)) return MIVIT_EINVAL;
  if (o.variant < 0 || o.variant > 2) return MIVIT_EINVAL;
  for (int c = 0; c < n_codes; ++c) {
    mivit_status s = check_code(codes[c]);
    if (s != MIVIT_OK) return s;
  }
  // frames: ranges and non-overlapping outputs
  std::vector<std::pair<int64_t, int64_t>> words;
  words.reserve(n_frames);
  for (int f = 0; f < n_frames; ++f) {
    const mivit_frame& fr = frames[f];
    if (fr.code < 0 || fr.code >= n_codes) return MIVIT_EINVAL;
    if (fr.n_stages < 0 || fr.out_begin < 0 || fr.n_out < 0) return MIVIT_EINVAL;
    if ((int64_t)fr.out_begin + fr.n_out > fr.n_stages) return MIVIT_EINVAL;
    if (fr.llr_offset < 0 || fr.bit_offset < 0 || (fr.bit_offset & 31)) return MIVIT_EINVAL;
    if (fr.flags & ~(MIVIT_START_KNOWN | MIVIT_END_ZERO)) return MIVIT_EINVAL;
    if (o.chunk > 0 && fr.n_stages > o.chunk && fr.out_begin != 0) return MIVIT_EUNSUPPORTED;
    if (fr.n_out > 0) words.push_back({fr.bit_offset >> 5, (fr.bit_offset + fr.n_out + 31) >> 5});
  }
  std::sort(words.begin(), words.end());
  for (size_t k = 1; k < words.size(); ++k)
    if (words[k].first < words[k - 1].second) return MIVIT_EINVAL;

  mivit_plan* p = nullptr;
  try {
    p = new mivit_plan();
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return MIVIT_EHIP;
    }
    p->dtype = o.dtype;
    p->radix = o.radix == 0 ? 2 : o.radix;
    p->variant = o.variant;
    p->n_frames = n_frames;
    // expand frames into work items
    std::vector<Item> items;
    bool chunked_any = false;
    bool tail_ok = true;
    for (int f = 0; f < n_frames; ++f) {
      const mivit_frame& fr = frames[f];
      const mivit_code& c = codes[fr.code];
      const int S = fr.n_stages;
      if (fr.out_begin != 0) tail_ok = false;
      if (o.chunk > 0 && S > o.chunk) {
        chunked_any = true;
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
    // choose the forward kernel of every item and group them
    const int radix = p->radix;
    auto kern_of = [&](const Item& it) {
      const mivit_code& c = codes[it.code];
      if (radix == 4)
        return (o.variant == 0 && c.beta == 2 && (c.K == 5 || c.K == 7)) ? (int)kKernRot4P
                                                                          : (int)kKernGeneric4;
      if (c.K <= 7) return (int)kKernRot2;
      return (int)kKernGeneric2;
    };
    auto key_of = [&](const Item& it) {
      const mivit_code& c = codes[it.code];
      const int kern = kern_of(it);
      // generic kernels group by states per lane; the rotating ones by (K, beta)
      return (kern == kKernRot2 || kern == kKernRot4P) ? (kern << 16) | (c.K << 8) | c.beta
                                                       : (kern << 16) | nsl_of(c.K);
    };
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
      const int ka = key_of(a), kb = key_of(b);
      if (ka != kb) return ka > kb;
      if (a.n_stages != b.n_stages) return a.n_stages > b.n_stages;
      if (a.out_begin != b.out_begin) return a.out_begin < b.out_begin;
      return a.n_out < b.n_out;
    });
    for (size_t k = 0; k < items.size(); ++k) {
      Item& it = items[k];
      const mivit_code& c = codes[it.code];
      const int kern = kern_of(it);
      it.slot = (int32_t)k;
      p->total_stages += it.n_stages;
      const int key = key_of(it);
      if (p->groups.empty() || p->group_keys.back() != key) {
        PlanGroup g;
        g.kern = kern;
        g.layout = kern == kKernRot2    ? kLayoutRotR2
                   : kern == kKernRot4P ? kLayoutRot4P
                   : kern == kKernGeneric4 ? kLayoutNatR4
                                           : kLayoutNatR2;
        g.nsl = nsl_of(c.K);
        g.K = c.K;
        g.beta = c.beta;
        g.first = (int)k;
        g.count = 0;
        g.pair_off = 0;
        g.n_pairs = 0;
        p->groups.push_back(g);
        p->group_keys.push_back(key);
      }
      p->groups.back().count++;
    }
    // rotating kernels: wavefronts of frames of equal length (radix 2: up to
    // 64/2^(K-1) frames; packed radix 4: up to 2*64/2^(K-1), where the two
    // frames of a lane group must also emit the same stages)
    std::vector<int2> waves, pairs;
    std::vector<char> pair_hi(items.size(), 0);
    for (PlanGroup& g : p->groups) {
      g.wave_off = (int)waves.size();
      g.n_waves = 0;
      if (g.kern != kKernRot2 && g.kern != kKernRot4P) continue;
      const bool packed = g.kern == kKernRot4P;
      const int fpw = (packed ? 2 : 1) * (64 >> (g.K - 1));
      for (int k = g.first; k < g.first + g.count; ++k) {
        if (g.n_waves > 0) {
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
        g.n_waves++;
      }
      if (packed) {
        g.pair_off = (int)pairs.size();
        for (int w = g.wave_off; w < g.wave_off + g.n_waves; ++w)
          for (int s = 0; s < waves[w].y; s += 2)
            pairs.push_back(make_int2(waves[w].x + s, std::min(2, waves[w].y - s)));
        g.n_pairs = (int)pairs.size() - g.pair_off;
      }
    }
    // survivor memory, 16-byte aligned per item (per frame pair when packed)
    int64_t words_total = 0;
    for (size_t k = 0; k < items.size(); ++k) {
      Item& it = items[k];
      const mivit_code& c = codes[it.code];
      const int kern = kern_of(it);
      if (kern == kKernRot4P && pair_hi[k]) {
        it.surv_off = items[k - 1].surv_off;
        continue;
      }
      it.surv_off = words_total;
      int64_t words;
      if (kern == kKernRot2)
        words = (int64_t)((it.n_stages + 31) / 32) * (1 << (c.K - 1)) / 2;
      else if (kern == kKernRot4P)  // 2^(K-1) 32-bit words per 8 iterations
        words = (int64_t)((it.n_stages / 2 + 7) / 8) * (1 << (c.K - 1)) / 2;
      else
        words = (int64_t)it.n_stages * words_per_stage(c.K);
      words_total += (words + 1) & ~(int64_t)1;
    }
    words_total += 32;  // the traceback reads whole blocks past an item's end
    p->surv_words = words_total;
    p->items = items;

    std::vector<DevCode> dc(n_codes);
    for (int c = 0; c < n_codes; ++c) {
      dc[c].K = codes[c].K;
      dc[c].beta = codes[c].beta;
      for (int b = 0; b < 4; ++b) dc[c].gen[b] = b < codes[c].beta ? codes[c].gen[b] : 0;
    }
    hipError_t e = upload(&p->d_codes, dc.data(), dc.size());
    if (e == hipSuccess) e = upload(&p->d_waves, waves.data(), waves.size());
    if (e == hipSuccess) e = upload(&p->d_pairs, pairs.data(), pairs.size());
    if (e == hipSuccess) e = upload(&p->d_items, items.data(), items.size());
    if (e == hipSuccess && !items.empty())
      e = hipMalloc((void**)&p->d_item_end, items.size() * sizeof(int32_t));
    if (e == hipSuccess && words_total > 0)
      e = hipMalloc((void**)&p->d_surv, (size_t)words_total * sizeof(uint64_t));
    // gradient support: whole frames whose bits cover every stage but a zero tail
    if (e == hipSuccess && !chunked_any && tail_ok) {
      std::vector<GradFrame> gf(n_frames);
      bool ok = true;
      for (int f = 0; f < n_frames && ok; ++f) {
        const mivit_frame& fr = frames[f];
        const int K = codes[fr.code].K;
        const bool term = (fr.flags & MIVIT_END_ZERO) && (fr.flags & MIVIT_START_KNOWN);
        if (!(fr.n_out == fr.n_stages || (term && fr.n_out + K - 1 == fr.n_stages))) ok = false;
        gf[f].llr_off = fr.llr_offset;
        gf[f].bit_off = fr.bit_offset;
        gf[f].n_stages = fr.n_stages;
        gf[f].n_out = fr.n_out;
        gf[f].code = fr.code;
        gf[f].pad = 0;
        p->grad_max_stages = std::max(p->grad_max_stages, fr.n_stages);
      }
      if (ok) {
        e = upload(&p->d_gframes, gf.data(), gf.size());
        p->grad_ok = (e == hipSuccess);
      }
    }
    if (e != hipSuccess) {
      mivit_status s = (e == hipErrorOutOfMemory) ? MIVIT_ENOMEM : MIVIT_EHIP;
      free_plan(p);
      return s;
    }
  } catch (const std::bad_alloc&) {
    free_plan(p);
    return MIVIT_ENOMEM;
  } catch (...) {
    free_plan(p);
    return MIVIT_EHIP;
  }
  *out = p;
  return MIVIT_OK;
}

mivit_status mivit_forward(mivit_plan* p, const void* llr, void* metric, int32_t* end_state,
                           void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (p->items.empty()) return MIVIT_OK;
  if (!llr) return MIVIT_EINVAL;
  DeviceGuard guard(p->device);
  hipStream_t st = (hipStream_t)stream;
  const bool is_int = p->dtype == MIVIT_I8;
  for (const PlanGroup& g : p->groups) {
    hipError_t e;
    if (g.kern == kKernRot4P)
      e = launch_fwd_r4p(g.K, p->d_codes, p->d_items, p->d_waves + g.wave_off, g.n_waves,
                         (const int8_t*)llr, p->d_surv, (int64_t*)metric, end_state,
                         p->d_item_end, st);
    else if (g.kern == kKernRot2)
      e = launch_fwd_rot(g.K, g.beta, is_int, kRotMode[p->variant], p->d_codes, p->d_items,
                         p->d_waves + g.wave_off,
                         g.n_waves, llr, p->d_surv, metric, end_state, p->d_item_end, st);
    else
      e = launch_fwd(g.kern == kKernGeneric4 ? 4 : 2, g.nsl, is_int, p->d_codes,
                     p->d_items + g.first, g.count, llr, p->d_surv, metric, end_state,
                     p->d_item_end, st);
    if (e != hipSuccess) return MIVIT_EHIP;
  }
  return MIVIT_OK;
}

mivit_status mivit_traceback(mivit_plan* p, uint32_t* bits, void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (p->items.empty()) return MIVIT_OK;
  if (!bits) return MIVIT_EINVAL;
  DeviceGuard guard(p->device);
  for (const PlanGroup& g : p->groups) {
    hipError_t e =
        g.kern == kKernRot4P
            ? launch_tb_r4p(g.K, p->d_items, p->d_pairs + g.pair_off, g.n_pairs, p->d_surv,
                            p->d_item_end, bits, kWarmStages, (hipStream_t)stream)
            : launch_tb_seg(g.layout, p->d_codes, p->d_items + g.first, g.count, p->d_surv,
                            p->d_item_end, bits, kWarmStages, (hipStream_t)stream);
    if (e != hipSuccess) return MIVIT_EHIP;
  }
  return MIVIT_OK;
}

mivit_status mivit_decode(mivit_plan* p, const void* llr, uint32_t* bits, void* metric,
                          int32_t* end_state, void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (p->items.empty()) return MIVIT_OK;
  if (!llr || !bits) return MIVIT_EINVAL;
  mivit_status s = mivit_forward(p, llr, metric, end_state, stream);
  if (s != MIVIT_OK) return s;
  return mivit_traceback(p, bits, stream);
}

mivit_status mivit_decode_grad(mivit_plan* p, const uint32_t* bits, const float* grad_metric,
                               float* grad_llr, void* stream) {
  if (!p) return MIVIT_EINVAL;
  if (!p->grad_ok) return MIVIT_EUNSUPPORTED;
  if (p->n_frames == 0) return MIVIT_OK;
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
  }
  free_plan(p);
  return MIVIT_OK;
}

mivit_status mivit_plan_get_info(const mivit_plan* p, mivit_plan_info* info) {
  if (!p || !info) return MIVIT_EINVAL;
  info->n_items = (int64_t)p->items.size();
  info->survivor_bytes = p->surv_words * 8;
  info->total_stages = p->total_stages;
  info->radix = p->radix;
  info->dtype = p->dtype;
  return MIVIT_OK;
}

mivit_status mivit_quantize_i8(const float* llr, int8_t* q, int64_t n, float scale,
                               void* stream) {
  if (n < 0 || (n > 0 && (!llr || !q))) return MIVIT_EINVAL;
  if (!(scale > 0.0f) || scale > 3.0e38f) return MIVIT_EINVAL;
  hipError_t e = launch_quant(llr, q, n, scale, (hipStream_t)stream);
  return e == hipSuccess ? MIVIT_OK : MIVIT_EHIP;
}

}  // extern "C"
