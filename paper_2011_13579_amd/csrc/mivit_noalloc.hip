// One-call decode of equal-length frames that allocates no device memory:
// every table and the survivor memory of the call live in one fixed,
// file-scope device array of kScratchBytes, which each GPU the library runs
// on holds until the process ends.  Host code never names the array's
// symbol directly: at the first call on a device (that device current) its
// device address is read once with hipGetSymbolAddress and kept per device;
// every kernel receives that address.
//
// The batch's tables (code, work items, wavefront and frame-pair tables) are
// written into the array by a small kernel from the batch shape, so the call
// copies nothing from the host either: a table kernel, the forward kernel
// and the traceback kernel are all it launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <mutex>

#include "../../include/mivit.h"
#include "mivit_device.h"

namespace mivit {
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
hipError_t launch_tb_r4p(int K, const Item* items, const int2* pairs, int n_pairs,
                         const uint64_t* surv, const int32_t* item_end, uint32_t* bits, int warm,
                         hipStream_t st);
}  // namespace mivit

using namespace mivit;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

// kernel families of the one-call path (the choices mivit_decode_uniform's
// plans make for a uniform batch with default options)
enum : int { kFamRot2 = 0, kFamR4P = 1, kFamWide = 2 };
// survivor layouts of the segmented traceback (as the plan code numbers them)
constexpr int kLayoutRotR2 = 2, kLayoutRotByte = 4;
constexpr int kWarm = 64, kWarmR4P = 96;  // traceback warm-up stages, as in plans
constexpr int kRotModeDefault = 2;        // rotating kernel, exchanges in the VALU

struct Layout {
  int fam;
  int fpw;             // frames per wavefront entry (table-driven kernels)
  int n_waves, n_pairs;
  int64_t ws;          // survivor words per item (per frame pair for radix 4)
  size_t off_items, off_waves, off_pairs, off_end, off_surv, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool make_layout(const mivit_code& c, int dtype, int F, int S, Layout& L) {
  const bool packed = dtype == MIVIT_I8 && c.beta == 2 && (c.K == 5 || c.K == 7);
  L.fam = packed ? kFamR4P : (c.K <= 7 ? kFamRot2 : kFamWide);
  L.fpw = L.fam == kFamR4P ? 2 * (64 >> (c.K - 1)) : L.fam == kFamRot2 ? (64 >> (c.K - 1)) : 1;
  L.n_waves = (F + L.fpw - 1) / L.fpw;  // the wide kernel: one unit per frame (fpw 1)
  L.n_pairs = L.fam == kFamR4P ? (F + 1) / 2 : 0;
  L.ws = L.fam == kFamR4P ? surv_words_r4p(c.K, S) : surv_words_blocks32(c.K, S);
  const int64_t units = L.fam == kFamR4P ? (F + 1) / 2 : F;
  size_t o = align256(sizeof(DevCode));
  L.off_items = o;
  o = align256(o + (size_t)F * sizeof(Item));
  L.off_waves = o;  // radix 2: (first, count) per entry; else one whole-frame unit per entry
  o = align256(o + (size_t)L.n_waves * (L.fam == kFamRot2 ? sizeof(int2) : sizeof(SplitUnit)));
  L.off_pairs = o;
  o = align256(o + (size_t)L.n_pairs * sizeof(int2));
  L.off_end = o;
  o = align256(o + (size_t)F * sizeof(int32_t));
  L.off_surv = o;
  const double surv_bytes = ((double)units * (double)L.ws + (double)kSurvSlackWords) * 8.0;
  if ((double)o + surv_bytes > (double)kScratchBytes) return false;
  L.total = o + (size_t)(units * L.ws + kSurvSlackWords) * 8;
  return true;
}

// The tables of a uniform batch, as a plan builds them: items in frame
// order (equal lengths keep the longest-first order stable), wavefront
// entries of fpw consecutive frames, frame pairs (2p, 2p+1).
__global__ void k_uniform_tables(uint8_t* base, DevCode code, int F, int S, int n_info,
                                 int terminated, int fam, int fpw, int n_waves, int n_pairs,
                                 int64_t ws, size_t off_items, size_t off_waves,
                                 size_t off_pairs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *(DevCode*)base = code;
  if (k < F) {
    Item it;
    it.llr_off = (int64_t)k * S * code.beta;
    it.surv_off = (fam == kFamR4P ? (int64_t)(k >> 1) : (int64_t)k) * ws;
    it.bit_off = (int64_t)k * ((n_info + 31) / 32) * 32;
    it.n_stages = S;
    it.out_begin = 0;
    it.n_out = n_info;
    it.code = 0;
    it.start_known = 1;
    it.end_state = terminated ? 0 : -1;
    it.frame = k;
    it.slot = k;
    ((Item*)(base + off_items))[k] = it;
  }
  if (k < n_waves) {
    const int first = k * fpw;
    const int count = F - first < fpw ? F - first : fpw;
    if (fam != kFamRot2) {
      SplitUnit u;
      u.first = first;
      u.count = count;
      u.it_begin = 0;
      u.it_end = fam == kFamR4P ? S >> 1 : S;  // iterations (radix 4) or stages
      u.warm = 0;
      u.part = 0;
      u.n_parts = 1;
      u.bnd = -1;
      ((SplitUnit*)(base + off_waves))[k] = u;
    } else {
      ((int2*)(base + off_waves))[k] = make_int2(first, count);
    }
  }
  if (k < n_pairs) ((int2*)(base + off_pairs))[k] = make_int2(2 * k, F - 2 * k < 2 ? 1 : 2);
}

std::mutex g_mu;
void* g_ptr[kMaxDevices];

// Device address of this device's scratch array (read once per device).
hipError_t scratch_ptr(int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_ptr[dev] = ptr;
  }
  *out = (uint8_t*)g_ptr[dev];
  return hipSuccess;
}

mivit_status status_of(hipError_t e) { return e == hipSuccess ? MIVIT_OK : MIVIT_EHIP; }

}  // namespace

extern "C" mivit_status mivit_decode_uniform_noalloc(const void* llr, int32_t dtype,
                                                      const mivit_code* code, int32_t n_frames,
                                                      int32_t n_info, int32_t terminated,
                                                      uint32_t* bits, void* metric,
                                                      void* stream) {
  if (!code || n_frames < 0 || n_info < 0) return MIVIT_EINVAL;
  if (dtype != MIVIT_F32 && dtype != MIVIT_I8 && dtype != MIVIT_F16) return MIVIT_EINVAL;
  if (terminated != 0 && terminated != 1) return MIVIT_EINVAL;
  const mivit_code& c = *code;
  if (c.K < 3 || c.K > kMaxK || c.beta < 2 || c.beta > 4) return MIVIT_EINVAL;
  for (int b = 0; b < c.beta; ++b) {
    if (c.gen[b] == 0 || c.gen[b] >= (1u << c.K)) return MIVIT_EINVAL;
    if (!((c.gen[b] >> (c.K - 1)) & 1u) || !(c.gen[b] & 1u)) return MIVIT_EUNSUPPORTED;
  }
  const int64_t S64 = (int64_t)n_info + (terminated ? c.K - 1 : 0);
  if (S64 > INT32_MAX) return MIVIT_EINVAL;
  const int S = (int)S64;
  if (n_frames == 0 || S == 0) return MIVIT_OK;
  if (!llr || !bits) return MIVIT_EINVAL;
  Layout L;
  if (!make_layout(c, dtype, n_frames, S, L)) return MIVIT_ENOMEM;  // exceeds the fixed scratch
  (void)hipGetLastError();  // launches report through it: clear an unrelated earlier error
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MIVIT_EHIP;
  uint8_t* base = nullptr;
  hipError_t e = scratch_ptr(dev, &base);
  if (e != hipSuccess) return MIVIT_EHIP;
  hipStream_t st = (hipStream_t)stream;
  DevCode dc;
  std::memset(&dc, 0, sizeof dc);
  dc.K = c.K;
  dc.beta = c.beta;
  for (int b = 0; b < c.beta; ++b) dc.gen[b] = c.gen[b];
  const int nt = n_frames > L.n_waves ? n_frames : L.n_waves;
  hipLaunchKernelGGL(k_uniform_tables, dim3((nt + 255) / 256), dim3(256), 0, st, base, dc,
                     n_frames, S, n_info, terminated, L.fam, L.fpw, L.n_waves, L.n_pairs, L.ws,
                     L.off_items, L.off_waves, L.off_pairs);
  e = hipGetLastError();
  if (e != hipSuccess) return status_of(e);
  const DevCode* d_code = (const DevCode*)base;
  const Item* items = (const Item*)(base + L.off_items);
  const int2* waves = (const int2*)(base + L.off_waves);
  const int2* pairs = (const int2*)(base + L.off_pairs);
  int32_t* item_end = (int32_t*)(base + L.off_end);
  uint64_t* surv = (uint64_t*)(base + L.off_surv);
  if (L.fam == kFamR4P) {
    e = launch_fwd_r4p(c.K, d_code, items, (const SplitUnit*)waves, L.n_waves, (const int8_t*)llr,
                       surv, (int64_t*)metric, nullptr, item_end, nullptr, 0, nullptr, nullptr,
                       nullptr, 0, nullptr, st);
    if (e == hipSuccess)
      e = launch_tb_r4p(c.K, items, pairs, L.n_pairs, surv, item_end, bits, kWarmR4P, st);
  } else if (L.fam == kFamRot2) {
    e = launch_fwd_rot(c.K, c.beta, dtype, kRotModeDefault, d_code, items, waves, L.n_waves, llr,
                       surv, metric, nullptr, item_end, nullptr, 0, st);
    if (e == hipSuccess)
      e = launch_tb_seg(kLayoutRotR2, d_code, items, n_frames, surv, item_end, bits, kWarm, st);
  } else {
    e = launch_fwd_wide(c.K, c.beta, dtype, 1, false, d_code, items, (const SplitUnit*)waves, n_frames, llr,
                        surv, metric, nullptr, item_end, nullptr, nullptr, nullptr, 0, nullptr,
                        nullptr, nullptr, st);
    if (e == hipSuccess)
      e = launch_tb_seg(kLayoutRotByte, d_code, items, n_frames, surv, item_end, bits, kWarm, st);
  }
  return status_of(e);
}
