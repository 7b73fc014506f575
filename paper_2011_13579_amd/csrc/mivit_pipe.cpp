// Host pipeline over the C ABI: batches of soft values in host memory are
// copied to the device, decoded and their bits (and metrics) copied back,
// with the copy-in of one batch, the decode of another and the copy-out of
// a third in flight at once on three streams.  Uses only the public plan
// API (mivit_decode, mivit_plan_get_info).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "../../include/mivit.h"

struct mivit_pipe {
  mivit_plan* plan = nullptr;
  int device = 0;
  int depth = 0;
  size_t llr_bytes = 0, bits_bytes = 0, metric_bytes = 0;
  hipStream_t s_in = nullptr, s_dec = nullptr, s_out = nullptr;
  std::vector<void*> d_llr, d_bits, d_metric;
  std::vector<hipEvent_t> ev_in, ev_dec, ev_out;
};

namespace {

void release(mivit_pipe* p) {
  for (void* b : p->d_llr) (void)hipFree(b);
  for (void* b : p->d_bits) (void)hipFree(b);
  for (void* b : p->d_metric) (void)hipFree(b);
  for (auto* v : {&p->ev_in, &p->ev_dec, &p->ev_out})
    for (hipEvent_t e : *v) (void)hipEventDestroy(e);
  for (hipStream_t s : {p->s_in, p->s_dec, p->s_out})
    if (s) (void)hipStreamDestroy(s);
  delete p;
}

struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" {

mivit_status mivit_pipe_create(mivit_pipe** out, mivit_plan* plan, int32_t depth) {
  if (!out || !plan || depth < 2 || depth > 8) return MIVIT_EINVAL;
  *out = nullptr;
  mivit_plan_info info;
  mivit_status st = mivit_plan_get_info(plan, &info);
  if (st != MIVIT_OK) return st;
  mivit_pipe* p = new (std::nothrow) mivit_pipe();
  if (!p) return MIVIT_ENOMEM;
  p->plan = plan;
  p->device = info.device;
  p->depth = depth;
  const size_t esz = info.dtype == MIVIT_I8 ? 1 : info.dtype == MIVIT_F16 ? 2 : 4;
  p->llr_bytes = (size_t)info.llr_elems * esz;
  p->bits_bytes = (size_t)info.bit_words * 4;
  p->metric_bytes = (size_t)info.n_frames * (info.dtype == MIVIT_I8 ? 8 : 4);
  DeviceScope scope(p->device);
  hipError_t e = hipSuccess;
  for (hipStream_t* s : {&p->s_in, &p->s_dec, &p->s_out})
    if (e == hipSuccess) e = hipStreamCreateWithFlags(s, hipStreamNonBlocking);
  for (int k = 0; k < depth && e == hipSuccess; ++k) {
    void *a = nullptr, *b = nullptr, *m = nullptr;
    e = hipMalloc(&a, p->llr_bytes > 0 ? p->llr_bytes : 1);
    if (e == hipSuccess) p->d_llr.push_back(a);
    if (e == hipSuccess) e = hipMalloc(&b, p->bits_bytes > 0 ? p->bits_bytes : 4);
    if (e == hipSuccess) p->d_bits.push_back(b);
    if (e == hipSuccess) e = hipMalloc(&m, p->metric_bytes > 0 ? p->metric_bytes : 8);
    if (e == hipSuccess) p->d_metric.push_back(m);
    for (auto* v : {&p->ev_in, &p->ev_dec, &p->ev_out}) {
      hipEvent_t ev = nullptr;
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) v->push_back(ev);
    }
  }
  if (e != hipSuccess) {
    release(p);
    return e == hipErrorOutOfMemory ? MIVIT_ENOMEM : MIVIT_EHIP;
  }
  *out = p;
  return MIVIT_OK;
}

mivit_status mivit_pipe_run(mivit_pipe* p, const void* host_llr, uint32_t* host_bits,
                            void* host_metric, int64_t n_batches) {
  if (!p || n_batches < 0) return MIVIT_EINVAL;
  if (n_batches == 0) return MIVIT_OK;
  if (!host_llr || !host_bits) return MIVIT_EINVAL;
  DeviceScope scope(p->device);
  const char* in = (const char*)host_llr;
  char* bits = (char*)host_bits;
  char* met = (char*)host_metric;
  hipError_t e = hipSuccess;
  mivit_status st = MIVIT_OK;
  for (int64_t b = 0; b < n_batches && e == hipSuccess && st == MIVIT_OK; ++b) {
    const int k = (int)(b % p->depth);
    const bool reuse = b >= p->depth;
    // copy in once the slot's previous decode has read its soft values
    if (reuse) e = hipStreamWaitEvent(p->s_in, p->ev_dec[k], 0);
    if (e == hipSuccess && p->llr_bytes)
      e = hipMemcpyAsync(p->d_llr[k], in + (size_t)b * p->llr_bytes, p->llr_bytes,
                         hipMemcpyHostToDevice, p->s_in);
    if (e == hipSuccess) e = hipEventRecord(p->ev_in[k], p->s_in);
    // decode once the soft values are in and the slot's last bits are out
    if (e == hipSuccess) e = hipStreamWaitEvent(p->s_dec, p->ev_in[k], 0);
    if (e == hipSuccess && reuse) e = hipStreamWaitEvent(p->s_dec, p->ev_out[k], 0);
    if (e == hipSuccess)
      st = mivit_decode(p->plan, p->d_llr[k], (uint32_t*)p->d_bits[k],
                        met ? p->d_metric[k] : nullptr, nullptr, p->s_dec);
    if (e == hipSuccess && st == MIVIT_OK) e = hipEventRecord(p->ev_dec[k], p->s_dec);
    // copy out
    if (e == hipSuccess && st == MIVIT_OK) e = hipStreamWaitEvent(p->s_out, p->ev_dec[k], 0);
    if (e == hipSuccess && st == MIVIT_OK && p->bits_bytes)
      e = hipMemcpyAsync(bits + (size_t)b * p->bits_bytes, p->d_bits[k], p->bits_bytes,
                         hipMemcpyDeviceToHost, p->s_out);
    if (e == hipSuccess && st == MIVIT_OK && met && p->metric_bytes)
      e = hipMemcpyAsync(met + (size_t)b * p->metric_bytes, p->d_metric[k], p->metric_bytes,
                         hipMemcpyDeviceToHost, p->s_out);
    if (e == hipSuccess && st == MIVIT_OK) e = hipEventRecord(p->ev_out[k], p->s_out);
  }
  // drain all three streams whatever happened
  for (hipStream_t s : {p->s_in, p->s_dec, p->s_out}) {
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
  }
  if (st != MIVIT_OK) return st;
  return e == hipSuccess ? MIVIT_OK : MIVIT_EHIP;
}

mivit_status mivit_pipe_destroy(mivit_pipe* p) {
  if (!p) return MIVIT_EINVAL;
  DeviceScope scope(p->device);
  for (hipStream_t s : {p->s_in, p->s_dec, p->s_out})
    if (s) (void)hipStreamSynchronize(s);
  release(p);
  return MIVIT_OK;
}

}  // extern "C"
