// Host-side streaming over the C ABI, built only on the public plan API.
//
// Pipeline: batches of soft values in host memory are copied to the device,
// decoded and their bits (and metrics) copied back, with the copy-in of one
// batch, the decode of another and the copy-out of a third in flight at once
// on three streams.
//
// Continuous stream: the soft values of one long stream arrive in pieces of
// any size.  The stream is cut into the windows of §III (cores of `chunk`
// stages with `overlap` stages on each side, the windows a plan forms for
// the whole stream as one chunked frame); a window is decoded as soon as its
// right overlap has arrived and its core bits are emitted in stream order,
// so the concatenated output equals that plan's.  The soft values not yet
// consumed stay in a device buffer between calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <utility>
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

// ---------------------------------------------------------------------------
// Continuous stream.
// ---------------------------------------------------------------------------

struct mivit_stream {
  mivit_code code;
  mivit_opts opts;   // the stream's options; window plans use chunk = overlap = 0
  uint16_t flags = 0;  // MIVIT_START_KNOWN | MIVIT_END_ZERO of the whole stream
  int device = 0;
  int64_t chunk = 0, overlap = 0, max_push = 0;
  size_t stage_bytes = 0;  // beta soft values
  void* buf[2] = {nullptr, nullptr};  // unconsumed soft values; the other one is the spare
  int cur = 0;
  int64_t base = 0;       // stream stage of buf[cur]'s first soft value
  int64_t have = 0;       // stages held from base on
  int64_t next_core = 0;  // first window not yet decoded
  bool finished = false;
  // window plans by (first window, or the first window whose start is above
  // stage 0 if later; number of windows)
  std::map<std::pair<int64_t, int64_t>, mivit_plan*> plans;
};

namespace {

constexpr size_t kMaxStreamPlans = 8;

void release_stream(mivit_stream* s) {
  for (auto& kv : s->plans) (void)mivit_plan_destroy(kv.second);
  for (void* b : s->buf) (void)hipFree(b);
  delete s;
}

// The window of core c (stages [c*chunk, (c+1)*chunk) of a stream of S
// stages; S < 0: not yet known, so the window is not clipped at the end).
struct Window {
  int64_t w0, w1, c0, c1;
};

Window window_of(const mivit_stream* s, int64_t c, int64_t S) {
  Window w;
  w.c0 = c * s->chunk;
  w.c1 = S < 0 ? w.c0 + s->chunk : std::min(S, w.c0 + s->chunk);
  w.w0 = std::max<int64_t>(0, w.c0 - s->overlap);
  w.w1 = S < 0 ? w.c1 + s->overlap : std::min(S, w.c1 + s->overlap);
  return w;
}

// Plan for windows c0 .. c0+n-1 read from a buffer starting at stream stage
// window_of(c0).w0, bits written from bit 0.  S as in window_of.
mivit_status make_window_plan(const mivit_stream* s, int64_t c0, int64_t n, int64_t S,
                              mivit_plan** out) {
  std::vector<mivit_frame> fr((size_t)n);
  const int64_t base = window_of(s, c0, S).w0;
  for (int64_t k = 0; k < n; ++k) {
    const Window w = window_of(s, c0 + k, S);
    mivit_frame& f = fr[(size_t)k];
    std::memset(&f, 0, sizeof f);
    f.llr_offset = (w.w0 - base) * s->code.beta;
    f.bit_offset = k * s->chunk;
    f.n_stages = (int32_t)(w.w1 - w.w0);
    f.out_begin = (int32_t)(w.c0 - w.w0);
    f.n_out = (int32_t)(w.c1 - w.c0);
    f.code = 0;
    uint16_t fl = 0;
    if (w.w0 == 0 && (s->flags & MIVIT_START_KNOWN)) fl |= MIVIT_START_KNOWN;
    if (S >= 0 && w.c1 == S && (s->flags & MIVIT_END_ZERO)) fl |= MIVIT_END_ZERO;
    f.flags = fl;
  }
  mivit_opts o = s->opts;
  o.chunk = 0;
  o.overlap = 0;
  return mivit_plan_create(out, &s->code, 1, fr.data(), (int32_t)n, &o);
}

// Keep the soft values from stream stage new_base on (in buf[cur]) at the
// start of the spare buffer and make it current.
hipError_t shift_carry(mivit_stream* s, int64_t new_base, hipStream_t st) {
  if (new_base == s->base) return hipSuccess;
  const int64_t keep = s->base + s->have - new_base;
  hipError_t e = hipSuccess;
  if (keep > 0)
    e = hipMemcpyAsync(s->buf[s->cur ^ 1],
                       (const char*)s->buf[s->cur] + (size_t)(new_base - s->base) * s->stage_bytes,
                       (size_t)keep * s->stage_bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  s->cur ^= 1;
  s->base = new_base;
  s->have = keep;
  return hipSuccess;
}

}  // namespace

extern "C" {

mivit_status mivit_stream_create(mivit_stream** out, const mivit_code* code,
                                 const mivit_opts* opts, uint32_t flags,
                                 int64_t max_push_stages) {
  if (!out) return MIVIT_EINVAL;
  *out = nullptr;
  if (!code || !opts || opts->chunk <= 0 || opts->chunk % 32 != 0 || opts->overlap < 0 ||
      max_push_stages <= 0 || (flags & ~(uint32_t)(MIVIT_START_KNOWN | MIVIT_END_ZERO)))
    return MIVIT_EINVAL;
  if ((int64_t)opts->chunk + 2 * (int64_t)opts->overlap > INT32_MAX / 2) return MIVIT_EINVAL;
  // the code and the remaining options are checked by an empty plan
  mivit_opts o = *opts;
  o.chunk = 0;
  o.overlap = 0;
  mivit_plan* probe = nullptr;
  mivit_status st = mivit_plan_create(&probe, code, 1, nullptr, 0, &o);
  if (st != MIVIT_OK) return st;
  mivit_plan_info info;
  st = mivit_plan_get_info(probe, &info);
  (void)mivit_plan_destroy(probe);
  if (st != MIVIT_OK) return st;
  mivit_stream* s = new (std::nothrow) mivit_stream();
  if (!s) return MIVIT_ENOMEM;
  s->code = *code;
  s->opts = *opts;
  s->flags = (uint16_t)flags;
  s->device = info.device;
  s->chunk = opts->chunk;
  s->overlap = opts->overlap;
  s->max_push = max_push_stages;
  const size_t esz = opts->dtype == MIVIT_I8 ? 1 : opts->dtype == MIVIT_F16 ? 2 : 4;
  s->stage_bytes = esz * (size_t)code->beta;
  // unconsumed values stay below chunk + 2*overlap stages between calls
  const size_t cap = (size_t)(s->chunk + 2 * s->overlap + max_push_stages) * s->stage_bytes;
  DeviceScope scope(s->device);
  hipError_t e = hipMalloc(&s->buf[0], cap);
  if (e == hipSuccess) e = hipMalloc(&s->buf[1], cap);
  if (e != hipSuccess) {
    release_stream(s);
    return e == hipErrorOutOfMemory ? MIVIT_ENOMEM : MIVIT_EHIP;
  }
  *out = s;
  return MIVIT_OK;
}

mivit_status mivit_stream_push(mivit_stream* s, const void* llr, int64_t n_stages,
                               uint32_t* bits, int64_t* n_bits, void* stream) {
  if (!s || !n_bits || n_stages < 0 || n_stages > s->max_push || s->finished) return MIVIT_EINVAL;
  if ((n_stages > 0 && !llr) || !bits) return MIVIT_EINVAL;
  *n_bits = 0;
  DeviceScope scope(s->device);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (n_stages > 0)
    e = hipMemcpyAsync((char*)s->buf[s->cur] + (size_t)s->have * s->stage_bytes, llr,
                       (size_t)n_stages * s->stage_bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return MIVIT_EHIP;
  s->have += n_stages;
  // windows whose right overlap has arrived: (c+1)*chunk + overlap <= received
  const int64_t received = s->base + s->have;
  const int64_t ready =
      received >= s->chunk + s->overlap ? (received - s->overlap) / s->chunk : 0;
  const int64_t n = ready - s->next_core;
  if (n > 0) {
    // windows from c_flat on start at core start - overlap > 0, so their
    // frames do not depend on where the run of windows begins
    const int64_t c_flat = s->overlap / s->chunk + 1;
    const std::pair<int64_t, int64_t> key(std::min(s->next_core, c_flat), n);
    auto it = s->plans.find(key);
    mivit_plan* plan = nullptr;
    if (it != s->plans.end()) {
      plan = it->second;
    } else {
      if (s->plans.size() >= kMaxStreamPlans) {
        for (auto& kv : s->plans) (void)mivit_plan_destroy(kv.second);
        s->plans.clear();
      }
      mivit_status ps = make_window_plan(s, s->next_core, n, -1, &plan);
      if (ps != MIVIT_OK) return ps;
      s->plans[key] = plan;
    }
    mivit_status ds = mivit_decode(plan, s->buf[s->cur], bits, nullptr, nullptr, stream);
    if (ds != MIVIT_OK) return ds;
    s->next_core = ready;
    *n_bits = n * s->chunk;
    e = shift_carry(s, window_of(s, s->next_core, -1).w0, st);
    if (e != hipSuccess) return MIVIT_EHIP;
  }
  return MIVIT_OK;
}

mivit_status mivit_stream_finish(mivit_stream* s, uint32_t* bits, int64_t* n_bits,
                                 void* stream) {
  if (!s || !n_bits || !bits || s->finished) return MIVIT_EINVAL;
  *n_bits = 0;
  DeviceScope scope(s->device);
  const int64_t S = s->base + s->have;
  s->finished = true;
  const int64_t total = (S + s->chunk - 1) / s->chunk;  // windows of the whole stream
  const int64_t n = total - s->next_core;
  if (n <= 0) return MIVIT_OK;
  mivit_plan* plan = nullptr;
  mivit_status st = make_window_plan(s, s->next_core, n, S, &plan);
  if (st != MIVIT_OK) return st;
  st = mivit_decode(plan, s->buf[s->cur], bits, nullptr, nullptr, stream);
  // destroying the plan waits for the device, so the decode is complete
  const mivit_status ds = mivit_plan_destroy(plan);
  if (st != MIVIT_OK) return st;
  if (ds != MIVIT_OK) return ds;
  *n_bits = S - s->next_core * s->chunk;
  s->next_core = total;
  return MIVIT_OK;
}

mivit_status mivit_stream_destroy(mivit_stream* s) {
  if (!s) return MIVIT_EINVAL;
  DeviceScope scope(s->device);
  (void)hipDeviceSynchronize();
  release_stream(s);
  return MIVIT_OK;
}

}  // extern "C"
