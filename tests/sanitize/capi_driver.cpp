// Host-side argument validation of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer: every call below is rejected (or is a no-op)
// before any device work, so the driver runs without a GPU.  The cases
// mirror tests/test_capi.py.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/mivit.h"

static int failures = 0;

static void expect(const char* what, mivit_status got, mivit_status want) {
  if (got != want) {
    std::printf("FAIL %s: got %d want %d\n", what, (int)got, (int)want);
    ++failures;
  }
}

static mivit_code code(int K, std::vector<uint32_t> gens) {
  mivit_code c;
  std::memset(&c, 0, sizeof c);
  c.K = K;
  c.beta = (int32_t)gens.size();
  for (size_t b = 0; b < gens.size() && b < 4; ++b) c.gen[b] = gens[b];
  return c;
}

static mivit_frame frame() {
  mivit_frame f;
  std::memset(&f, 0, sizeof f);
  f.llr_offset = 0;
  f.bit_offset = 0;
  f.n_stages = 10;
  f.out_begin = 0;
  f.n_out = 4;
  f.code = 0;
  f.flags = MIVIT_START_KNOWN | MIVIT_END_ZERO;
  return f;
}

static mivit_status plan(const std::vector<mivit_code>& codes, const std::vector<mivit_frame>& fr,
                         const mivit_opts& o) {
  mivit_plan* p = nullptr;
  mivit_status s = mivit_plan_create(&p, codes.data(), (int32_t)codes.size(),
                                     fr.empty() ? nullptr : fr.data(), (int32_t)fr.size(), &o);
  if (p) {
    std::printf("FAIL a rejected plan left a handle\n");
    ++failures;
    mivit_plan_destroy(p);
  }
  return s;
}

int main() {
  const mivit_code k7 = code(7, {0133, 0171});
  mivit_opts o0;
  std::memset(&o0, 0, sizeof o0);

  // codes
  expect("K too small", plan({code(2, {3, 3})}, {frame()}, o0), MIVIT_EINVAL);
  expect("K too large", plan({code(10, {01001, 01001})}, {frame()}, o0), MIVIT_EINVAL);
  expect("beta 1", plan({code(7, {0133})}, {frame()}, o0), MIVIT_EINVAL);
  expect("generator too wide", plan({code(7, {0333, 0171})}, {frame()}, o0), MIVIT_EINVAL);
  expect("no LSB tap", plan({code(7, {0132, 0171})}, {frame()}, o0), MIVIT_EUNSUPPORTED);
  expect("no MSB tap", plan({code(7, {0033, 0171})}, {frame()}, o0), MIVIT_EUNSUPPORTED);

  // frames
  for (int k = 0; k < 8; ++k) {
    mivit_frame f = frame();
    switch (k) {
      case 0: f.code = 1; break;
      case 1: f.code = -1; break;
      case 2: f.n_stages = -1; break;
      case 3: f.n_out = 11; break;
      case 4: f.out_begin = 8; break;
      case 5: f.bit_offset = 5; break;
      case 6: f.llr_offset = -2; break;
      case 7: f.flags = 8; break;
    }
    expect("bad frame", plan({k7}, {f}, o0), MIVIT_EINVAL);
  }
  expect("overlapping outputs", plan({k7}, {frame(), frame()}, o0), MIVIT_EINVAL);

  // options
  struct { int dtype, radix, chunk, overlap, variant; uint32_t flags; } bad[] = {
      {3, 0, 0, 0, 0, 0},  {-1, 0, 0, 0, 0, 0}, {0, 3, 0, 0, 0, 0},   {0, 16, 0, 0, 0, 0},
      {0, 4, 0, 0, 0, 0},  {2, 4, 0, 0, 0, 0},  {0, 8, 0, 0, 0, 0},   {2, 8, 0, 0, 0, 0},
      {0, 0, -1, 0, 0, 0}, {0, 0, 100, 0, 0, 0}, {0, 0, 0, -1, 0, 0}, {0, 0, 0, 0, 9, 0},
      {0, 0, 0, 0, 0, 16}, {0, 0, 0, 0, 0, 1u << 31},
  };
  for (const auto& b : bad) {
    mivit_opts o = o0;
    o.dtype = b.dtype;
    o.radix = b.radix;
    o.chunk = b.chunk;
    o.overlap = b.overlap;
    o.variant = b.variant;
    o.flags = b.flags;
    expect("bad options", plan({k7}, {frame()}, o), MIVIT_EINVAL);
  }
  for (int r = 0; r < 2; ++r) {
    mivit_opts o = o0;
    o.reserved[r] = 1;
    expect("reserved option", plan({k7}, {frame()}, o), MIVIT_EINVAL);
  }
  for (int v = 1; v <= 2; ++v) {
    mivit_opts o = o0;
    o.dtype = MIVIT_F16;
    o.variant = v;
    expect("float16 variant", plan({k7}, {frame()}, o), MIVIT_EUNSUPPORTED);
  }
  {
    mivit_opts o = o0;
    o.dtype = MIVIT_I8;
    o.radix = 8;
    expect("radix 8, K = 3", plan({code(3, {7, 5})}, {frame()}, o), MIVIT_EUNSUPPORTED);
    o.variant = 1;
    expect("radix 8, variant 1", plan({k7}, {frame()}, o), MIVIT_EUNSUPPORTED);
    o.radix = 2;
    o.variant = 5;
    expect("variant 5, radix 2", plan({k7}, {frame()}, o), MIVIT_EUNSUPPORTED);
    o.variant = 6;
    expect("variant 6, int8", plan({code(9, {0557, 0663, 0711})}, {frame()}, o),
           MIVIT_EUNSUPPORTED);
    o.dtype = MIVIT_F32;
    expect("variant 6, K = 7", plan({k7}, {frame()}, o), MIVIT_EUNSUPPORTED);
    o.variant = 7;
    expect("variant 7, K = 8", plan({code(8, {0247, 0371})}, {frame()}, o), MIVIT_EUNSUPPORTED);
    o.variant = 8;
    expect("variant 8, float32", plan({code(9, {0557, 0663, 0711})}, {frame()}, o),
           MIVIT_EUNSUPPORTED);
    o.dtype = MIVIT_I8;
    expect("variant 8, K = 7", plan({k7}, {frame()}, o), MIVIT_EUNSUPPORTED);
  }

  // null handles and pointers
  expect("plan_create null", mivit_plan_create(nullptr, nullptr, 0, nullptr, 0, nullptr),
         MIVIT_EINVAL);
  expect("plan_create_on null", mivit_plan_create_on(nullptr, 0, nullptr, 0, nullptr, 0, nullptr),
         MIVIT_EINVAL);
  expect("decode null", mivit_decode(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("grad null", mivit_decode_grad(nullptr, nullptr, nullptr, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("destroy null", mivit_plan_destroy(nullptr), MIVIT_EINVAL);
  expect("info null", mivit_plan_get_info(nullptr, nullptr), MIVIT_EINVAL);
  expect("describe null", mivit_plan_describe(nullptr, nullptr, 0), MIVIT_EINVAL);
  expect("quantize n < 0", mivit_quantize_i8(nullptr, nullptr, -1, 1.0f, nullptr), MIVIT_EINVAL);
  expect("quantize null", mivit_quantize_i8(nullptr, nullptr, 10, 1.0f, nullptr), MIVIT_EINVAL);
  expect("quantize scale 0", mivit_quantize_i8(nullptr, nullptr, 0, 0.0f, nullptr), MIVIT_EINVAL);
  expect("pipe null", mivit_pipe_create(nullptr, nullptr, 3), MIVIT_EINVAL);
  expect("pipe run null", mivit_pipe_run(nullptr, nullptr, nullptr, nullptr, 1), MIVIT_EINVAL);
  expect("pipe destroy null", mivit_pipe_destroy(nullptr), MIVIT_EINVAL);
  {
    mivit_opts o = o0;
    o.dtype = MIVIT_I8;
    o.chunk = 2048;
    o.overlap = 64;
    mivit_stream* h = nullptr;
    expect("stream null out", mivit_stream_create(nullptr, &k7, &o, 1, 1024), MIVIT_EINVAL);
    expect("stream null code", mivit_stream_create(&h, nullptr, &o, 1, 1024), MIVIT_EINVAL);
    o.chunk = 100;
    expect("stream bad chunk", mivit_stream_create(&h, &k7, &o, 1, 1024), MIVIT_EINVAL);
    int64_t nb = 0;
    expect("stream push null", mivit_stream_push(nullptr, nullptr, 0, nullptr, &nb, nullptr),
           MIVIT_EINVAL);
    expect("stream destroy null", mivit_stream_destroy(nullptr), MIVIT_EINVAL);
  }

  // the one-call entry point
  uint32_t buf[16];
  uint32_t* fake = buf;  // never dereferenced: every case fails validation
  const mivit_code k10 = code(10, {01001, 01777}), k7lsb = code(7, {0132, 0171});
  expect("uniform no llr", mivit_decode_uniform(nullptr, 0, &k7, 4, 100, 1, fake, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform no bits", mivit_decode_uniform(fake, 0, &k7, 4, 100, 1, nullptr, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform dtype", mivit_decode_uniform(fake, 7, &k7, 4, 100, 1, fake, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform frames", mivit_decode_uniform(fake, 0, &k7, -1, 100, 1, fake, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform length", mivit_decode_uniform(fake, 0, &k7, 4, -5, 1, fake, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform terminated", mivit_decode_uniform(fake, 0, &k7, 4, 100, 2, fake, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform K 10", mivit_decode_uniform(fake, 0, &k10, 4, 100, 1, fake, nullptr, nullptr),
         MIVIT_EINVAL);
  expect("uniform no LSB tap",
         mivit_decode_uniform(fake, 0, &k7lsb, 4, 100, 1, fake, nullptr, nullptr),
         MIVIT_EUNSUPPORTED);
  expect("uniform empty", mivit_decode_uniform(nullptr, 0, &k7, 0, 100, 1, nullptr, nullptr, nullptr),
         MIVIT_OK);

  if (std::strlen(mivit_version()) == 0 || std::strlen(mivit_strerror(MIVIT_EINVAL)) == 0) {
    std::printf("FAIL version or strerror\n");
    ++failures;
  }
  if (failures) return 1;
  std::printf("capi sanitizer driver: ok\n");
  return 0;
}
