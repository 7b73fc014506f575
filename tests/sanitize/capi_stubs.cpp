// Stand-ins for the library's kernel launchers, so that the host-side plan
// and argument code (mivit_api.cpp, mivit_pipe.cpp) links into the
// sanitizer driver without any device code.  The driver's calls are all
// rejected before a launch, so none of these runs; each would report an
// error if it did.
#include "../../paper_2011_13579_amd/csrc/mivit_device.h"

namespace mivit {
hipError_t launch_fwd(int, int, int, const DevCode*, const Item*, int, const void*, uint64_t*,
                      void*, int32_t*, int32_t*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_grad(const DevCode*, const GradFrame*, int, int, const uint32_t*, const float*,
                       float*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_quant(const float*, int8_t*, int64_t, float, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fwd_rot(int, int, int, int, const DevCode*, const Item*, const int2*, int,
                          const void*, uint64_t*, void*, int32_t*, int32_t*, int32_t*, int,
                          hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fwd_wide(int, int, int, int, bool, const DevCode*, const Item*, const SplitUnit*, int,
                           const void*, uint64_t*, void*, int32_t*, int32_t*, WideBound*, int64_t*,
                           const SplitUnit*, int, int64_t*, SplitUnit*, int32_t*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_tb_seg(int, const DevCode*, const Item*, int, const uint64_t*, const int32_t*,
                         uint32_t*, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fwd_r4p(int, const DevCode*, const Item*, const SplitUnit*, int, const int8_t*,
                          uint64_t*, int64_t*, int32_t*, int32_t*, int32_t*, int, R4Bound*,
                          int64_t*, const SplitUnit*, int, int64_t*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fwd_r4q(const DevCode*, const Item*, const SplitUnit*, int, const int8_t*,
                          uint64_t*, int64_t*, int32_t*, int32_t*, int32_t*, int, R4Bound*,
                          int64_t*, const SplitUnit*, int, int64_t*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_tb_r4p(int, const Item*, const int2*, int, const uint64_t*, const int32_t*,
                         uint32_t*, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fwd_r4_mfma(const MfmaGroups&, const DevCode*, const Item*, int, const int8_t*,
                              uint64_t*, int64_t*, int32_t*, int32_t*, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_zero_i32(int32_t*, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_fill_random(void*, int64_t, int, uint32_t, hipStream_t) {
  return hipErrorInvalidValue;
}
bool mfma_groups(int, int, const uint32_t*, MfmaGroups*) { return false; }
}  // namespace mivit
