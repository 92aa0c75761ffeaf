// Test-only stand-ins for the kernel objects, so that the C-ABI host code (srtm_api.hip) can be
// built alone with host sanitizers: a call that passes validation gets SRTM_E_UNSUPPORTED here
// instead of launching anything.
#include "srtm_entry.h"

namespace srtm {
#define SRTM_STUB(a, b)                                                                                            \
  srtm_status run_pair_##a##_##b(int, const srtm_shape&, const Ptrs&, bool, hipStream_t, hipEvent_t const*, int,   \
                                 int, void*, void*, void*, void*) {                                                \
    return SRTM_E_UNSUPPORTED;                                                                                     \
  }                                                                                                                \
  srtm_status run_batch_pair_##a##_##b(int, const void*, int, int64_t, int, void*, int32_t*, hipStream_t, bool) {  \
    return SRTM_E_UNSUPPORTED;                                                                                     \
  }
SRTM_PAIRS(SRTM_STUB)
#undef SRTM_STUB
srtm_status run_mixed_double(const SeqDesc*, const void*, int, int64_t, int, void*, int32_t*, hipStream_t) {
  return SRTM_E_UNSUPPORTED;
}
srtm_status run_mixed_float(const SeqDesc*, const void*, int, int64_t, int, void*, int32_t*, hipStream_t) {
  return SRTM_E_UNSUPPORTED;
}
}  // namespace srtm
