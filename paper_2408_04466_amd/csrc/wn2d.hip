// 2D cubic Bezier loops (placeholder until the kernels land).
#include "kernels.hpp"

extern "C" wn_status wn_eval_2d(wn_dtype, const void*, int64_t, const int64_t*, const uint8_t*, int32_t,
                                int32_t, const void*, const void*, int64_t, int64_t, void*, int32_t*, void*) {
  return WN_ERR_UNSUPPORTED;
}
