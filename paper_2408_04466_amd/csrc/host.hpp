// Host-side helpers shared by the C ABI translation units: the per-thread
// error message, status helpers, loop-table validation and the BVH handle.
#pragma once

#include <string>

#include "kernels.hpp"

namespace wn {
namespace host {

extern thread_local std::string g_err;

wn_status fail(wn_status s, const char* fmt, ...);
wn_status hip_fail(hipError_t e, const char* what);
wn_status make_loops(const int64_t* loop_off, int32_t nloops, int32_t min_len, int64_t* nb_out,
                     LoopTable* L);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace host
}  // namespace wn

#define WN_HIP(call, what)                                     \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return ::wn::host::hip_fail(e_, what); \
  } while (0)

struct wn_bvh {
  wn::Frame F;
  double dir[3];
  int32_t nv = 0, nf = 0;
  double4* Vr = nullptr;
  int4* tris = nullptr;
  wn::BvhNode* nodes = nullptr;
  float4* leafbox = nullptr;
  float* leafz = nullptr;
  void* mem = nullptr;   // the one allocation holding the arrays above
};

