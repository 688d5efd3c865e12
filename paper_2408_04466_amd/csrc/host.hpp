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
// A table of more than WN_MAX_LOOPS loops (validated by make_loops) copied to
// device memory allocated on s; *owned is that allocation (null for a short
// table), to be freed on s after the launches that read it.
wn_status upload_loops(const int64_t* loop_off, LoopTable* L, hipStream_t s, int32_t** owned);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Launch plan of the 3D adjoint for nq queries over nb boundary vertices:
// the tile shape, the boundary ranges and the element counts of the
// workspace arrays (0 where an array is not needed).
struct AdjPlan {
  int qpl = 1;
  int64_t nblocks = 0, rows = 0;
  int parts = 1;
  int32_t span = 0;
  size_t n_pv = 0;    // float [rows][nb][3]: per-wavefront vertex partials
  size_t n_pl = 0;    // float [rows][nloops][3]: closing-edge shares of first vertices
  size_t n_tmp = 0;   // double [groups][nb][3]: first reduction stage
  size_t n_pc = 0;    // float [rows][parts][3]: carry slots of split ranges
  size_t n_gqp = 0;   // float [parts][nq][3]: per-range query gradients
};
struct AdjWork {
  float* pv = nullptr;
  float* pl = nullptr;
  double* tmp = nullptr;
  float* pc = nullptr;
  float* gqp = nullptr;
};

wn_status check_backward(const float* bnd_xyz, const int64_t* loop_off, int32_t nloops, const float* qx,
                         const float* qy, const float* qz, int64_t nq, const float* grad_w, LoopTable* L,
                         int64_t* nb);
AdjPlan plan_backward(int64_t nq, int64_t nb, int32_t nloops, bool want_q, bool want_bnd);
// Bytes of one block holding every workspace array of the plan (each
// 256-byte aligned), and the arrays carved out of such a block.
size_t plan_bytes(const AdjPlan& P);
AdjWork carve_backward(const AdjPlan& P, void* base);
// Enqueue the adjoint kernels and reductions of the plan on s.
wn_status run_backward(const AdjPlan& P, const float* bnd_xyz, const LoopTable& L, int64_t nb, const float* qx,
                       const float* qy, const float* qz, int64_t nq, const float* grad_w, float* grad_q,
                       float* grad_bnd, const AdjWork& W, hipStream_t s);

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
  wn::TriRec* tris = nullptr;
  wn::BvhNode4* nodes = nullptr;   // four-wide tree, indexed like the binary one
  float4* leafbox = nullptr;
  float* leafz = nullptr;
  void* mem = nullptr;   // the one allocation holding the arrays above
};

