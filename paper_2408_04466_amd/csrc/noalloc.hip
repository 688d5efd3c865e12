// wn_backward_noalloc: the 3D adjoint with its workspace in a library-held
// device array instead of stream allocations, for callers that cannot
// allocate (code under graph capture, serving loops that forbid it).
//
// `scratch` is a file-scope device array; each GPU the library runs on holds
// its own copy for the life of the process.  In host code its name is only a
// stand-in: its device address comes from hipGetSymbolAddress, looked up
// once per device with that device current and kept here.  Every call on a
// device shares that device's array, so calls that overlap on one GPU race.
#include <mutex>

#include "host.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)WN_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on first use
// with the device current).
wn_status scratch_ptr(void** out) {
  int dev = -1;
  WN_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return wn::host::fail(WN_ERR_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    WN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return wn::host::fail(WN_ERR_INTERNAL, "scratch has no device address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return WN_OK;
}

}  // namespace

extern "C" wn_status wn_backward_noalloc(const float* bnd_xyz, const int64_t* loop_off, int32_t nloops,
                                         const float* qx, const float* qy, const float* qz, int64_t nq,
                                         const float* grad_w, float* grad_q, float* grad_bnd, void* stream) {
  wn::host::g_err.clear();
  wn::LoopTable L;
  int64_t nb = 0;
  wn_status st = wn::host::check_backward(bnd_xyz, loop_off, nloops, qx, qy, qz, nq, grad_w, &L, &nb);
  if (st) return st;
  if (nloops > WN_MAX_LOOPS)   // a longer table would have to be copied to device memory
    return wn::host::fail(WN_ERR_UNSUPPORTED, "wn_backward_noalloc takes at most %d boundary loops (got %d; use "
                          "wn_backward)", WN_MAX_LOOPS, nloops);
  const wn::host::AdjPlan P = wn::host::plan_backward(nq, nb, nloops, grad_q != nullptr, grad_bnd != nullptr);
  const size_t need = wn::host::plan_bytes(P);
  if (need > kScratchBytes)
    return wn::host::fail(WN_ERR_UNSUPPORTED,
                          "wn_backward_noalloc needs %zu bytes of workspace for %lld queries over %lld boundary "
                          "vertices; its scratch holds %zu (use wn_backward)",
                          need, (long long)nq, (long long)nb, kScratchBytes);
  void* base = nullptr;
  if ((st = scratch_ptr(&base))) return st;
  const wn::host::AdjWork W = wn::host::carve_backward(P, base);
  return wn::host::run_backward(P, bnd_xyz, L, nb, qx, qy, qz, nq, grad_w, grad_q, grad_bnd, W,
                                wn::host::as_stream(stream));
}
