// Host side of the C ABI declared in include/wn.h: argument validation,
// handles, the frame of the ray direction, boundary extraction, and the
// launch sequence of each entry point.
#include <new>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adj3d.hpp"
#include "bvh_build.hpp"
#include "host.hpp"
#include "adj3d.hpp"
#include "kernels.hpp"

namespace wn {
namespace host {

thread_local std::string g_err;

wn_status fail(wn_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

wn_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(WN_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
  return fail(WN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Validate a host loop table and copy it into the kernel-argument form (a
// table of more than WN_MAX_LOOPS loops is left for upload_loops).
wn_status make_loops(const int64_t* loop_off, int32_t nloops, int32_t min_len, int64_t* nb_out,
                     wn::LoopTable* L) {
  if (nloops < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nloops must be >= 0 (got %d)", nloops);
  std::memset(L, 0, sizeof *L);
  L->n = nloops;
  if (nloops == 0) {
    *nb_out = 0;
    return WN_OK;
  }
  if (!loop_off) return fail(WN_ERR_INVALID_ARGUMENT, "loop_off is NULL with nloops = %d", nloops);
  if (loop_off[0] != 0) return fail(WN_ERR_INVALID_ARGUMENT, "loop_off[0] must be 0");
  for (int32_t l = 0; l < nloops; ++l) {
    const int64_t len = loop_off[l + 1] - loop_off[l];
    if (len < min_len)
      return fail(WN_ERR_INVALID_ARGUMENT, "loop %d has %lld entries (need >= %d)", l, (long long)len, min_len);
  }
  if (loop_off[nloops] > INT32_MAX - 1)
    return fail(WN_ERR_UNSUPPORTED, "too many boundary vertices (%lld)", (long long)loop_off[nloops]);
  if (nloops <= WN_MAX_LOOPS)
    for (int32_t l = 0; l <= nloops; ++l) L->off[l] = (int32_t)loop_off[l];
  *nb_out = loop_off[nloops];
  return WN_OK;
}

wn_status upload_loops(const int64_t* loop_off, LoopTable* L, hipStream_t s, int32_t** owned) {
  *owned = nullptr;
  if (L->n <= WN_MAX_LOOPS) return WN_OK;
  std::vector<int32_t> h((size_t)L->n + 1);
  for (int32_t l = 0; l <= L->n; ++l) h[l] = (int32_t)loop_off[l];
  int32_t* d = nullptr;
  hipError_t e = hipMallocAsync((void**)&d, h.size() * sizeof(int32_t), s);
  if (e == hipSuccess) e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  // the host copy must outlive the transfer
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    if (d) hipFreeAsync(d, s);
    return hip_fail(e, "loop table");
  }
  L->dev = d;
  *owned = d;
  return WN_OK;
}

// Argument checks of the 3D adjoint entry points.
wn_status check_backward(const float* bnd_xyz, const int64_t* loop_off, int32_t nloops, const float* qx,
                         const float* qy, const float* qz, int64_t nq, const float* grad_w, LoopTable* L,
                         int64_t* nb) {
  wn_status st = make_loops(loop_off, nloops, 3, nb, L);
  if (st) return st;
  if (*nb > 0 && !bnd_xyz) return fail(WN_ERR_INVALID_ARGUMENT, "bnd_xyz is NULL");
  if (nq < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nq must be >= 0");
  if (nq > 0 && (!qx || !qy || !qz)) return fail(WN_ERR_INVALID_ARGUMENT, "NULL query pointer");
  if (nq > 0 && !grad_w) return fail(WN_ERR_INVALID_ARGUMENT, "grad_w is NULL");
  return WN_OK;
}

AdjPlan plan_backward(int64_t nq, int64_t nb, int32_t nloops, bool want_q, bool want_bnd) {
  AdjPlan P;
  P.qpl = wn::adj3d_qpl_ranges(nq, nb);
  P.nblocks = wn::adj3d_blocks(nq, P.qpl);
  P.rows = wn::adj3d_rows(P.nblocks);
  // few query tiles over a long boundary: split the boundary into ranges
  P.parts = wn::adj3d_parts(P.nblocks, nb);
  P.span = wn::adj3d_span(nb, P.parts);
  if (want_bnd && nb > 0 && P.rows > 0) {
    P.n_pv = (size_t)(P.rows * nb * 3);
    P.n_pl = (size_t)(P.rows * nloops * 3);
    P.n_tmp = (size_t)(wn::reduce_groups(P.rows) * nb * 3);
    if (P.parts > 1) P.n_pc = (size_t)(P.rows * P.parts * 3);
  }
  if (P.parts > 1 && want_q && nq > 0 && nb > 0) P.n_gqp = (size_t)(P.parts * nq * 3);
  return P;
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t plan_bytes(const AdjPlan& P) {
  return round256(P.n_pv * sizeof(float)) + round256(P.n_pl * sizeof(float)) +
         round256(P.n_tmp * sizeof(double)) + round256(P.n_pc * sizeof(float)) +
         round256(P.n_gqp * sizeof(float));
}

AdjWork carve_backward(const AdjPlan& P, void* base) {
  AdjWork W;
  char* b = static_cast<char*>(base);
  size_t o = 0;
  auto take = [&](size_t bytes) -> void* {
    if (!bytes) return nullptr;
    void* p = b + o;
    o += round256(bytes);
    return p;
  };
  W.pv = static_cast<float*>(take(P.n_pv * sizeof(float)));
  W.pl = static_cast<float*>(take(P.n_pl * sizeof(float)));
  W.tmp = static_cast<double*>(take(P.n_tmp * sizeof(double)));
  W.pc = static_cast<float*>(take(P.n_pc * sizeof(float)));
  W.gqp = static_cast<float*>(take(P.n_gqp * sizeof(float)));
  return W;
}

wn_status run_backward(const AdjPlan& P, const float* bnd_xyz, const LoopTable& L, int64_t nb, const float* qx,
                       const float* qy, const float* qz, int64_t nq, const float* grad_w, float* grad_q,
                       float* grad_bnd, const AdjWork& W, hipStream_t s) {
  if (grad_bnd && nb > 0 && P.rows == 0)
    WN_HIP(wn::fill_u32(reinterpret_cast<unsigned*>(grad_bnd), nb * 3, 0u, s), "zero grad_bnd");
  float* pv = grad_bnd ? W.pv : nullptr;
  if (nq == 0 || !(grad_q || pv)) return WN_OK;
  if (nb == 0) {
    if (grad_q) WN_HIP(wn::fill_u32(reinterpret_cast<unsigned*>(grad_q), nq * 3, 0u, s), "zero grad_q");
    return WN_OK;
  }
  wn::AdjArgs a;
  a.bnd = bnd_xyz;
  a.nb = (int32_t)nb;
  a.qx = qx;
  a.qy = qy;
  a.qz = qz;
  a.nq = nq;
  a.gw = grad_w;
  a.gq = grad_q;
  a.partial = pv;
  a.partial_loop = pv ? W.pl : nullptr;
  hipError_t e;
  if (P.parts > 1) {
    e = wn::launch_adj3d_split(a, L, P.nblocks, P.qpl, P.parts, P.span, pv ? W.pc : nullptr, W.gqp, s);
    if (e == hipSuccess && grad_q) e = wn::launch_sum_parts(W.gqp, P.parts, nq * 3, grad_q, s);
    if (e == hipSuccess && pv)
      e = wn::launch_reduce_partials_split(pv, W.pl, W.pc, P.parts, P.span, P.rows, (int32_t)nb, L, W.tmp,
                                           grad_bnd, s);
  } else {
    e = wn::launch_adj3d(a, L, P.nblocks, P.qpl, s);
    if (e == hipSuccess && pv) e = wn::launch_reduce_partials(pv, W.pl, P.rows, (int32_t)nb, L, W.tmp, grad_bnd, s);
  }
  if (e != hipSuccess) return hip_fail(e, "backward");
  return WN_OK;
}

}  // namespace host
}  // namespace wn

using wn::host::fail;
using wn::host::hip_fail;
using wn::host::g_err;
using wn::host::as_stream;
using wn::host::make_loops;

namespace {

// Unit direction and orthonormal frame (rows e1, e2, d; det +1) in float64.
bool make_rotation(const double dir[3], double d[3], double R[9]) {
  if (!dir) return false;
  const double n = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  if (!std::isfinite(n) || n == 0.0) return false;
  for (int k = 0; k < 3; ++k) d[k] = dir[k] / n;
  int m = 0;
  for (int k = 1; k < 3; ++k)
    if (std::fabs(d[k]) < std::fabs(d[m])) m = k;
  double ax[3] = {0, 0, 0};
  ax[m] = 1.0;
  double e1[3] = {d[1] * ax[2] - d[2] * ax[1], d[2] * ax[0] - d[0] * ax[2], d[0] * ax[1] - d[1] * ax[0]};
  const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int k = 0; k < 3; ++k) e1[k] /= l1;
  const double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
  for (int k = 0; k < 3; ++k) {
    R[k] = e1[k];
    R[3 + k] = e2[k];
    R[6 + k] = d[k];
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------

namespace {

__global__ __launch_bounds__(256) void k_bbox_f32(const float* __restrict__ V, int32_t nv, unsigned* __restrict__ out) {
  // grid-stride over few workgroups (one atomic per value and workgroup)
  __shared__ unsigned red[6][4];
  unsigned v[6] = {0xffffffffu, 0u, 0xffffffffu, 0u, 0xffffffffu, 0u};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nv; i += gridDim.x * 256)
    for (int c = 0; c < 3; ++c) {
      const unsigned u = __float_as_uint(V[3 * i + c]);
      const unsigned o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
      v[2 * c] = min(v[2 * c], o);
      v[2 * c + 1] = max(v[2 * c + 1], o);
    }
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 6; ++k) {
      const unsigned w = (unsigned)__shfl_xor((int)v[k], o, 64);
      v[k] = (k % 2 == 0) ? min(v[k], w) : max(v[k], w);
    }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    unsigned r = red[k][0];
    for (int w = 1; w < 4; ++w) r = (k % 2 == 0) ? min(r, red[k][w]) : max(r, red[k][w]);
    if (k % 2 == 0) atomicMin(&out[k], r);
    else atomicMax(&out[k], r);
  }
}

float ord_to_float(unsigned o) {
  const unsigned u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Several device arrays carved out of one allocation (256-byte aligned).
struct Carve {
  struct Req {
    void** p;
    size_t bytes;
  };
  std::vector<Req> reqs;
  template <class T>
  void add(T** p, size_t n) {
    reqs.push_back({(void**)p, n * sizeof(T)});
  }
  hipError_t alloc(void** base) {
    size_t total = 0;
    for (const Req& r : reqs) total += (r.bytes + 255) & ~(size_t)255;
    *base = nullptr;
    const hipError_t e = hipMalloc(base, total > 0 ? total : 256);
    if (e != hipSuccess) {
      *base = nullptr;
      return e;
    }
    size_t o = 0;
    for (const Req& r : reqs) {
      *r.p = r.bytes ? (void*)((char*)*base + o) : nullptr;
      o += (r.bytes + 255) & ~(size_t)255;
    }
    return hipSuccess;
  }
};

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

int32_t wn_version(void) { return 10000; }

const char* wn_status_string(wn_status s) {
  switch (s) {
    case WN_OK: return "WN_OK";
    case WN_ERR_INVALID_ARGUMENT: return "WN_ERR_INVALID_ARGUMENT";
    case WN_ERR_UNSUPPORTED: return "WN_ERR_UNSUPPORTED";
    case WN_ERR_OUT_OF_MEMORY: return "WN_ERR_OUT_OF_MEMORY";
    case WN_ERR_HIP: return "WN_ERR_HIP";
    case WN_ERR_INTERNAL: return "WN_ERR_INTERNAL";
    default: return "WN_ERR_UNKNOWN";
  }
}

const char* wn_last_error(void) { return g_err.c_str(); }

wn_status wn_boundary_loops(const int32_t* F, int64_t nf, int64_t nv, int32_t* bnd_idx,
                            int64_t* loop_off, int64_t cap, int64_t* nb_out, int32_t* nloops_out) {
  g_err.clear();
  if (nf < 0 || nv < 0) return fail(WN_ERR_INVALID_ARGUMENT, "negative count");
  if (nf > 0 && !F) return fail(WN_ERR_INVALID_ARGUMENT, "F is NULL");
  if (!nb_out || !nloops_out) return fail(WN_ERR_INVALID_ARGUMENT, "NULL output count");
  if (cap < 0 || (cap > 0 && (!bnd_idx || !loop_off)))
    return fail(WN_ERR_INVALID_ARGUMENT, "bad output capacity/buffers");
  // undirected edge key (lo, hi) -> (count, directed a->b of the first use)
  struct HE { int64_t key; int32_t a, b; };
  std::vector<HE> he;
  he.reserve((size_t)(3 * nf));
  for (int64_t f = 0; f < nf; ++f) {
    for (int k = 0; k < 3; ++k) {
      const int32_t a = F[3 * f + k], b = F[3 * f + (k + 1) % 3];
      if (a < 0 || a >= nv || b < 0 || b >= nv)
        return fail(WN_ERR_INVALID_ARGUMENT, "face %lld has an index outside [0, %lld)", (long long)f, (long long)nv);
      const int64_t lo = std::min(a, b), hi = std::max(a, b);
      he.push_back({lo * (nv + 1) + hi, a, b});
    }
  }
  std::stable_sort(he.begin(), he.end(), [](const HE& x, const HE& y) { return x.key < y.key; });
  std::vector<int32_t> next((size_t)nv, -1);
  size_t i = 0;
  int64_t nbe = 0;
  while (i < he.size()) {
    size_t j = i + 1;
    while (j < he.size() && he[j].key == he[i].key) ++j;
    if (j - i == 1) {
      const int32_t a = he[i].a, b = he[i].b;
      if (next[(size_t)a] != -1)
        return fail(WN_ERR_INVALID_ARGUMENT, "vertex %d has two outgoing boundary edges", a);
      next[(size_t)a] = b;
      ++nbe;
    }
    i = j;
  }
  *nb_out = nbe;
  std::vector<char> seen((size_t)nv, 0);
  int64_t pos = 0;
  int32_t nl = 0;
  if (cap > 0) loop_off[0] = 0;
  for (int64_t s = 0; s < nv; ++s) {
    if (next[(size_t)s] < 0 || seen[(size_t)s]) continue;
    int64_t v = s;
    do {
      if (seen[(size_t)v] || next[(size_t)v] < 0)
        return fail(WN_ERR_INVALID_ARGUMENT, "boundary half-edges do not close into loops");
      seen[(size_t)v] = 1;
      if (pos >= cap) return fail(WN_ERR_INVALID_ARGUMENT, "capacity %lld too small", (long long)cap);
      bnd_idx[pos++] = (int32_t)v;
      v = next[(size_t)v];
    } while (v != s);
    ++nl;
    if (nl > cap) return fail(WN_ERR_INVALID_ARGUMENT, "capacity %lld too small", (long long)cap);
    loop_off[nl] = pos;
  }
  *nloops_out = nl;
  return WN_OK;
}

wn_status wn_build_bvh(const float* V, int64_t nv, const int32_t* F, int64_t nf, const double dir[3],
                       void* stream, wn_bvh** out) {
  g_err.clear();
  if (!out) return fail(WN_ERR_INVALID_ARGUMENT, "out is NULL");
  if (nv < 0 || nf < 0) return fail(WN_ERR_INVALID_ARGUMENT, "negative count");
  if (nv > INT32_MAX - 2 || nf > INT32_MAX - 2) return fail(WN_ERR_INVALID_ARGUMENT, "mesh too large");
  if ((nv > 0 && !V) || (nf > 0 && !F)) return fail(WN_ERR_INVALID_ARGUMENT, "NULL mesh pointer");
  if (nf > 0 && nv == 0) return fail(WN_ERR_INVALID_ARGUMENT, "faces without vertices");
  double d[3], R[9];
  if (!make_rotation(dir, d, R)) return fail(WN_ERR_INVALID_ARGUMENT, "dir must be finite and nonzero");
  hipStream_t s = as_stream(stream);

  wn_bvh* h = new wn_bvh();
  std::memcpy(h->dir, d, sizeof d);
  h->nv = (int32_t)nv;
  h->nf = (int32_t)nf;

  // every temporary of the build in one allocation, the BVH's arrays in another
  const int64_t nint = nf > 1 ? nf - 1 : 0;
  wn::BuildBufs b{};
  unsigned* dbb = nullptr;
  Carve tc;
  tc.add(&dbb, 6);
  tc.add(&b.Vr, (size_t)nv);
  tc.add(&b.box, (size_t)nf);
  tc.add(&b.zmax, (size_t)nf);
  tc.add(&b.cen, (size_t)nf);
  tc.add(&b.cbounds, 4);
  tc.add(&b.keys, (size_t)nf);
  tc.add(&b.vals, (size_t)nf);
  tc.add(&b.keys2, (size_t)nf);
  tc.add(&b.vals2, (size_t)nf);
  tc.add((char**)&b.sort_tmp, nf > 1 ? wn::radix_sort_tmp_bytes(nf) : 0);
  tc.add(&b.left, (size_t)nint);
  tc.add(&b.right, (size_t)nint);
  tc.add(&b.parent_int, (size_t)nint);
  tc.add(&b.parent_leaf, (size_t)nf);
  tc.add(&b.ibox, (size_t)nint);
  tc.add(&b.iz, (size_t)nint);
  tc.add(&b.flags, (size_t)nint);
  tc.add(&b.nodes, (size_t)nint);
  void* tmp = nullptr;
  hipError_t e = tc.alloc(&tmp);
  if (e != hipSuccess) { delete h; return hip_fail(e, "hipMalloc"); }
  Carve pc;
  pc.add(&h->tris, (size_t)nf);
  pc.add(&h->nodes, (size_t)nint);
  pc.add(&h->leafbox, (size_t)nf);
  pc.add(&h->leafz, (size_t)nf);
  e = pc.alloc(&h->mem);
  if (e != hipSuccess) { hipFree(tmp); delete h; return hip_fail(e, "hipMalloc"); }
  b.tris = h->tris;
  b.nodes4 = h->nodes;
  b.leafbox = h->leafbox;
  b.leafz = h->leafz;

  // bounding box of V -> centre and power-of-two scale of the frame
  double c[3] = {0, 0, 0};
  double half = 1.0;
  if (nv > 0) {
    unsigned hbb[6];
    const unsigned init[6] = {0xffffffffu, 0u, 0xffffffffu, 0u, 0xffffffffu, 0u};
    e = hipMemcpyAsync(dbb, init, sizeof init, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_bbox_f32, dim3((unsigned)std::min<int64_t>((nv + 255) / 256, 256)), dim3(256), 0, s, V,
                         (int32_t)nv, dbb);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hbb, dbb, sizeof hbb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { hipFree(tmp); wn_free_bvh(h); return hip_fail(e, "bounding box"); }
    double m2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double lo = ord_to_float(hbb[2 * k]), hi = ord_to_float(hbb[2 * k + 1]);
      if (!std::isfinite(lo) || !std::isfinite(hi)) {
        hipFree(tmp);
        wn_free_bvh(h);
        return fail(WN_ERR_INVALID_ARGUMENT, "non-finite vertex");
      }
      c[k] = (double)(float)(0.5 * (lo + hi));
      const double hk = 0.5 * (hi - lo);
      m2 += hk * hk;
    }
    half = std::sqrt(m2);
    if (!(half > 0.0)) half = 1.0;
  }
  const double scale = std::ldexp(1.0, -std::ilogb(half) - 1);   // half*scale in [0.5, 1)
  for (int k = 0; k < 9; ++k) h->F.r[k] = R[k] * scale;
  for (int k = 0; k < 3; ++k) h->F.c[k] = c[k];

  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  // pad: scaled coordinates are O(1); 2^-19 covers float32 rounding of
  // queries and vertices near the mesh with a wide margin
  const float pad = std::ldexp(1.0f, -19);
  if (e == hipSuccess) chk(wn::build_bvh_device(b, h->F, V, (int32_t)nv, F, (int32_t)nf, pad, s));
  if (e == hipSuccess) chk(hipStreamSynchronize(s));
  hipFree(tmp);
  if (e != hipSuccess) {
    wn_free_bvh(h);
    return hip_fail(e, "wn_build_bvh");
  }
  *out = h;
  return WN_OK;
}

wn_status wn_free_bvh(wn_bvh* h) {
  g_err.clear();
  if (!h) return WN_OK;
  if (h->mem) hipFree(h->mem);
  delete h;
  return WN_OK;
}

wn_status wn_bvh_direction(const wn_bvh* h, double dir[3]) {
  g_err.clear();
  if (!h || !dir) return fail(WN_ERR_INVALID_ARGUMENT, "NULL argument");
  std::memcpy(dir, h->dir, sizeof h->dir);
  return WN_OK;
}

static wn_status check_queries(const float* qx, const float* qy, const float* qz, int64_t nq) {
  if (nq < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nq must be >= 0");
  if (nq > 0 && (!qx || !qy || !qz)) return fail(WN_ERR_INVALID_ARGUMENT, "NULL query pointer");
  return WN_OK;
}

static wn::CrossArgs cross_args(const wn_bvh* h, const float* qx, const float* qy, const float* qz,
                                int64_t nq, int32_t* chi) {
  wn::CrossArgs a;
  a.F = h->F;
  a.nodes = h->nodes;
  a.tris = h->tris;
  a.leafbox = h->leafbox;
  a.leafz = h->leafz;
  a.nf = h->nf;
  a.qx = qx;
  a.qy = qy;
  a.qz = qz;
  a.nq = nq;
  a.chi = chi;
  return a;
}

wn_status wn_crossings_3d(const wn_bvh* h, const float* qx, const float* qy, const float* qz,
                          int64_t nq, int32_t* chi_out, void* stream) {
  g_err.clear();
  if (!h) return fail(WN_ERR_INVALID_ARGUMENT, "bvh is NULL");
  wn_status st = check_queries(qx, qy, qz, nq);
  if (st) return st;
  if (nq == 0) return WN_OK;
  if (!chi_out) return fail(WN_ERR_INVALID_ARGUMENT, "chi_out is NULL");
  WN_HIP(wn::launch_cross3d(cross_args(h, qx, qy, qz, nq, chi_out), as_stream(stream)), "crossings");
  return WN_OK;
}

static wn_status eval_boundary(const wn::Frame& F, const float* bnd, const wn::LoopTable& L, int64_t nb,
                               const float* qx, const float* qy, const float* qz, int64_t nq,
                               const int32_t* chi, float* w, hipStream_t s) {
  wn::BndArgs a;
  a.F = F;
  a.bnd = bnd;
  a.nb = (int32_t)nb;
  a.qx = qx;
  a.qy = qy;
  a.qz = qz;
  a.nq = nq;
  a.chi_in = chi;
  a.w_out = w;
  WN_HIP(wn::launch_bnd3d(a, L, s), "boundary integral");
  return WN_OK;
}

wn_status wn_eval_3d(const wn_bvh* h, const float* bnd_xyz, const int64_t* loop_off, int32_t nloops,
                     const float* qx, const float* qy, const float* qz, int64_t nq, float* w_out,
                     int32_t* chi_out, void* stream) {
  g_err.clear();
  if (!h) return fail(WN_ERR_INVALID_ARGUMENT, "bvh is NULL");
  wn::LoopTable L;
  int64_t nb = 0;
  wn_status st = make_loops(loop_off, nloops, 3, &nb, &L);
  if (st) return st;
  if (nb > 0 && !bnd_xyz) return fail(WN_ERR_INVALID_ARGUMENT, "bnd_xyz is NULL");
  if ((st = check_queries(qx, qy, qz, nq))) return st;
  if (nq == 0) return WN_OK;
  if (!w_out) return fail(WN_ERR_INVALID_ARGUMENT, "w_out is NULL");
  int32_t* owned = nullptr;
  if ((st = wn::host::upload_loops(loop_off, &L, as_stream(stream), &owned))) return st;
  // one fused kernel: traversal, boundary walk and combine per query
  wn::BndArgs a;
  a.F = h->F;
  a.bnd = bnd_xyz;
  a.nb = (int32_t)nb;
  a.qx = qx;
  a.qy = qy;
  a.qz = qz;
  a.nq = nq;
  a.chi_in = nullptr;
  a.w_out = w_out;
  const hipError_t e = wn::launch_fwd3d(cross_args(h, qx, qy, qz, nq, chi_out), a, L, chi_out, as_stream(stream));
  if (owned) hipFreeAsync(owned, as_stream(stream));
  WN_HIP(e, "forward");
  return WN_OK;
}

wn_status wn_eval_3d_curves(const wn_bvh* h, const float* ctrl, int64_t ncurves, const float* qx, const float* qy,
                            const float* qz, int64_t nq, const int32_t* chi_in, float* w_out, int32_t* chi_out,
                            void* stream) {
  g_err.clear();
  if (!h) return fail(WN_ERR_INVALID_ARGUMENT, "bvh is NULL");
  if (ncurves < 0) return fail(WN_ERR_INVALID_ARGUMENT, "ncurves must be >= 0");
  if (ncurves > INT32_MAX / 12) return fail(WN_ERR_UNSUPPORTED, "too many curves");
  if (ncurves > 0 && !ctrl) return fail(WN_ERR_INVALID_ARGUMENT, "ctrl is NULL");
  wn_status st = check_queries(qx, qy, qz, nq);
  if (st) return st;
  if (nq == 0) return WN_OK;
  if (!w_out) return fail(WN_ERR_INVALID_ARGUMENT, "w_out is NULL");
  hipStream_t s = as_stream(stream);
  if (chi_in && nq >= wn::kSortQueriesMin && nq <= INT32_MAX && ncurves > 0) {
    // the boundary term alone: run on a coarse Morton-ordered copy (chi_in
    // travels with the queries as 32-bit words) and scatter w back
    wn::SortedQueries sq;
    WN_HIP(wn::sort_queries(qx, qy, qz, reinterpret_cast<const float*>(chi_in), nq, chi_out ? 2 : 1, s, &sq),
           "query order");
    float* w = (float*)sq.out_block(0);
    int32_t* chi = chi_out ? (int32_t*)sq.out_block(1) : nullptr;
    WN_HIP(wn::launch_curves3d(cross_args(h, sq.x, sq.y, sq.z, nq, chi), ctrl, ncurves,
                               reinterpret_cast<const int32_t*>(sq.g), w, chi, s),
           "wn_eval_3d_curves");
    WN_HIP(wn::scatter_rows(w, sq.order, nq, 1, w_out, s), "wn_eval_3d_curves");
    if (chi_out) WN_HIP(wn::scatter_rows(chi, sq.order, nq, 1, chi_out, s), "wn_eval_3d_curves");
    return WN_OK;
  }
  WN_HIP(wn::launch_curves3d(cross_args(h, qx, qy, qz, nq, chi_out), ctrl, ncurves, chi_in, w_out, chi_out, s),
         "wn_eval_3d_curves");
  return WN_OK;
}

wn_status wn_backward_curves(const float* ctrl, int64_t ncurves, const float* qx, const float* qy, const float* qz,
                             int64_t nq, const float* grad_w, float* grad_q, float* grad_ctrl, void* stream) {
  g_err.clear();
  if (ncurves < 0) return fail(WN_ERR_INVALID_ARGUMENT, "ncurves must be >= 0");
  if (ncurves > INT32_MAX / 12) return fail(WN_ERR_UNSUPPORTED, "too many curves");
  if (ncurves > 0 && !ctrl) return fail(WN_ERR_INVALID_ARGUMENT, "ctrl is NULL");
  wn_status st = check_queries(qx, qy, qz, nq);
  if (st) return st;
  if (nq > 0 && !grad_w) return fail(WN_ERR_INVALID_ARGUMENT, "grad_w is NULL");
  if (!grad_q && !grad_ctrl) return WN_OK;
  hipStream_t s = as_stream(stream);
  if (nq >= wn::kSortQueriesMin && nq <= INT32_MAX && ncurves > 0) {
    // neighbouring lanes then refine the same panels: run on sorted copies
    // and scatter grad_q back (the workspace is freed on the stream on return)
    wn::SortedQueries sq;
    WN_HIP(wn::sort_queries(qx, qy, qz, grad_w, nq, grad_q ? 3 : 0, s, &sq), "query order");
    float* gq = grad_q ? (float*)sq.out_block(0) : nullptr;
    WN_HIP(wn::backward_curves(ctrl, ncurves, sq.x, sq.y, sq.z, nq, sq.g, gq, grad_ctrl, s), "wn_backward_curves");
    if (grad_q) WN_HIP(wn::scatter_rows(gq, sq.order, nq, 3, grad_q, s), "wn_backward_curves");
    return WN_OK;
  }
  WN_HIP(wn::backward_curves(ctrl, ncurves, qx, qy, qz, nq, grad_w, grad_q, grad_ctrl, s), "wn_backward_curves");
  return WN_OK;
}

wn_status wn_eval_3d_patches(const double dir[3], const float* nets, int64_t npatch, const float* curves,
                             int64_t ncurves, const float* qx, const float* qy, const float* qz, int64_t nq,
                             float* w_out, int32_t* chi_out, void* stream) {
  g_err.clear();
  double d[3], R[9];
  if (!make_rotation(dir, d, R)) return fail(WN_ERR_INVALID_ARGUMENT, "dir must be finite and nonzero");
  if (npatch < 0 || ncurves < 0) return fail(WN_ERR_INVALID_ARGUMENT, "negative patch or curve count");
  if (npatch > INT32_MAX / 48 || ncurves > INT32_MAX / 12) return fail(WN_ERR_UNSUPPORTED, "too many patches or curves");
  if (npatch > 0 && !nets) return fail(WN_ERR_INVALID_ARGUMENT, "nets is NULL");
  if (ncurves > 0 && !curves) return fail(WN_ERR_INVALID_ARGUMENT, "curves is NULL");
  wn_status st = check_queries(qx, qy, qz, nq);
  if (st) return st;
  if (nq == 0) return WN_OK;
  if (!w_out && !chi_out) return fail(WN_ERR_INVALID_ARGUMENT, "w_out and chi_out are both NULL");
  wn::Frame F;
  for (int k = 0; k < 9; ++k) F.r[k] = R[k];
  for (int k = 0; k < 3; ++k) F.c[k] = 0.0;
  hipStream_t s = as_stream(stream);
  if (w_out && nq >= wn::kSortQueriesMin && nq <= INT32_MAX && npatch + ncurves > 0) {
    // neighbouring lanes then walk the same sub-squares and panels: run on
    // sorted copies and scatter the results back (every result depends on
    // its query alone, so the values are the same bits)
    wn::SortedQueries sq;
    WN_HIP(wn::sort_queries(qx, qy, qz, nullptr, nq, chi_out ? 2 : 1, s, &sq), "query order");
    float* w = (float*)sq.out_block(0);
    int32_t* chi = chi_out ? (int32_t*)sq.out_block(1) : nullptr;
    WN_HIP(wn::launch_psurf_single(F, nets, npatch, curves, ncurves, sq.x, sq.y, sq.z, nq, w, chi, s),
           "wn_eval_3d_patches");
    WN_HIP(wn::scatter_rows(w, sq.order, nq, 1, w_out, s), "wn_eval_3d_patches");
    if (chi_out) WN_HIP(wn::scatter_rows(chi, sq.order, nq, 1, chi_out, s), "wn_eval_3d_patches");
    return WN_OK;
  }
  // w: crossings and curve term in one launch (no temporary chi buffer);
  // crossings only: the crossing kernel alone
  const hipError_t e = w_out ? wn::launch_psurf_single(F, nets, npatch, curves, ncurves, qx, qy, qz, nq, w_out,
                                                       chi_out, s)
                             : wn::launch_patches3d(F, nets, npatch, qx, qy, qz, nq, chi_out, s);
  if (e != hipSuccess) return hip_fail(e, "wn_eval_3d_patches");
  return WN_OK;
}

struct wn_patch_batch {
  wn::PBatch b;
};

wn_status wn_patch_batch_create(const wn_patch_surface* surfs, int32_t nsurf, void* stream, wn_patch_batch** out) {
  g_err.clear();
  if (!out) return fail(WN_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (nsurf < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nsurf must be >= 0");
  if (nsurf > 0 && !surfs) return fail(WN_ERR_INVALID_ARGUMENT, "surfs is NULL");
  std::vector<wn::PSurf> d((size_t)nsurf);
  int64_t patches = 0, curves = 0, blocks = 0;
  for (int32_t k = 0; k < nsurf; ++k) {
    const wn_patch_surface& c = surfs[k];
    if (c.npatch < 0 || c.ncurves < 0 || c.nq < 0) return fail(WN_ERR_INVALID_ARGUMENT, "surface %d: negative count", k);
    double dn[3], R[9];
    if (!make_rotation(c.dir, dn, R))
      return fail(WN_ERR_INVALID_ARGUMENT, "surface %d: dir must be finite and nonzero", k);
    if (c.npatch > INT32_MAX / 48 || c.ncurves > INT32_MAX / 12)
      return fail(WN_ERR_UNSUPPORTED, "surface %d: too many patches or curves", k);
    patches += c.npatch;
    curves += c.ncurves;
    blocks += (c.nq + 255) / 256;
    if (patches > INT64_MAX / 256 || curves > INT64_MAX / 256 || blocks > INT32_MAX)
      return fail(WN_ERR_UNSUPPORTED, "batch too large for one launch (split it)");
    wn::PSurf& p = d[(size_t)k];
    for (int j = 0; j < 9; ++j) p.F.r[j] = R[j];
    for (int j = 0; j < 3; ++j) p.F.c[j] = 0.0;
    p.nq = c.nq;
    p.npatch = (int32_t)c.npatch;
    p.ncurve = (int32_t)c.ncurves;
  }
  wn_patch_batch* h = new (std::nothrow) wn_patch_batch();
  if (!h) return fail(WN_ERR_OUT_OF_MEMORY, "host allocation");
  const hipError_t e = wn::pbatch_create(d.data(), nsurf, as_stream(stream), &h->b);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "wn_patch_batch_create");
  }
  *out = h;
  return WN_OK;
}

wn_status wn_patch_batch_free(wn_patch_batch* batch) {
  g_err.clear();
  delete batch;
  return WN_OK;
}

wn_status wn_eval_3d_patches_batched(const wn_patch_batch* batch, const float* nets, const float* curves,
                                     const float* qx, const float* qy, const float* qz, float* w_out,
                                     int32_t* chi_out, void* stream) {
  g_err.clear();
  if (!batch) return fail(WN_ERR_INVALID_ARGUMENT, "batch is NULL");
  const wn::PBatch& b = batch->b;
  if (b.nq == 0) return WN_OK;
  if (b.npatch > 0 && !nets) return fail(WN_ERR_INVALID_ARGUMENT, "nets is NULL");
  if (b.ncurve > 0 && w_out && !curves) return fail(WN_ERR_INVALID_ARGUMENT, "curves is NULL");
  if (!qx || !qy || !qz) return fail(WN_ERR_INVALID_ARGUMENT, "NULL query pointer");
  if (!w_out && !chi_out) return fail(WN_ERR_INVALID_ARGUMENT, "w_out and chi_out are both NULL");
  WN_HIP(wn::eval_pbatch(b, nets, curves, qx, qy, qz, w_out, chi_out, as_stream(stream)),
         "wn_eval_3d_patches_batched");
  return WN_OK;
}

wn_status wn_diagnose(const float* qx, const float* qy, const float* qz, const int32_t* chi, int64_t nq,
                      int64_t* counts_out, void* stream) {
  g_err.clear();
  wn_status st = check_queries(qx, qy, qz, nq);
  if (st) return st;
  if (!counts_out) return fail(WN_ERR_INVALID_ARGUMENT, "counts_out is NULL");
  if (nq > 0 && !chi) return fail(WN_ERR_INVALID_ARGUMENT, "chi is NULL");
  WN_HIP(wn::diagnose(qx, qy, qz, chi, nq, counts_out, as_stream(stream)), "wn_diagnose");
  return WN_OK;
}

wn_status wn_device_info(int32_t* cu_count, int32_t* clock_khz) {
  g_err.clear();
  if (!cu_count || !clock_khz) return fail(WN_ERR_INVALID_ARGUMENT, "NULL output");
  int dev = 0, cus = 0, clk = 0;
  WN_HIP(hipGetDevice(&dev), "hipGetDevice");
  WN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  WN_HIP(hipDeviceGetAttribute(&clk, hipDeviceAttributeClockRate, dev), "hipDeviceGetAttribute");
  *cu_count = cus;
  *clock_khz = clk;
  return WN_OK;
}

wn_status wn_spatial_order(const float* qx, const float* qy, const float* qz, int64_t nq, int32_t* order_out,
                           void* stream) {
  g_err.clear();
  wn_status st = check_queries(qx, qy, qz, nq);
  if (st) return st;
  if (nq > INT32_MAX) return fail(WN_ERR_UNSUPPORTED, "nq must be <= INT32_MAX");
  if (nq == 0) return WN_OK;
  if (!order_out) return fail(WN_ERR_INVALID_ARGUMENT, "order_out is NULL");
  WN_HIP(wn::spatial_order(qx, qy, qz, nq, order_out, as_stream(stream)), "wn_spatial_order");
  return WN_OK;
}

wn_status wn_eval_3d_grid(const wn_bvh* h, const float* bnd_xyz, const int64_t* loop_off, int32_t nloops,
                          const float* gx, const float* gy, const float* gz, int64_t nx, int64_t ny, int64_t nz,
                          float* w_out, int32_t* chi_out, void* stream) {
  g_err.clear();
  if (!h) return fail(WN_ERR_INVALID_ARGUMENT, "bvh is NULL");
  if (!(h->dir[0] == 0.0 && h->dir[1] == 0.0 && h->dir[2] > 0.0))
    return fail(WN_ERR_UNSUPPORTED, "grid mode needs a BVH built for the direction +z");
  wn::LoopTable L;
  int64_t nb = 0;
  wn_status st = make_loops(loop_off, nloops, 3, &nb, &L);
  if (st) return st;
  if (nb > 0 && !bnd_xyz) return fail(WN_ERR_INVALID_ARGUMENT, "bnd_xyz is NULL");
  if (nx < 0 || ny < 0 || nz < 0) return fail(WN_ERR_INVALID_ARGUMENT, "negative grid size");
  if (nx == 0 || ny == 0 || nz == 0) return WN_OK;
  if (nx > (int64_t)UINT32_MAX || ny > (int64_t)UINT32_MAX / nx || nz > (int64_t)UINT32_MAX / (nx * ny))
    return fail(WN_ERR_INVALID_ARGUMENT, "grid of 2^32 points or more");
  if (!gx || !gy || !gz || !w_out) return fail(WN_ERR_INVALID_ARGUMENT, "NULL grid axis or output pointer");
  const int64_t nq = nx * ny * nz;
  hipStream_t s = as_stream(stream);
  int32_t* owned = nullptr;
  if ((st = wn::host::upload_loops(loop_off, &L, s, &owned))) return st;
  wn::CrossArgs ca = cross_args(h, nullptr, nullptr, nullptr, 0, nullptr);
  wn::BndArgs a;
  a.F = h->F;
  a.bnd = bnd_xyz;
  a.nb = (int32_t)nb;
  a.qx = a.qy = a.qz = nullptr;
  a.nq = nq;
  a.chi_in = nullptr;
  a.w_out = w_out;
  const hipError_t e = wn::launch_grid3d_fwd(ca, a, L, gx, gy, gz, nx, ny, nz, chi_out, s);
  if (owned) hipFreeAsync(owned, s);
  WN_HIP(e, "grid forward");
  return WN_OK;
}

wn_status wn_eval_3d_boundary(const wn_bvh* h, const float* bnd_xyz, const int64_t* loop_off,
                              int32_t nloops, const float* qx, const float* qy, const float* qz,
                              int64_t nq, const int32_t* chi_in, float* w_out, void* stream) {
  g_err.clear();
  if (!h) return fail(WN_ERR_INVALID_ARGUMENT, "bvh is NULL");
  wn::LoopTable L;
  int64_t nb = 0;
  wn_status st = make_loops(loop_off, nloops, 3, &nb, &L);
  if (st) return st;
  if (nb > 0 && !bnd_xyz) return fail(WN_ERR_INVALID_ARGUMENT, "bnd_xyz is NULL");
  if ((st = check_queries(qx, qy, qz, nq))) return st;
  if (nq == 0) return WN_OK;
  if (!w_out || !chi_in) return fail(WN_ERR_INVALID_ARGUMENT, "w_out or chi_in is NULL");
  int32_t* owned = nullptr;
  if ((st = wn::host::upload_loops(loop_off, &L, as_stream(stream), &owned))) return st;
  st = eval_boundary(h->F, bnd_xyz, L, nb, qx, qy, qz, nq, chi_in, w_out, as_stream(stream));
  if (owned) hipFreeAsync(owned, as_stream(stream));
  return st;
}

wn_status wn_backward(const float* bnd_xyz, const int64_t* loop_off, int32_t nloops, const float* qx,
                      const float* qy, const float* qz, int64_t nq, const float* grad_w, float* grad_q,
                      float* grad_bnd, void* stream) {
  g_err.clear();
  wn::LoopTable L;
  int64_t nb = 0;
  wn_status st = wn::host::check_backward(bnd_xyz, loop_off, nloops, qx, qy, qz, nq, grad_w, &L, &nb);
  if (st) return st;
  hipStream_t s = as_stream(stream);
  int32_t* owned = nullptr;
  if ((st = wn::host::upload_loops(loop_off, &L, s, &owned))) return st;
  const wn::host::AdjPlan P = wn::host::plan_backward(nq, nb, nloops, grad_q != nullptr, grad_bnd != nullptr);
  // the workspace arrays in one block on the stream, freed on the stream
  // after the launches
  const size_t bytes = wn::host::plan_bytes(P);
  void* base = nullptr;
  hipError_t e = bytes ? hipMallocAsync(&base, bytes, s) : hipSuccess;
  if (e == hipSuccess) {
    const wn::host::AdjWork W = wn::host::carve_backward(P, base);
    st = wn::host::run_backward(P, bnd_xyz, L, nb, qx, qy, qz, nq, grad_w, grad_q, grad_bnd, W, s);
  }
  if (base) hipFreeAsync(base, s);
  if (owned) hipFreeAsync(owned, s);
  if (e != hipSuccess) return hip_fail(e, "backward workspace");
  return st;
}

// Checks shared by the 2D entry points (curves, loop table, query layout).
static wn_status check_2d(wn_dtype dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                          const uint8_t* loop_closed, int32_t nloops, int32_t kind, int64_t nx, int64_t ny) {
  if (dtype != WN_F32 && dtype != WN_F64) return fail(WN_ERR_UNSUPPORTED, "dtype must be WN_F32 or WN_F64");
  if (kind != 0 && kind != 1) return fail(WN_ERR_INVALID_ARGUMENT, "kind must be 0 (points) or 1 (grid)");
  if (nseg < 0 || nx < 0 || (kind == 1 && ny < 0)) return fail(WN_ERR_INVALID_ARGUMENT, "negative count");
  if (nseg > (INT32_MAX - 3) / 3) return fail(WN_ERR_UNSUPPORTED, "too many segments");
  if (nseg > 0 && !ctrl) return fail(WN_ERR_INVALID_ARGUMENT, "ctrl is NULL");
  if (nloops < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nloops must be >= 0");
  if (nloops > WN_MAX_LOOPS) return fail(WN_ERR_UNSUPPORTED, "at most %d loops per call", WN_MAX_LOOPS);
  if (nloops > 0 && (!loop_off || !loop_closed)) return fail(WN_ERR_INVALID_ARGUMENT, "loop table is NULL");
  if (nloops > 0) {
    if (loop_off[0] != 0) return fail(WN_ERR_INVALID_ARGUMENT, "loop_off[0] must be 0");
    for (int32_t l = 0; l < nloops; ++l)
      if (loop_off[l + 1] <= loop_off[l]) return fail(WN_ERR_INVALID_ARGUMENT, "loop %d is empty or reversed", l);
    if (loop_off[nloops] != nseg) return fail(WN_ERR_INVALID_ARGUMENT, "loop_off[nloops] must equal nseg");
  } else if (nseg > 0) {
    return fail(WN_ERR_INVALID_ARGUMENT, "segments without loops");
  }
  return WN_OK;
}

wn_status wn_backward_2d(wn_dtype dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                         const uint8_t* loop_closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                         int64_t nx, int64_t ny, const void* grad_w, void* grad_q, void* grad_ctrl, void* stream) {
  g_err.clear();
  wn_status st = check_2d(dtype, ctrl, nseg, loop_off, loop_closed, nloops, kind, nx, ny);
  if (st) return st;
  if (kind == 1 && nx > 0 && ny > INT64_MAX / nx) return fail(WN_ERR_INVALID_ARGUMENT, "grid too large");
  const int64_t n = kind == 0 ? nx : nx * ny;
  if (n > 0 && (!x || !y || !grad_w)) return fail(WN_ERR_INVALID_ARGUMENT, "query coordinates or grad_w are NULL");
  if (!grad_q && !grad_ctrl) return WN_OK;
  int64_t lo_local[1] = {0};
  uint8_t cl_local[1] = {0};
  WN_HIP(wn::backward_2d(dtype, ctrl, nseg, nloops ? loop_off : lo_local, nloops ? loop_closed : cl_local, nloops,
                         kind, x, y, nx, ny, grad_w, grad_q, grad_ctrl, as_stream(stream)),
         "wn_backward_2d");
  return WN_OK;
}

wn_status wn_eval_2d(wn_dtype dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                     const uint8_t* loop_closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                     int64_t nx, int64_t ny, void* w_out, int32_t* chi_out, void* stream) {
  g_err.clear();
  if (dtype != WN_F32 && dtype != WN_F64) return fail(WN_ERR_UNSUPPORTED, "dtype must be WN_F32 or WN_F64");
  if (kind != 0 && kind != 1) return fail(WN_ERR_INVALID_ARGUMENT, "kind must be 0 (points) or 1 (grid)");
  if (nseg < 0 || nx < 0 || (kind == 1 && ny < 0)) return fail(WN_ERR_INVALID_ARGUMENT, "negative count");
  if (nseg > (INT32_MAX - 3) / 3) return fail(WN_ERR_UNSUPPORTED, "too many segments");
  if (nseg > 0 && !ctrl) return fail(WN_ERR_INVALID_ARGUMENT, "ctrl is NULL");
  if (nloops < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nloops must be >= 0");
  if (nloops > 0 && (!loop_off || !loop_closed)) return fail(WN_ERR_INVALID_ARGUMENT, "loop table is NULL");
  if (nloops > 0) {
    if (loop_off[0] != 0) return fail(WN_ERR_INVALID_ARGUMENT, "loop_off[0] must be 0");
    for (int32_t l = 0; l < nloops; ++l)
      if (loop_off[l + 1] <= loop_off[l]) return fail(WN_ERR_INVALID_ARGUMENT, "loop %d is empty or reversed", l);
    if (loop_off[nloops] != nseg) return fail(WN_ERR_INVALID_ARGUMENT, "loop_off[nloops] must equal nseg");
  } else if (nseg > 0) {
    return fail(WN_ERR_INVALID_ARGUMENT, "segments without loops");
  }
  const int64_t nout = kind == 0 ? nx : nx * ny;
  if (nout == 0) return WN_OK;
  if (!x || !y) return fail(WN_ERR_INVALID_ARGUMENT, "query coordinates are NULL");
  if (!w_out) return fail(WN_ERR_INVALID_ARGUMENT, "w_out is NULL");
  if (kind == 1 && ny > 65535) return fail(WN_ERR_UNSUPPORTED, "at most 65535 grid rows per call");
  int64_t lo_local[1] = {0};
  uint8_t cl_local[1] = {0};
  WN_HIP(wn::eval_2d(dtype, ctrl, nseg, nloops ? loop_off : lo_local, nloops ? loop_closed : cl_local, nloops,
                     kind, x, y, nx, ny, w_out, chi_out, as_stream(stream)),
         "wn_eval_2d");
  return WN_OK;
}

struct wn_batch2d {
  wn::Batch2D b;
};

wn_status wn_batch2d_create(wn_dtype dtype, const wn_curveset_2d* sets, int32_t nsets, void* stream,
                            wn_batch2d** out) {
  g_err.clear();
  if (!out) return fail(WN_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (dtype != WN_F32 && dtype != WN_F64) return fail(WN_ERR_UNSUPPORTED, "dtype must be WN_F32 or WN_F64");
  if (nsets < 0) return fail(WN_ERR_INVALID_ARGUMENT, "nsets must be >= 0");
  if (nsets > 0 && !sets) return fail(WN_ERR_INVALID_ARGUMENT, "sets is NULL");
  int64_t seg = 0, items_g = 0, items_w = 0, loops = 0;
  for (int32_t k = 0; k < nsets; ++k) {
    const wn_curveset_2d& c = sets[k];
    if (c.nseg < 0 || c.nx < 0 || c.ny < 0 || c.nloops < 0)
      return fail(WN_ERR_INVALID_ARGUMENT, "set %d: negative count", k);
    if (c.nx > INT32_MAX || c.ny > INT32_MAX) return fail(WN_ERR_UNSUPPORTED, "set %d: grid side over 2^31 - 1", k);
    if (c.nloops > 0 && (!c.loop_off || !c.loop_closed))
      return fail(WN_ERR_INVALID_ARGUMENT, "set %d: loop table is NULL", k);
    if (c.nloops > 0) {
      if (c.loop_off[0] != 0) return fail(WN_ERR_INVALID_ARGUMENT, "set %d: loop_off[0] must be 0", k);
      for (int32_t l = 0; l < c.nloops; ++l)
        if (c.loop_off[l + 1] <= c.loop_off[l])
          return fail(WN_ERR_INVALID_ARGUMENT, "set %d: loop %d is empty or reversed", k, l);
      if (c.loop_off[c.nloops] != c.nseg)
        return fail(WN_ERR_INVALID_ARGUMENT, "set %d: loop_off[nloops] must equal nseg", k);
    } else if (c.nseg > 0) {
      return fail(WN_ERR_INVALID_ARGUMENT, "set %d: segments without loops", k);
    }
    if (c.nx > 0 && c.ny > INT64_MAX / c.nx) return fail(WN_ERR_INVALID_ARGUMENT, "set %d: grid too large", k);
    seg += c.nseg;
    loops += c.nloops + 1;
    if (seg > (INT32_MAX - 3) / 3 || loops > INT32_MAX / 2)
      return fail(WN_ERR_UNSUPPORTED, "too many segments or loops");
    if (3 * c.nseg <= wn::kRowPieces2D)
      items_w += (c.nx + wn::kRowColTile2D - 1) / wn::kRowColTile2D * c.ny;
    else
      items_g += (c.nx + wn::kGridColTile2D - 1) / wn::kGridColTile2D * c.ny;
    if (items_g > wn::kMaxItemsG2D || items_w > wn::kMaxItemsW2D)
      return fail(WN_ERR_UNSUPPORTED, "batch too large for one launch (split it)");
  }
  wn_batch2d* h = new (std::nothrow) wn_batch2d();
  if (!h) return fail(WN_ERR_OUT_OF_MEMORY, "host allocation");
  const hipError_t e = wn::batch2d_create(dtype, sets, nsets, as_stream(stream), &h->b);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "wn_batch2d_create");
  }
  *out = h;
  return WN_OK;
}

wn_status wn_batch2d_free(wn_batch2d* batch) {
  g_err.clear();
  delete batch;
  return WN_OK;
}

wn_status wn_eval_2d_batched(const wn_batch2d* batch, const void* ctrl, const void* x, const void* y, void* w_out,
                             int32_t* chi_out, void* stream) {
  g_err.clear();
  if (!batch) return fail(WN_ERR_INVALID_ARGUMENT, "batch is NULL");
  const wn::Batch2D& b = batch->b;
  if (b.nseg > 0 && !ctrl) return fail(WN_ERR_INVALID_ARGUMENT, "ctrl is NULL");
  if (b.nout == 0) return WN_OK;
  if (!x || !y) return fail(WN_ERR_INVALID_ARGUMENT, "query coordinates are NULL");
  if (!w_out) return fail(WN_ERR_INVALID_ARGUMENT, "w_out is NULL");
  WN_HIP(wn::eval_2d_batched(b, ctrl, x, y, w_out, chi_out, as_stream(stream)), "wn_eval_2d_batched");
  return WN_OK;
}

}  // extern "C"
