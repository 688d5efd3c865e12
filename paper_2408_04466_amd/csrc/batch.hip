// Many surfaces of uneven size, each with its own queries, evaluated in one
// persistent launch (forward: crossing count + boundary integral fused per
// work item; backward: the adjoint), captured in a hipGraph and replayed.
//
// Work list: every surface's queries are cut into tiles; an item is one
// (surface, tile).  Items are sorted by decreasing estimated cost
// (tile size x (boundary edges + a crossing-count allowance)), the
// longest-processing-time-first order, and a fixed grid of workgroups pulls
// them from an atomic counter until the list is exhausted, so a few large
// surfaces cannot leave most compute units idle at the end.  The forward
// runs either fused (one kernel: traversal, then boundary walk, per query)
// or split (a persistent crossing kernel, then a persistent boundary kernel,
// each at its own register footprint).  Mode, tile size and workgroups per
// compute unit come from a small autotuner that times candidates on the
// first evaluation (optionally cached in a JSON file).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "adjloop.hpp"
#include "bndloop.hpp"
#include "bvh_build.hpp"
#include "host.hpp"
#include "traverse.hpp"

namespace wn {

namespace {

struct SurfDesc {
  Frame F;
  const BvhNode4* nodes;
  const TriRec* tris;
  const float4* leafbox;
  const float* leafz;
  int32_t nf;
  int32_t nb;
  int64_t bnd_off;     // first vertex of this surface in the boundary arena
  int32_t loop_off;    // first entry of its loop table
  int32_t nloops;
  int64_t q_off;       // first query
  int64_t nq;
  int64_t pv_off;      // backward: first float of its vertex partials
  int64_t pl_off;      // backward: first float of its loop partials
  int32_t tiles_bwd;   // backward tiles of this surface
  int32_t groups;      // backward: groups of kRowsPerGroup partial rows
  int64_t tmp_off;     // backward: first double of its group sums
};

// One workgroup of the first reduction stage: columns [col0, col0 + 256) of
// row group `group` of surface `surf`.
struct RBlock {
  int32_t surf;
  int32_t group;
  int32_t col0;
  int32_t pad;
};

constexpr int kRowsPerGroup = 16;

struct Item {
  int32_t surf;
  int32_t cnt;
  int64_t q0;
  int32_t tile;        // tile index within the surface (backward partial slot)
  int32_t pad;
};

struct FwdArgs {
  const SurfDesc* descs;
  const Item* items;
  int32_t n_items;
  int32_t direct;          // 1: one workgroup per item (item = blockIdx.x, no counter)
  int32_t* counter;        // [0]: fused or crossing kernel, [1]: boundary kernel
  int32_t* chi_buf;        // split mode: crossing counts (chi_out or a batch buffer)
  const RPt* bndr;         // rotated boundary arena (bnd::stage_vertex of every vertex)
  const int32_t* loops;
  const float* qx;
  const float* qy;
  const float* qz;
  float* w;
  int32_t* chi;
};

struct BwdArgs {
  const SurfDesc* descs;
  const Item* items;
  int32_t n_items;
  int32_t* counter;
  const float* bnd;
  const int32_t* loops;
  const float* qx;
  const float* qy;
  const float* qz;
  const float* gw;
  float* gq;
  float* pv;
  float* pl;
};

constexpr int kThreads = 256;

__global__ void k_reset(int32_t* counter) {
  if (threadIdx.x < 2) counter[threadIdx.x] = 0;
}

// Item lists and surface descriptors are written by the host before any
// launch and only read by the kernels, so they are read through the
// constant address space: with a wave-uniform index the compiler then uses
// scalar loads and keeps the descriptor (frame, pointers, counts) in scalar
// registers.
template <class T>
__device__ __forceinline__ T load_const(const T* p, int64_t i) {
  static_assert(sizeof(T) % 4 == 0, "word-sized records only");
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)(p + i);
  T out;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
  return out;
}

// Pull the next item index (uniform across the workgroup).  readfirstlane
// tells the compiler so: the item and its surface descriptor are then read
// with scalar loads into scalar registers instead of occupying vector
// registers in every lane.
__device__ __forceinline__ int next_item(int32_t* counter, int* s_item) {
  __syncthreads();
  if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*s_item);
}

// Item for this pass of the persistent loop: from the counter, or in direct
// mode blockIdx.x on the first pass and none after it.
__device__ __forceinline__ int item_for(int direct, int pass, int n_items, int32_t* counter, int* s_item) {
  if (direct) return pass == 0 ? (int)blockIdx.x : n_items;
  return next_item(counter, s_item);
}

__device__ __forceinline__ CrossArgs cross_args(const SurfDesc& D) {
  CrossArgs ca;
  ca.F = D.F;
  ca.nodes = D.nodes;
  ca.tris = D.tris;
  ca.leafbox = D.leafbox;
  ca.leafz = D.leafz;
  ca.nf = D.nf;
  return ca;
}

// Fused mode: per query, the crossing count and then the boundary walk.
// Eight waves per SIMD (64 registers, no spills; seven measured slower).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_fwd(FwdArgs a) {
  __shared__ RPt sv[bnd::kChunk];
  __shared__ int s_item;
  for (int pass = 0;; ++pass) {
    const int it = item_for(a.direct, pass, a.n_items, a.counter, &s_item);
    if (it >= a.n_items) return;
    const Item item = load_const(a.items, it);
    const SurfDesc D = load_const(a.descs, item.surf);
    const CrossArgs ca = cross_args(D);
    const bnd::DeviceLoops L{a.loops + D.loop_off, D.nloops};
    const bnd::StageCopy stage{a.bndr + D.bnd_off};
    int staged = -1;
    for (int r = 0; r < item.cnt; r += kThreads) {
      const bool ok = r + (int)threadIdx.x < item.cnt;
      const int64_t q = item.q0 + (ok ? r + (int)threadIdx.x : 0);
      const float px = a.qx[q], py = a.qy[q], pz = a.qz[q];
      const bool fin = isfinite(px) && isfinite(py) && isfinite(pz);
      bnd::Lane<1> s;
      {
        double X, Y, Z;
        rotate(D.F, px, py, pz, X, Y, Z);
        s.p[0] = make_qp(X, Y, Z);
      }
      turns_init(s.T[0]);
      bnd::lane_range(s);
      // odd workgroups walk the boundary first: then waves waiting on node
      // fetches and waves issuing boundary arithmetic share every SIMD from
      // the start (each workgroup stays uniform, so its barriers still meet)
      int chi = 0, pend = 0;
      if (blockIdx.x & 1) bnd::boundary_walk(s, stage, D.nb, L, sv, staged, pend);
      if (ok && fin) chi = traverse<kShortStack>(ca, s.p[0]);
      if (!(blockIdx.x & 1)) bnd::boundary_walk(s, stage, D.nb, L, sv, staged, pend);
      bnd::finish_turns(s, pend);
      if (ok) {
        const bool valid = fin && chi != WN_CHI_INVALID;
        a.w[q] = valid ? bnd::lane_w(s, 0, chi) : __int_as_float(0x7fc00000);
        if (a.chi) a.chi[q] = valid ? chi : WN_CHI_INVALID;
      }
    }
  }
}

// Split mode, first kernel: crossing counts into chi_buf (WN_CHI_INVALID
// for a non-finite query or an abandoned traversal).
__global__ __launch_bounds__(kThreads) void k_batch_cross(FwdArgs a) {
  __shared__ int s_item;
  for (int pass = 0;; ++pass) {
    const int it = item_for(a.direct, pass, a.n_items, a.counter, &s_item);
    if (it >= a.n_items) return;
    const Item item = load_const(a.items, it);
    const SurfDesc D = load_const(a.descs, item.surf);
    const CrossArgs ca = cross_args(D);
    for (int r = threadIdx.x; r < item.cnt; r += kThreads) {
      const int64_t q = item.q0 + r;
      const float px = a.qx[q], py = a.qy[q], pz = a.qz[q];
      int chi = WN_CHI_INVALID;
      if (isfinite(px) && isfinite(py) && isfinite(pz)) {
        double X, Y, Z;
        rotate(D.F, px, py, pz, X, Y, Z);
        chi = traverse<kShortStack>(ca, make_qp(X, Y, Z));
      }
      a.chi_buf[q] = chi;
    }
  }
}

// Split mode, second kernel: boundary walk, combined with chi_buf into w.
__global__ __launch_bounds__(kThreads) void k_batch_bnd(FwdArgs a) {
  __shared__ RPt sv[bnd::kChunk];
  __shared__ int s_item;
  for (int pass = 0;; ++pass) {
    const int it = item_for(a.direct, pass, a.n_items, a.counter + 1, &s_item);
    if (it >= a.n_items) return;
    const Item item = load_const(a.items, it);
    const SurfDesc D = load_const(a.descs, item.surf);
    const bnd::DeviceLoops L{a.loops + D.loop_off, D.nloops};
    const bnd::StageCopy stage{a.bndr + D.bnd_off};
    int staged = -1;
    for (int r = 0; r < item.cnt; r += kThreads) {
      const bool ok = r + (int)threadIdx.x < item.cnt;
      const int64_t q = item.q0 + (ok ? r + (int)threadIdx.x : 0);
      bnd::Lane<1> s;
      {
        double X, Y, Z;
        rotate(D.F, a.qx[q], a.qy[q], a.qz[q], X, Y, Z);
        s.p[0] = make_qp(X, Y, Z);
      }
      turns_init(s.T[0]);
      bnd::lane_range(s);
      int pend = 0;
      bnd::boundary_walk(s, stage, D.nb, L, sv, staged, pend);
      bnd::finish_turns(s, pend);
      if (ok) {
        const int chi = a.chi_buf[q];
        a.w[q] = chi != WN_CHI_INVALID ? bnd::lane_w(s, 0, chi) : __int_as_float(0x7fc00000);
      }
    }
  }
}

// Four waves per SIMD (128 registers): the few spills are per-item
// addresses, outside the walk.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_bwd(BwdArgs a) {
  __shared__ adj::AdjLds lds;
  __shared__ int s_item;
  for (int pass = 0;; ++pass) {
    const int it = item_for(1, pass, a.n_items, a.counter, &s_item);
    if (it >= a.n_items) return;
    const Item item = load_const(a.items, it);
    const SurfDesc D = load_const(a.descs, item.surf);
    const bnd::DeviceLoops L{a.loops + D.loop_off, D.nloops};
    const int64_t row = item.tile;   // partial row
    float* pv = a.pv ? a.pv + D.pv_off + row * (int64_t)D.nb * 3 : nullptr;
    float* pl = a.pv ? a.pl + D.pl_off + row * (int64_t)D.nloops * 3 : nullptr;
    adj::QState S[adj::kQPL];
    adj::load_tile<adj::kQPL>(S, a.qx, a.qy, a.qz, a.gw, item.q0, item.cnt);
    if (D.nb > 0) adj::walk<adj::kQPL>(S, a.bnd + 3 * D.bnd_off, D.nb, L, lds, pv, pl);
    adj::store_gq<adj::kQPL>(S, item.q0, item.cnt, a.gq);
  }
}

// Boundary-vertex gradients from the per-tile partial rows, in
// two fixed-order float64 stages (the same grouping as the single-surface
// adjoint, so both give identical bits).  Stage 1: one group of
// kRowsPerGroup rows per column, plus the per-loop closing share at a loop's
// first vertex.
__global__ void k_batch_rows(const SurfDesc* __restrict__ descs, const RBlock* __restrict__ blocks,
                             const int32_t* __restrict__ loops, const float* __restrict__ pv,
                             const float* __restrict__ pl, double* __restrict__ tmp) {
  const RBlock rb = blocks[blockIdx.x];
  const SurfDesc D = descs[rb.surf];
  const int64_t n = (int64_t)D.nb * 3;
  const int64_t t = (int64_t)rb.col0 + threadIdx.x;
  if (t >= n) return;
  const int v = (int)(t / 3), c = (int)(t % 3);
  const int32_t* lo = loops + D.loop_off;
  int lf = -1;
  for (int l = 0; l < D.nloops; ++l)
    if (lo[l] == v && lo[l + 1] > v) lf = l;
  const int64_t rows = D.tiles_bwd;
  const int64_t r0 = (int64_t)rb.group * kRowsPerGroup;
  const int64_t r1 = min(rows, r0 + kRowsPerGroup);
  const float* p = pv + D.pv_off;
  const float* q = pl + D.pl_off;
  double s = 0.0;
  if (lf < 0) {
    s = adj::ordered_sum(p + r0 * n + t, n, r1 - r0, 0.0);
  } else {
    for (int64_t r = r0; r < r1; ++r) {
      s += (double)p[r * n + t];
      s += (double)q[(r * D.nloops + lf) * 3 + c];
    }
  }
  tmp[D.tmp_off + (int64_t)rb.group * n + t] = s;
}

// Stage 2: out[3 * (bnd_off + v) + c] = -(1/4pi) * sum over the surface's
// groups, in group order.
__global__ void k_batch_groups(const SurfDesc* __restrict__ descs, const int32_t* __restrict__ surf_of,
                               const double* __restrict__ tmp, int64_t total3, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total3) return;
  const SurfDesc D = descs[surf_of[t / 3]];
  const int64_t n = (int64_t)D.nb * 3;
  const int64_t col = t - 3 * D.bnd_off;
  const double s = adj::ordered_sum(tmp + D.tmp_off + col, n, D.groups, 0.0);
  out[t] = (float)(-s * 0.07957747154594767 + 0.0);
}

// Rotated boundary arena of a batch: vertex gv of the concatenated
// boundaries, staged exactly as the plain kernels stage it.
__global__ void k_rotate_bnd(const SurfDesc* __restrict__ descs, const int32_t* __restrict__ loops,
                             const float* __restrict__ bnd, const int32_t* __restrict__ surf_of, int64_t nb_tot,
                             RPt* __restrict__ out) {
  const int64_t gv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gv >= nb_tot) return;
  const SurfDesc D = descs[surf_of[gv]];
  const bnd::DeviceLoops L{loops + D.loop_off, D.nloops};
  out[gv] = bnd::stage_vertex(D.F, bnd + 3 * D.bnd_off, L, (int)(gv - D.bnd_off));
}

__global__ void k_fill_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

}  // namespace
}  // namespace wn

using wn::host::as_stream;
using wn::host::fail;
using wn::host::hip_fail;

struct wn_batch {
  int32_t ns = 0;
  int dev = 0;
  int cus = 0;
  std::vector<wn_bvh*> bvh;
  std::vector<wn::SurfDesc> desc;     // host copy
  std::vector<int64_t> q_off;         // [ns + 1]
  int64_t total_q = 0, total_b = 0, total_pairs = 0;
  wn::SurfDesc* d_desc = nullptr;
  int32_t* d_loops = nullptr;
  float* d_bnd = nullptr;
  wn::RPt* d_bndr = nullptr;          // rotated boundary arena (forward)
  int32_t* d_surf_of = nullptr;       // boundary vertex -> surface
  int32_t* d_counter = nullptr;
  // forward work list
  wn::Item* d_items = nullptr;
  int32_t n_items = 0;
  int tile = 1024, wgpcu = 4;
  int mode = 0;                       // forward: 0 fused, 1 split
  int mode_fixed = -1;                // $WN_BATCH_MODE: the tuner keeps this mode
  int32_t* d_chi = nullptr;           // split mode without chi_out
  int tune_mode = 0;
  bool tuned = false;
  double tune_ms = 0.0;
  // backward work list and partials
  wn::Item* d_bitems = nullptr;
  int32_t n_bitems = 0;
  float* d_pv = nullptr;
  float* d_pl = nullptr;
  double* d_tmp = nullptr;
  wn::RBlock* d_rblocks = nullptr;
  int32_t n_rblocks = 0;
  int64_t n_tmp = 0;
  // graph of the forward
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t fwd_node = nullptr;  // fused kernel, or the crossing kernel
  hipGraphNode_t bnd_node = nullptr;  // split mode: the boundary kernel
  wn::FwdArgs graph_args{};
  bool use_graph = true;
};

namespace {

wn_status upload_items(wn_batch* b, int tile) {
  std::vector<wn::Item> items;
  std::vector<double> cost;
  for (int s = 0; s < b->ns; ++s) {
    const wn::SurfDesc& D = b->desc[s];
    int t = 0;
    for (int64_t q = 0; q < D.nq; q += tile, ++t) {
      wn::Item it;
      it.surf = s;
      it.q0 = D.q_off + q;
      it.cnt = (int32_t)std::min<int64_t>(tile, D.nq - q);
      it.tile = t;
      it.pad = 0;
      items.push_back(it);
      cost.push_back((double)it.cnt * ((double)D.nb + 24.0));
    }
  }
  std::vector<size_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  std::vector<wn::Item> sorted(items.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
  if (b->d_items) hipFree(b->d_items);
  b->d_items = nullptr;
  b->n_items = (int32_t)sorted.size();
  if (!sorted.empty()) {
    WN_HIP(hipMalloc((void**)&b->d_items, sorted.size() * sizeof(wn::Item)), "batch items");
    WN_HIP(hipMemcpy(b->d_items, sorted.data(), sorted.size() * sizeof(wn::Item), hipMemcpyHostToDevice),
           "batch items");
  }
  b->tile = tile;
  return WN_OK;
}

wn::FwdArgs fwd_args(const wn_batch* b, const float* qx, const float* qy, const float* qz, float* w,
                     int32_t* chi) {
  wn::FwdArgs a;
  std::memset(&a, 0, sizeof a);   // padding too: arguments are compared bytewise
  a.descs = b->d_desc;
  a.items = b->d_items;
  a.n_items = b->n_items;
  a.direct = b->wgpcu == 0 ? 1 : 0;
  a.counter = b->d_counter;
  a.bndr = b->d_bndr;
  a.loops = b->d_loops;
  a.qx = qx;
  a.qy = qy;
  a.qz = qz;
  a.w = w;
  a.chi = chi;
  a.chi_buf = chi ? chi : b->d_chi;
  return a;
}

// wgpcu > 0: a persistent grid of wgpcu workgroups per compute unit;
// wgpcu == 0: one workgroup per item (the hardware dispatcher hands them out
// in list order, which keeps the longest-first order of the items).
int grid_of(const wn_batch* b, int n_items) {
  if (b->wgpcu == 0) return std::max(1, n_items);
  return std::max(1, std::min(n_items, b->wgpcu * b->cus));
}

hipError_t launch_fwd(const wn_batch* b, const wn::FwdArgs& a, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (!a.direct) {
    hipLaunchKernelGGL(wn::k_reset, dim3(1), dim3(64), 0, s, b->d_counter);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (a.n_items == 0) return hipSuccess;
  const dim3 grid(grid_of(b, a.n_items));
  if (b->mode == 0) {
    hipLaunchKernelGGL(wn::k_batch_fwd, grid, dim3(wn::kThreads), 0, s, a);
    return hipGetLastError();
  }
  if (!a.chi_buf) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wn::k_batch_cross, grid, dim3(wn::kThreads), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wn::k_batch_bnd, grid, dim3(wn::kThreads), 0, s, a);
  return hipGetLastError();
}

// Crossing-count buffer of the split mode when the caller passes no chi_out.
wn_status ensure_chi(wn_batch* b) {
  if (b->d_chi || b->total_q == 0) return WN_OK;
  WN_HIP(hipMalloc((void**)&b->d_chi, (size_t)b->total_q * sizeof(int32_t)), "crossing buffer");
  return WN_OK;
}

void drop_graph(wn_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->fwd_node = nullptr;
  b->bnd_node = nullptr;
}

// Capture reset + persistent forward into a graph (on a private stream).
wn_status capture(wn_batch* b, const wn::FwdArgs& a) {
  drop_graph(b);
  if (!b->cap) WN_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream");
  WN_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  const hipError_t le = launch_fwd(b, a, b->cap);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(b->cap, &g);
  if (le != hipSuccess) { if (g) hipGraphDestroy(g); return hip_fail(le, "capture launch"); }
  if (ce != hipSuccess) return hip_fail(ce, "end capture");
  b->graph = g;
  WN_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
  size_t n = 0;
  WN_HIP(hipGraphGetNodes(g, nullptr, &n), "graph nodes");
  std::vector<hipGraphNode_t> nodes(n);
  WN_HIP(hipGraphGetNodes(g, nodes.data(), &n), "graph nodes");
  for (auto nd : nodes) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(nd, &t) != hipSuccess || t != hipGraphNodeTypeKernel) continue;
    hipKernelNodeParams p;
    if (hipGraphKernelNodeGetParams(nd, &p) != hipSuccess) continue;
    if (p.func == reinterpret_cast<void*>(wn::k_batch_fwd) || p.func == reinterpret_cast<void*>(wn::k_batch_cross))
      b->fwd_node = nd;
    if (p.func == reinterpret_cast<void*>(wn::k_batch_bnd)) b->bnd_node = nd;
  }
  b->graph_args = a;
  return WN_OK;
}

bool same_args(const wn::FwdArgs& x, const wn::FwdArgs& y) {
  return std::memcmp(&x, &y, sizeof x) == 0;
}

// Best of two trials of three back-to-back graph replays, and the same for
// direct launches, in ms per forward.
wn_status time_graph_vs_direct(wn_batch* b, const wn::FwdArgs& a, hipStream_t s, float* tg, float* td) {
  hipEvent_t e0, e1;
  WN_HIP(hipEventCreate(&e0), "event");
  WN_HIP(hipEventCreate(&e1), "event");
  float best[2] = {1e30f, 1e30f};
  for (int v = 0; v < 2; ++v) {
    for (int r = 0; r < 3; ++r) {      // first pass warms up
      WN_HIP(hipEventRecord(e0, s), "event");
      for (int k = 0; k < 3; ++k) {
        if (v == 0) WN_HIP(hipGraphLaunch(b->exec, s), "graph launch");
        else WN_HIP(launch_fwd(b, a, s), "batched forward");
      }
      WN_HIP(hipEventRecord(e1, s), "event");
      WN_HIP(hipEventSynchronize(e1), "event");
      float ms = 0.f;
      WN_HIP(hipEventElapsedTime(&ms, e0, e1), "event");
      if (r > 0) best[v] = std::min(best[v], ms / 3.0f);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *tg = best[0];
  *td = best[1];
  return WN_OK;
}

// --- autotuner ---------------------------------------------------------------

std::string tune_key(const wn_batch* b) {
  char k[160];
  const int lq = b->total_q > 0 ? (int)std::lround(std::log2((double)b->total_q)) : 0;
  const int lp = b->total_pairs > 0 ? (int)std::lround(std::log2((double)b->total_pairs)) : 0;
  hipDeviceProp_t prop;
  const char* arch = "gfx";
  if (hipGetDeviceProperties(&prop, b->dev) == hipSuccess) arch = prop.gcnArchName;
  std::string a(arch);
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a = a.substr(0, colon);
  std::snprintf(k, sizeof k, "%s_cu%d_s%d_q%d_p%d", a.c_str(), b->cus, b->ns, lq, lp);
  return k;
}

bool cache_lookup(const std::string& key, int* tile, int* wgpcu, int* mode) {
  const char* path = std::getenv("WN_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  std::fclose(f);
  const std::string pat = "\"" + key + "\"";
  const size_t p = txt.find(pat);
  if (p == std::string::npos) return false;
  int a = 0, c = 0, m = -1;
  if (std::sscanf(txt.c_str() + p + pat.size(), " : [ %d , %d , %d ]", &a, &c, &m) != 3) return false;
  if (a <= 0 || c < 0 || m < 0 || m > 1) return false;
  *tile = a;
  *wgpcu = c;
  *mode = m;
  return true;
}

void cache_store(const std::string& key, int tile, int wgpcu, int mode) {
  const char* path = std::getenv("WN_TUNE_CACHE");
  if (!path) return;
  // flat JSON object {"key": [tile, wg_per_cu, mode], ...}; entries of other keys are kept
  std::vector<std::string> lines;
  if (FILE* f = std::fopen(path, "r")) {
    char buf[512];
    while (std::fgets(buf, sizeof buf, f)) {
      std::string l(buf);
      const size_t q = l.find('"');
      if (q == std::string::npos) continue;
      const size_t q2 = l.find('"', q + 1);
      if (q2 == std::string::npos) continue;
      if (l.substr(q + 1, q2 - q - 1) == key) continue;
      while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' ')) l.pop_back();
      lines.push_back(l);
    }
    std::fclose(f);
  }
  char e[256];
  std::snprintf(e, sizeof e, "  \"%s\": [%d, %d, %d]", key.c_str(), tile, wgpcu, mode);
  lines.push_back(e);
  if (FILE* f = std::fopen(path, "w")) {
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < lines.size(); ++i)
      std::fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
  }
}

// Time candidate (tile, workgroups per CU) pairs on the real inputs; every
// run writes complete outputs, the last run uses the winner.
wn_status autotune(wn_batch* b, const wn::FwdArgs& base, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  int tile = b->tile, wg = b->wgpcu, mode = b->mode;
  const std::string key = tune_key(b);
  if (!base.chi) {
    wn_status st = ensure_chi(b);   // the split candidates need a crossing buffer
    if (st) return st;
  }
  if (!cache_lookup(key, &tile, &wg, &mode) || (b->mode_fixed >= 0 && mode != b->mode_fixed)) {
    std::vector<int> tiles, wgs;
    if (b->tune_mode >= 2) {
      tiles = {256, 512, 1024, 2048, 4096};
      wgs = {1, 2, 4, 8, 0};
    } else {
      tiles = {256, 512, 1024, 2048};
      wgs = {4, 8, 0};
    }
    hipEvent_t e0, e1;
    WN_HIP(hipEventCreate(&e0), "event");
    WN_HIP(hipEventCreate(&e1), "event");
    // back-to-back launches as in use (a single launch after a sync ranks the
    // candidates differently): best of `trials` trials of `reps` launches
    auto time_config = [&](int t, int m, int w, int trials, int reps, float* out) -> wn_status {
      wn_status st = upload_items(b, t);
      if (st) return st;
      b->wgpcu = w;
      b->mode = m;
      const wn::FwdArgs a = fwd_args(b, base.qx, base.qy, base.qz, base.w, base.chi);
      WN_HIP(launch_fwd(b, a, s), "tune launch");   // warm-up
      float ms = 1e30f;
      for (int r = 0; r < trials; ++r) {
        WN_HIP(hipEventRecord(e0, s), "event");
        for (int k = 0; k < reps; ++k) WN_HIP(launch_fwd(b, a, s), "tune launch");
        WN_HIP(hipEventRecord(e1, s), "event");
        WN_HIP(hipEventSynchronize(e1), "event");
        float total = 0.f;
        WN_HIP(hipEventElapsedTime(&total, e0, e1), "event");
        ms = std::min(ms, total / (float)reps);
      }
      *out = ms;
      return WN_OK;
    };
    struct Cand {
      float ms;
      int tile, mode, wg;
    };
    std::vector<Cand> cands;
    for (int t : tiles)
      for (int m = 0; m < 2; ++m) {
        if (b->mode_fixed >= 0 && m != b->mode_fixed) continue;
        for (int w : wgs) {
          float ms = 0.f;
          wn_status st = time_config(t, m, w, 2, 3, &ms);
          if (st) return st;
          if (std::getenv("WN_TUNE_LOG"))
            std::fprintf(stderr, "wn tune: tile %d mode %s wg/cu %d: %.4f ms\n", t, m ? "split" : "fused", w, ms);
          cands.push_back({ms, t, m, w});
        }
      }
    // the sweep's early candidates run on a colder GPU: the three best are
    // timed again, longer, in the opposite order, and the fastest is kept
    std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    const size_t nfinal = std::min<size_t>(3, cands.size());
    float best = 1e30f;
    for (size_t i = nfinal; i-- > 0;) {
      float ms = 0.f;
      wn_status st = time_config(cands[i].tile, cands[i].mode, cands[i].wg, 3, 5, &ms);
      if (st) return st;
      if (std::getenv("WN_TUNE_LOG"))
        std::fprintf(stderr, "wn tune final: tile %d mode %s wg/cu %d: %.4f ms\n", cands[i].tile,
                     cands[i].mode ? "split" : "fused", cands[i].wg, ms);
      if (ms < best) {
        best = ms;
        tile = cands[i].tile;
        wg = cands[i].wg;
        mode = cands[i].mode;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    cache_store(key, tile, wg, mode);
  }
  b->wgpcu = wg;
  b->mode = mode;
  wn_status st = upload_items(b, tile);
  if (st) return st;
  b->tuned = true;
  b->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return WN_OK;
}

}  // namespace

extern "C" {

wn_status wn_batch_create(const wn_surface* surfs, int32_t ns, const double dir[3], int32_t tune_mode,
                          void* stream, wn_batch** out) {
  wn::host::g_err.clear();
  if (!out) return fail(WN_ERR_INVALID_ARGUMENT, "out is NULL");
  if (ns < 0 || (ns > 0 && !surfs)) return fail(WN_ERR_INVALID_ARGUMENT, "bad surface list");
  if (tune_mode < 0 || tune_mode > 2) return fail(WN_ERR_INVALID_ARGUMENT, "tune_mode must be 0, 1 or 2");
  hipStream_t s = as_stream(stream);
  // validate every surface before building anything
  std::vector<wn::LoopTable> lts((size_t)ns);
  std::vector<int64_t> nbs((size_t)ns);
  for (int32_t i = 0; i < ns; ++i) {
    const wn_surface& S = surfs[i];
    if (S.nq < 0) return fail(WN_ERR_INVALID_ARGUMENT, "surface %d: negative query count", i);
    wn_status st = wn::host::make_loops(S.loop_off, S.nloops, 3, &nbs[i], &lts[i]);
    if (st) return fail(st, "surface %d: %s", i, wn::host::g_err.c_str());
    if (nbs[i] > 0 && !S.bnd_xyz) return fail(WN_ERR_INVALID_ARGUMENT, "surface %d: bnd_xyz is NULL", i);
  }
  wn_batch* b = new wn_batch();
  b->ns = ns;
  b->tune_mode = tune_mode;
  b->use_graph = !std::getenv("WN_FORCE_NO_GRAPH");
  if (const char* m = std::getenv("WN_BATCH_MODE")) {
    if (!std::strcmp(m, "fused")) b->mode_fixed = 0;
    else if (!std::strcmp(m, "split")) b->mode_fixed = 1;
    if (b->mode_fixed >= 0) b->mode = b->mode_fixed;
  }
  hipGetDevice(&b->dev);
  hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->dev);
  if (b->cus <= 0) b->cus = 256;
  auto bail = [&](wn_status st) {
    const std::string msg = wn::host::g_err;
    wn_batch_free(b);
    wn::host::g_err = msg;
    return st;
  };
  b->q_off.assign((size_t)ns + 1, 0);
  std::vector<int32_t> loops_h;
  std::vector<int32_t> surf_of;
  int64_t boff = 0;
  for (int32_t i = 0; i < ns; ++i) {
    const wn_surface& S = surfs[i];
    wn_bvh* h = nullptr;
    wn_status st = wn_build_bvh(S.V, S.nv, S.F, S.nf, dir, stream, &h);
    if (st) return bail(st);
    b->bvh.push_back(h);
    wn::SurfDesc D{};
    D.F = h->F;
    D.nodes = h->nodes;
    D.tris = h->tris;
    D.leafbox = h->leafbox;
    D.leafz = h->leafz;
    D.nf = h->nf;
    D.nb = (int32_t)nbs[i];
    D.bnd_off = boff;
    D.loop_off = (int32_t)loops_h.size();
    D.nloops = S.nloops;
    for (int l = 0; l <= S.nloops && S.nloops > 0; ++l) loops_h.push_back((int32_t)S.loop_off[l]);
    if (S.nloops == 0) loops_h.push_back(0);
    D.q_off = b->q_off[i];
    D.nq = S.nq;
    b->q_off[i + 1] = b->q_off[i] + S.nq;
    for (int64_t v = 0; v < nbs[i]; ++v) surf_of.push_back(i);
    boff += nbs[i];
    b->desc.push_back(D);
    b->total_pairs += S.nq * nbs[i];
  }
  b->total_q = b->q_off[ns];
  b->total_b = boff;
  // backward partial layout (fixed per surface: tile index x wavefront)
  int64_t pv = 0, pl = 0;
  for (auto& D : b->desc) {
    D.tiles_bwd = (int32_t)((D.nq + wn::adj::kTile - 1) / wn::adj::kTile);
    D.pv_off = pv;
    D.pl_off = pl;
    pv += (int64_t)D.tiles_bwd * D.nb * 3;
    pl += (int64_t)D.tiles_bwd * D.nloops * 3;
    D.groups = (int32_t)(((int64_t)D.tiles_bwd + wn::kRowsPerGroup - 1) / wn::kRowsPerGroup);
    D.tmp_off = b->n_tmp;
    b->n_tmp += (int64_t)D.groups * D.nb * 3;
  }
  std::vector<wn::RBlock> rblocks;
  for (int32_t i = 0; i < ns; ++i) {
    const wn::SurfDesc& D = b->desc[i];
    for (int32_t g = 0; g < D.groups; ++g)
      for (int64_t c0 = 0; c0 < (int64_t)D.nb * 3; c0 += 256) rblocks.push_back({i, g, (int32_t)c0, 0});
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chk(hipMalloc((void**)&b->d_desc, std::max<size_t>(1, b->desc.size()) * sizeof(wn::SurfDesc)));
  chk(hipMalloc((void**)&b->d_loops, std::max<size_t>(1, loops_h.size()) * sizeof(int32_t)));
  chk(hipMalloc((void**)&b->d_bnd, std::max<int64_t>(1, boff) * 3 * sizeof(float)));
  chk(hipMalloc((void**)&b->d_surf_of, std::max<size_t>(1, surf_of.size()) * sizeof(int32_t)));
  chk(hipMalloc((void**)&b->d_counter, 64));
  if (e == hipSuccess && !b->desc.empty())
    chk(hipMemcpy(b->d_desc, b->desc.data(), b->desc.size() * sizeof(wn::SurfDesc), hipMemcpyHostToDevice));
  if (e == hipSuccess && !loops_h.empty())
    chk(hipMemcpy(b->d_loops, loops_h.data(), loops_h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (e == hipSuccess && !surf_of.empty())
    chk(hipMemcpy(b->d_surf_of, surf_of.data(), surf_of.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  for (int32_t i = 0; i < ns && e == hipSuccess; ++i)
    if (nbs[i] > 0)
      chk(hipMemcpyAsync(b->d_bnd + 3 * b->desc[i].bnd_off, surfs[i].bnd_xyz, (size_t)nbs[i] * 3 * sizeof(float),
                         hipMemcpyDeviceToDevice, s));
  if (e == hipSuccess) chk(hipMalloc((void**)&b->d_bndr, std::max<int64_t>(1, boff) * sizeof(wn::RPt)));
  if (e == hipSuccess && boff > 0) {
    hipLaunchKernelGGL(wn::k_rotate_bnd, dim3((unsigned)((boff + 255) / 256)), dim3(256), 0, s, b->d_desc,
                       b->d_loops, b->d_bnd, b->d_surf_of, boff, b->d_bndr);
    chk(hipGetLastError());
  }
  b->n_rblocks = (int32_t)rblocks.size();
  if (e == hipSuccess && !rblocks.empty()) {
    chk(hipMalloc((void**)&b->d_rblocks, rblocks.size() * sizeof(wn::RBlock)));
    if (e == hipSuccess)
      chk(hipMemcpy(b->d_rblocks, rblocks.data(), rblocks.size() * sizeof(wn::RBlock), hipMemcpyHostToDevice));
  }
  if (e == hipSuccess) chk(hipStreamSynchronize(s));
  if (e != hipSuccess) return bail(hip_fail(e, "wn_batch_create"));
  wn_status st = upload_items(b, b->tile);
  if (st) return bail(st);
  // backward items: one per (surface, tile of adj::kTile queries), LPT order
  {
    std::vector<wn::Item> items;
    std::vector<double> cost;
    for (int32_t i = 0; i < ns; ++i) {
      const wn::SurfDesc& D = b->desc[i];
      for (int32_t t = 0; t < D.tiles_bwd; ++t) {
        wn::Item it;
        it.surf = i;
        it.tile = t;
        it.q0 = D.q_off + (int64_t)t * wn::adj::kTile;
        it.cnt = (int32_t)std::min<int64_t>(wn::adj::kTile, D.nq - (int64_t)t * wn::adj::kTile);
        it.pad = 0;
        items.push_back(it);
        cost.push_back((double)it.cnt * (double)D.nb);
      }
    }
    std::vector<size_t> order(items.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<wn::Item> sorted(items.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = items[order[k]];
    b->n_bitems = (int32_t)sorted.size();
    if (!sorted.empty()) {
      e = hipMalloc((void**)&b->d_bitems, sorted.size() * sizeof(wn::Item));
      if (e == hipSuccess)
        e = hipMemcpy(b->d_bitems, sorted.data(), sorted.size() * sizeof(wn::Item), hipMemcpyHostToDevice);
      if (e != hipSuccess) return bail(hip_fail(e, "backward items"));
    }
  }
  *out = b;
  return WN_OK;
}

wn_status wn_batch_free(wn_batch* b) {
  wn::host::g_err.clear();
  if (!b) return WN_OK;
  drop_graph(b);
  if (b->cap) hipStreamDestroy(b->cap);
  for (auto h : b->bvh) wn_free_bvh(h);
  hipFree(b->d_desc);
  hipFree(b->d_loops);
  hipFree(b->d_bnd);
  hipFree(b->d_bndr);
  hipFree(b->d_surf_of);
  hipFree(b->d_counter);
  hipFree(b->d_items);
  hipFree(b->d_bitems);
  hipFree(b->d_pv);
  hipFree(b->d_pl);
  hipFree(b->d_tmp);
  hipFree(b->d_rblocks);
  hipFree(b->d_chi);
  delete b;
  return WN_OK;
}

wn_status wn_eval_batched(wn_batch* b, const float* qx, const float* qy, const float* qz, float* w_out,
                          int32_t* chi_out, void* stream) {
  wn::host::g_err.clear();
  if (!b) return fail(WN_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (b->total_q == 0) return WN_OK;
  if (!qx || !qy || !qz || !w_out) return fail(WN_ERR_INVALID_ARGUMENT, "NULL query or output pointer");
  hipStream_t s = as_stream(stream);
  const bool tuning = b->tune_mode > 0 && !b->tuned;
  if (tuning) {
    wn_status st = autotune(b, fwd_args(b, qx, qy, qz, w_out, chi_out), s);
    if (st) return st;
    drop_graph(b);
  }
  if (b->mode == 1 && !chi_out) {
    wn_status st = ensure_chi(b);
    if (st) return st;
  }
  const wn::FwdArgs a = fwd_args(b, qx, qy, qz, w_out, chi_out);
  if (!b->use_graph) {
    WN_HIP(launch_fwd(b, a, s), "batched forward");
    return WN_OK;
  }
  if (!b->exec) {
    wn_status st = capture(b, a);
    if (st) {
      // no graph on this system: direct launches give the same results
      drop_graph(b);
      b->use_graph = false;
      WN_HIP(launch_fwd(b, a, s), "batched forward");
      return WN_OK;
    }
    if (tuning) {
      // the tuner also decides graph replay against direct launches of the
      // winning configuration: a one-kernel graph saves no launch overhead,
      // and its replay has measured slower on some runtimes
      float tg = 0.f, td = 0.f;
      st = time_graph_vs_direct(b, a, s, &tg, &td);
      if (st) return st;
      if (std::getenv("WN_TUNE_LOG")) std::fprintf(stderr, "wn tune: graph %.4f ms, direct %.4f ms\n", tg, td);
      if (tg > 1.02f * td) {
        drop_graph(b);
        b->use_graph = false;
        WN_HIP(launch_fwd(b, a, s), "batched forward");
        return WN_OK;
      }
    }
  } else if (!same_args(a, b->graph_args) && (!b->fwd_node || (b->mode == 1 && !b->bnd_node))) {
    wn_status st = capture(b, a);   // cannot patch the nodes: capture again
    if (st) return st;
  } else if (!same_args(a, b->graph_args)) {
    hipGraphNode_t nodes[2] = {b->fwd_node, b->mode == 1 ? b->bnd_node : nullptr};
    for (hipGraphNode_t nd : nodes) {
      if (!nd) continue;
      hipKernelNodeParams p;
      WN_HIP(hipGraphKernelNodeGetParams(nd, &p), "graph params");
      wn::FwdArgs na = a;
      void* args[1] = {&na};
      p.kernelParams = args;
      p.extra = nullptr;
      WN_HIP(hipGraphExecKernelNodeSetParams(b->exec, nd, &p), "graph update");
    }
    b->graph_args = a;
  }
  WN_HIP(hipGraphLaunch(b->exec, s), "graph launch");
  return WN_OK;
}

wn_status wn_backward_batched(wn_batch* b, const float* qx, const float* qy, const float* qz,
                              const float* grad_w, float* grad_q, float* grad_bnd, void* stream) {
  wn::host::g_err.clear();
  if (!b) return fail(WN_ERR_INVALID_ARGUMENT, "batch is NULL");
  hipStream_t s = as_stream(stream);
  if (grad_bnd && b->total_b > 0 && b->total_q == 0) {
    hipLaunchKernelGGL(wn::k_fill_f32, dim3((unsigned)((3 * b->total_b + 255) / 256)), dim3(256), 0, s,
                       grad_bnd, 3 * b->total_b);
    WN_HIP(hipGetLastError(), "zero grad_bnd");
  }
  if (b->total_q == 0) return WN_OK;
  if (!qx || !qy || !qz || !grad_w) return fail(WN_ERR_INVALID_ARGUMENT, "NULL query or gradient pointer");
  if (grad_bnd && !b->d_pv && b->total_b > 0) {
    int64_t pv = 0, pl = 0;
    for (const auto& D : b->desc) {
      pv = std::max<int64_t>(pv, D.pv_off + (int64_t)D.tiles_bwd * D.nb * 3);
      pl = std::max<int64_t>(pl, D.pl_off + (int64_t)D.tiles_bwd * D.nloops * 3);
    }
    WN_HIP(hipMalloc((void**)&b->d_pv, std::max<int64_t>(pv, 1) * sizeof(float)), "backward partials");
    WN_HIP(hipMalloc((void**)&b->d_pl, std::max<int64_t>(pl, 1) * sizeof(float)), "backward partials");
    WN_HIP(hipMalloc((void**)&b->d_tmp, std::max<int64_t>(b->n_tmp, 1) * sizeof(double)), "backward partials");
  }
  wn::BwdArgs a;
  a.descs = b->d_desc;
  a.items = b->d_bitems;
  a.n_items = b->n_bitems;
  a.counter = b->d_counter;
  a.bnd = b->d_bnd;
  a.loops = b->d_loops;
  a.qx = qx;
  a.qy = qy;
  a.qz = qz;
  a.gw = grad_w;
  a.gq = grad_q;
  a.pv = grad_bnd ? b->d_pv : nullptr;
  a.pl = grad_bnd ? b->d_pl : nullptr;
  // one workgroup per item, dispatched in list (longest first) order
  hipLaunchKernelGGL(wn::k_batch_bwd, dim3((unsigned)std::max(1, b->n_bitems)), dim3(wn::kThreads), 0, s, a);
  WN_HIP(hipGetLastError(), "batched backward");
  if (grad_bnd && b->total_b > 0) {
    const int64_t n3 = 3 * b->total_b;
    if (b->n_rblocks > 0) {
      hipLaunchKernelGGL(wn::k_batch_rows, dim3((unsigned)b->n_rblocks), dim3(256), 0, s, b->d_desc,
                         b->d_rblocks, b->d_loops, b->d_pv, b->d_pl, b->d_tmp);
      WN_HIP(hipGetLastError(), "batched reduce");
    }
    hipLaunchKernelGGL(wn::k_batch_groups, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, b->d_desc,
                       b->d_surf_of, b->d_tmp, n3, grad_bnd);
    WN_HIP(hipGetLastError(), "batched reduce");
  }
  return WN_OK;
}

wn_status wn_batch_info(const wn_batch* b, int64_t info[9]) {
  wn::host::g_err.clear();
  if (!b || !info) return fail(WN_ERR_INVALID_ARGUMENT, "NULL argument");
  info[0] = b->total_q;
  info[1] = b->total_b;
  info[2] = b->total_pairs;
  info[3] = b->n_items;
  info[4] = b->tile;
  info[5] = b->wgpcu;
  info[6] = (b->use_graph && b->exec) ? 1 : 0;
  info[7] = (int64_t)std::llround(b->tune_ms * 1000.0);
  info[8] = b->mode;
  return WN_OK;
}

}  // extern "C"
