// Crossing count chi_d (Eq. chi; the ray-casting step of Alg. 1) through a linear BVH
// built on the GPU.
//
// All rays of one call are parallel to d, so in the frame of d (rows e1, e2,
// d) every ray is the vertical half line above (X_p, Y_p, Z_p).  A node
// therefore stores, for each child, the 2D box of the children's projections
// and the largest Z: a ray can reach the child only if its (X, Y) lies in the
// box and Z_p is below that largest Z.  The paper uses a k-d tree for its
// ray/mesh intersections (Sec. 5.1, "Meshes"); the tree here is a linear BVH
// (Karras 2012) over 2D Morton codes of the projected centroids, built with
// a project-written LSD radix sort, and traversed with a short stack held in
// registers.
#include <algorithm>

#include "kernels.hpp"
#include "bvh_build.hpp"
#include "traverse.hpp"

namespace wn {

// Workgroups of two wavefronts: finer-grained than 256 lanes for the
// scheduler to balance traversals of uneven length (3 % faster on 2^20
// random queries than 256, the same as 64).
constexpr int kCrossThreads = 128;

template <int S>
__global__ __launch_bounds__(kCrossThreads) void k_cross3d(CrossArgs a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.nq) return;
  const float px = a.qx[q], py = a.qy[q], pz = a.qz[q];
  if (!(isfinite(px) && isfinite(py) && isfinite(pz))) {
    a.chi[q] = WN_CHI_INVALID;
    return;
  }
  double Xp, Yp, Zp;
  rotate(a.F, px, py, pz, Xp, Yp, Zp);
  a.chi[q] = traverse<S>(a, make_qp(Xp, Yp, Zp));
}

hipError_t launch_cross3d(const CrossArgs& a, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.nq + kCrossThreads - 1) / kCrossThreads);
  hipLaunchKernelGGL(k_cross3d<kShortStack>, dim3(blocks), dim3(kCrossThreads), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Build
// ---------------------------------------------------------------------------

namespace {

__device__ __forceinline__ unsigned f2ord(float f) {
  const unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned o) {
  const unsigned u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}

// float32 not above / not below a float64 value
__device__ __forceinline__ float f_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
__device__ __forceinline__ float f_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

__global__ void k_rotate_vertices(Frame F, const float* __restrict__ V, int32_t nv, RPt* __restrict__ Vr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double X, Y, Z;
  rotate(F, V[3 * i], V[3 * i + 1], V[3 * i + 2], X, Y, Z);
  Vr[i] = make_rpt(X, Y, Z, 0.0);
}

// Projected box (+ pad) of each triangle and its centroid.
__global__ void k_tri_boxes(const RPt* __restrict__ Vr, const int32_t* __restrict__ Fc,
                            int32_t nf, float pad, float4* __restrict__ box,
                            float* __restrict__ zmax, float2* __restrict__ cen) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const RPt A = Vr[Fc[3 * i]];
  const RPt B = Vr[Fc[3 * i + 1]];
  const RPt C = Vr[Fc[3 * i + 2]];
  const double ax = hilo(A.xy.x, A.xy.y), bx = hilo(B.xy.x, B.xy.y), cx = hilo(C.xy.x, C.xy.y);
  const double ay = hilo(A.xy.z, A.xy.w), by = hilo(B.xy.z, B.xy.w), cy = hilo(C.xy.z, C.xy.w);
  const double az = hilo(A.zt.x, A.zt.y), bz = hilo(B.zt.x, B.zt.y), cz = hilo(C.zt.x, C.zt.y);
  const double x0 = fmin(ax, fmin(bx, cx)), x1 = fmax(ax, fmax(bx, cx));
  const double y0 = fmin(ay, fmin(by, cy)), y1 = fmax(ay, fmax(by, cy));
  const double z1 = fmax(az, fmax(bz, cz));
  box[i] = make_float4(f_down(x0) - pad, f_up(x1) + pad, f_down(y0) - pad, f_up(y1) + pad);
  zmax[i] = f_up(z1) + pad;
  cen[i] = make_float2((float)(0.5 * (x0 + x1)), (float)(0.5 * (y0 + y1)));
}

// Workgroups of the grid-stride reductions below: few enough that their one
// atomic per value and workgroup do not queue up on the same words.
constexpr int kReduceBlocks = 256;

// Bounds of the centroids as order-preserving integers: cb = {min x, max x,
// min y, max y}.
__global__ __launch_bounds__(256) void k_cen_bounds(const float2* __restrict__ cen, int32_t nf,
                                                    unsigned* __restrict__ cb) {
  __shared__ unsigned red[4][4];
  unsigned v[4] = {0xffffffffu, 0u, 0xffffffffu, 0u};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nf; i += gridDim.x * 256) {
    const float2 c = cen[i];
    const unsigned ox = f2ord(c.x), oy = f2ord(c.y);
    v[0] = min(v[0], ox);
    v[1] = max(v[1], ox);
    v[2] = min(v[2], oy);
    v[3] = max(v[3], oy);
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int k = 0; k < 4; ++k) {
      const unsigned w = (unsigned)__shfl_xor((int)v[k], o, 64);
      v[k] = (k % 2 == 0) ? min(v[k], w) : max(v[k], w);
    }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    unsigned r = red[k][0];
    for (int w = 1; w < 4; ++w) r = (k % 2 == 0) ? min(r, red[k][w]) : max(r, red[k][w]);
    if (k % 2 == 0) atomicMin(&cb[k], r);
    else atomicMax(&cb[k], r);
  }
}

__device__ __forceinline__ unsigned spread16(unsigned v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__global__ void k_morton(const float2* __restrict__ cen, int32_t nf, const unsigned* __restrict__ cb,
                         unsigned* __restrict__ keys, int32_t* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const float x0 = ord2f(cb[0]), x1 = ord2f(cb[1]), y0 = ord2f(cb[2]), y1 = ord2f(cb[3]);
  const float sx = (x1 > x0) ? 65535.0f / (x1 - x0) : 0.0f;
  const float sy = (y1 > y0) ? 65535.0f / (y1 - y0) : 0.0f;
  const float2 c = cen[i];
  const unsigned ix = (unsigned)fminf(fmaxf((c.x - x0) * sx, 0.0f), 65535.0f);
  const unsigned iy = (unsigned)fminf(fmaxf((c.y - y0) * sy, 0.0f), 65535.0f);
  keys[i] = spread16(ix) | (spread16(iy) << 1);
  vals[i] = i;
}

// Karras 2012: internal node i of n-1 covers a key range found from the
// common-prefix lengths of its neighbours; duplicate keys are split by index.
__device__ __forceinline__ int delta(const unsigned* __restrict__ k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  const unsigned long long a = ((unsigned long long)k[i] << 32) | (unsigned)i;
  const unsigned long long b = ((unsigned long long)k[j] << 32) | (unsigned)j;
  return __clzll(a ^ b);
}

__global__ void k_karras(const unsigned* __restrict__ keys, int32_t n, int32_t* __restrict__ left,
                         int32_t* __restrict__ right, int32_t* __restrict__ parent_int,
                         int32_t* __restrict__ parent_leaf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = delta(keys, n, i, i - d);
  int lmax = 2;
  while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = delta(keys, n, i, j);
  int s = 0;
  int t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  const int gamma = i + s * d + min(d, 0);
  const int lo = min(i, j), hi = max(i, j);
  const int32_t lc = (lo == gamma) ? ~gamma : gamma;
  const int32_t rc = (hi == gamma + 1) ? ~(gamma + 1) : gamma + 1;
  left[i] = lc;
  right[i] = rc;
  if (lc < 0) parent_leaf[~lc] = i; else parent_int[lc] = i;
  if (rc < 0) parent_leaf[~rc] = i; else parent_int[rc] = i;
  if (i == 0) parent_int[0] = -1;
}

// Sorted triangle records and leaf boxes in sorted order.  Each record
// carries its three vertices and the lexicographic order of each edge's end
// points (the sign of the edge's tie offset), so that a crossing test reads
// one line and recomputes no comparison.
__global__ void k_gather_leaves(const int32_t* __restrict__ Fc, const int32_t* __restrict__ order,
                                int32_t nf, const float4* __restrict__ box,
                                const float* __restrict__ zmax, const RPt* __restrict__ Vr,
                                TriRec* __restrict__ tris, float4* __restrict__ lbox, float* __restrict__ lz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  int f = order[i];
  if (f < 0 || f >= nf) f = 0;   // never taken for a permutation
  const RPt A = Vr[Fc[3 * f]], B = Vr[Fc[3 * f + 1]], C = Vr[Fc[3 * f + 2]];
  TriRec r;
  r.xy[0] = A.xy;
  r.xy[1] = B.xy;
  r.xy[2] = C.xy;
  r.zch = C.zt.x;
  r.zcl = C.zt.y;
  r.ties = (rpt_less(A, B) ? 1u : 0u) | (rpt_less(B, C) ? 2u : 0u) | (rpt_less(C, A) ? 4u : 0u);
  r.face = f;
  r.zab = make_float4(A.zt.x, A.zt.y, B.zt.x, B.zt.y);
  for (int k = 0; k < 12; ++k) r.pad[k] = 0u;
  tris[i] = r;
  lbox[i] = box[f];
  lz[i] = zmax[f];
}

// Depth of every internal node (distance to the root) by pointer jumping
// over the parent links: after r rounds anc[i] is the 2^r-th ancestor (or -1)
// and dep[i] the number of links walked.
__global__ void k_depth_init(const int32_t* __restrict__ parent_int, int32_t n, int32_t* __restrict__ anc,
                             int32_t* __restrict__ dep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t p = parent_int[i];
  anc[i] = p;
  dep[i] = p >= 0 ? 1 : 0;
}

__global__ void k_depth_jump(const int32_t* __restrict__ anc_in, const int32_t* __restrict__ dep_in, int32_t n,
                             int32_t* __restrict__ anc_out, int32_t* __restrict__ dep_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = anc_in[i];
  if (a >= 0 && a < n) {
    dep_out[i] = dep_in[i] + dep_in[a];
    anc_out[i] = anc_in[a];
  } else {
    dep_out[i] = dep_in[i];
    anc_out[i] = -1;
  }
}

// res[0] = deepest level, res[1] = 1 if some node has not reached the root.
__global__ __launch_bounds__(256) void k_depth_max(const int32_t* __restrict__ anc, const int32_t* __restrict__ dep,
                                                   int32_t n, int32_t* res) {
  __shared__ int red[2][4];
  int m = 0, open = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    m = max(m, dep[i]);
    open = max(open, anc[i] >= 0 ? 1 : 0);
  }
  for (int o = 32; o > 0; o >>= 1) {
    m = max(m, __shfl_xor(m, o));
    open = max(open, __shfl_xor(open, o));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = m;
    red[1][threadIdx.x >> 6] = open;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      m = max(m, red[0][w]);
      open = max(open, red[1][w]);
    }
    atomicMax(&res[0], m);
    if (open) atomicMax(&res[1], 1);
  }
}

// One level of the bottom-up refit: every node at depth `level` merges its
// children, which are leaves or nodes of the level below (written by the
// previous launch, so no fences are needed).
__global__ void k_refit_level(int32_t nf, int32_t level, const int32_t* __restrict__ dep,
                              const int32_t* __restrict__ left, const int32_t* __restrict__ right,
                              const float4* __restrict__ lbox, const float* __restrict__ lz, float4* ibox, float* iz,
                              BvhNode* __restrict__ nodes) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nf - 1 || dep[node] != level) return;
  const int32_t lc = left[node], rc = right[node];
  if (lc >= nf - 1 || rc >= nf - 1 || ~lc >= nf || ~rc >= nf) return;
  float4 bl, br;
  float zl, zr;
  if (lc < 0) { bl = lbox[~lc]; zl = lz[~lc]; }
  else { bl = ibox[lc]; zl = iz[lc]; }
  if (rc < 0) { br = lbox[~rc]; zr = lz[~rc]; }
  else { br = ibox[rc]; zr = iz[rc]; }
  BvhNode nd;
  nd.lbox = bl;
  nd.rbox = br;
  nd.lzmax = zl;
  nd.rzmax = zr;
  nd.left = lc;
  nd.right = rc;
  nodes[node] = nd;
  ibox[node] = make_float4(fminf(bl.x, br.x), fmaxf(bl.y, br.y), fminf(bl.z, br.z), fmaxf(bl.w, br.w));
  iz[node] = fmaxf(zl, zr);
}

// ---------------------------------------------------------------------------
// Four-wide tree
// ---------------------------------------------------------------------------

// One child slot of a four-wide node before quantisation.
struct Slot4 {
  float4 box;
  float z;
  int32_t ref;
};

// Grid of one axis of a four-wide node whose children span [lo, hi]: the
// inverse cell size i = 2^-e and the offset m of grid_cell, with cell(lo) >= 0
// and cell(hi) <= 255, so that by monotonicity every bound of a child has a
// cell in [0, 255].  e is the smallest exponent that fits the span in 256
// cells, and at least such that m = -lo i stays far inside float32's range;
// where m's rounding would put lo in cell -1, m is raised by an ulp.
__device__ __forceinline__ void axis_grid(float lo, float hi, float& i, float& m) {
  const double r = ((double)hi - (double)lo) / 255.0;
  int e = -126;
  if (r > 0.0) {
    int k;
    frexp(r, &k);            // r < 2^k
    e = max(k - 1, -126);    // start one below, the loop settles it
  }
  if (lo != 0.0f) {
    int k;
    frexp((double)lo, &k);   // |lo| < 2^k
    e = max(e, k - 100);     // |m| < 2^100
  }
  for (;; ++e) {
    i = __uint_as_float((uint32_t)(127 - e) << 23);
    m = __fmul_rn(-lo, i);
    while (grid_cell(lo, i, m) < 0.0f) m = nextafterf(m, INFINITY);
    if (e >= 126 || grid_cell(hi, i, m) <= 255.0f) break;
  }
}

// Four-wide node for every binary node at even depth: its children, with an
// internal child replaced by that child's two children.  A slot whose box
// can hold no point (a NaN or an empty range, as in unwritten nodes of a
// malformed tree) stays unoccupied, as the binary test never enters it.
__global__ void k_collapse4(int32_t nf, const int32_t* __restrict__ dep, const BvhNode* __restrict__ nodes,
                            const TriRec* __restrict__ tris, BvhNode4* __restrict__ out) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t nint = nf - 1;
  if (node >= nint || (dep[node] & 1)) return;
  const BvhNode nd = nodes[node];
  Slot4 sl[4];
  int n = 0;
  const int32_t cref[2] = {nd.left, nd.right};
  const float4 cbox[2] = {nd.lbox, nd.rbox};
  const float cz[2] = {nd.lzmax, nd.rzmax};
  for (int k = 0; k < 2; ++k) {
    const int32_t c = cref[k];
    if (c < 0 || c >= nint) {
      // a leaf, or an index out of range that the traversal reports
      sl[n++] = Slot4{cbox[k], cz[k], c};
    } else {
      const BvhNode cn = nodes[c];
      sl[n++] = Slot4{cn.lbox, cn.lzmax, cn.left};
      sl[n++] = Slot4{cn.rbox, cn.rzmax, cn.right};
    }
  }
  unsigned mask = 0;
  float x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY, z0 = INFINITY, z1 = -INFINITY;
  for (int k = 0; k < n; ++k) {
    const float4 b = sl[k].box;
    if (!(b.x <= b.y && b.z <= b.w && sl[k].z == sl[k].z)) continue;
    mask |= 1u << k;
    x0 = fminf(x0, b.x);
    x1 = fmaxf(x1, b.y);
    y0 = fminf(y0, b.z);
    y1 = fmaxf(y1, b.w);
    z0 = fminf(z0, sl[k].z);
    z1 = fmaxf(z1, sl[k].z);
  }
  BvhNode4 q;
  q.ties = 0u;
  for (int k = 0; k < 4; ++k) {
    q.child[k] = k < n ? sl[k].ref : -1;
    if (q.child[k] < 0) q.ties |= 1u << (12 + k);
    if (k < n && sl[k].ref < 0 && ~sl[k].ref < nf) q.ties |= (tris[~sl[k].ref].ties & 7u) << (3 * k);
  }
  q.xlo = q.xhi = q.ylo = q.yhi = q.zhi = 0u;
  q.ix = q.iy = q.iz = 1.0f;
  q.mx = q.my = q.mz = 0.0f;
  if (mask != 0) {
    axis_grid(x0, x1, q.ix, q.mx);
    axis_grid(y0, y1, q.iy, q.my);
    axis_grid(z0, z1, q.iz, q.mz);
  }
  for (int k = 0; k < 4; ++k) {
    if (!((mask >> k) & 1u)) {
      q.xlo |= 0xffu << (8 * k);   // xlo 255 > xhi 0: no cell passes
      continue;
    }
    const float4 b = sl[k].box;
    // cells in [0, 255] (axis_grid), exact as integers
    q.xlo |= (uint32_t)grid_cell(b.x, q.ix, q.mx) << (8 * k);
    q.xhi |= (uint32_t)grid_cell(b.y, q.ix, q.mx) << (8 * k);
    q.ylo |= (uint32_t)grid_cell(b.z, q.iy, q.my) << (8 * k);
    q.yhi |= (uint32_t)grid_cell(b.w, q.iy, q.my) << (8 * k);
    q.zhi |= (uint32_t)grid_cell(sl[k].z, q.iz, q.mz) << (8 * k);
  }
  out[node] = q;
}

__global__ void k_fill_u32(unsigned* p, int64_t n, unsigned v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t build_bvh_device(const BuildBufs& b, const Frame& F, const float* V, int32_t nv,
                            const int32_t* Fc, int32_t nf, float pad, hipStream_t s) {
  hipError_t e;
  const unsigned bv = (unsigned)((nv + 255) / 256);
  const unsigned bf = (unsigned)((nf + 255) / 256);
  if (nv > 0) {
    hipLaunchKernelGGL(k_rotate_vertices, dim3(bv), dim3(256), 0, s, F, V, nv, b.Vr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (nf == 0) return hipSuccess;
  unsigned init[4] = {0xffffffffu, 0u, 0xffffffffu, 0u};
  for (int k = 0; k < 4; ++k)
    if ((e = fill_u32(b.cbounds + k, 1, init[k], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_boxes, dim3(bf), dim3(256), 0, s, b.Vr, Fc, nf, pad, b.box, b.zmax, b.cen);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cen_bounds, dim3(std::min<unsigned>(bf, kReduceBlocks)), dim3(256), 0, s, b.cen, nf,
                     b.cbounds);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_morton, dim3(bf), dim3(256), 0, s, b.cen, nf, b.cbounds, b.keys, b.vals);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = radix_sort_pairs(b.keys, b.vals, b.keys2, b.vals2, nf, b.sort_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather_leaves, dim3(bf), dim3(256), 0, s, Fc, b.vals, nf, b.box, b.zmax, b.Vr,
                     b.tris, b.leafbox, b.leafz);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nf == 1) return hipSuccess;
  if ((e = fill_u32((unsigned*)b.parent_leaf, nf, 0xffffffffu, s)) != hipSuccess) return e;
  if ((e = fill_u32((unsigned*)b.parent_int, nf - 1, 0xffffffffu, s)) != hipSuccess) return e;
  // unwritten nodes would read as NaN boxes (never entered)
  if ((e = fill_u32((unsigned*)b.nodes, (int64_t)(nf - 1) * (sizeof(BvhNode) / 4), 0xffffffffu, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_karras, dim3(bf), dim3(256), 0, s, b.keys, nf, b.left, b.right,
                     b.parent_int, b.parent_leaf);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // node depths (the sort and Morton buffers are free by now), then the
  // refit one level per launch, deepest first
  const int32_t ni = nf - 1;
  const unsigned bi = (unsigned)((ni + 255) / 256);
  int32_t* anc[2] = {(int32_t*)b.keys2, b.flags};
  int32_t* dep[2] = {b.vals2, (int32_t*)b.keys};
  hipLaunchKernelGGL(k_depth_init, dim3(bi), dim3(256), 0, s, b.parent_int, ni, anc[0], dep[0]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // a Karras tree over 64-bit (key, index) codes is at most 64 levels deep:
  // 7 rounds reach the root from every node
  int cur = 0;
  for (int r = 0; r < 7; ++r, cur ^= 1) {
    hipLaunchKernelGGL(k_depth_jump, dim3(bi), dim3(256), 0, s, anc[cur], dep[cur], ni, anc[cur ^ 1], dep[cur ^ 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  int32_t* res = (int32_t*)b.cbounds;
  if ((e = fill_u32(b.cbounds, 2, 0u, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_depth_max, dim3(std::min<unsigned>(bi, kReduceBlocks)), dim3(256), 0, s, anc[cur], dep[cur],
                     ni, res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int32_t hres[2] = {0, 0};
  if ((e = hipMemcpyAsync(hres, res, sizeof hres, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if (hres[1] != 0 || hres[0] < 0 || hres[0] > 128) return hipErrorUnknown;
  for (int level = hres[0]; level >= 0; --level) {
    hipLaunchKernelGGL(k_refit_level, dim3(bi), dim3(256), 0, s, nf, level, dep[cur], b.left, b.right, b.leafbox,
                       b.leafz, b.ibox, b.iz, b.nodes);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = fill_u32((unsigned*)b.nodes4, (int64_t)ni * (sizeof(BvhNode4) / 4), 0xffffffffu, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_collapse4, dim3(bi), dim3(256), 0, s, nf, dep[cur], b.nodes, b.tris, b.nodes4);
  return hipGetLastError();
}

}  // namespace wn
