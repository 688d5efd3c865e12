// Spatial order of query points.
//
// The per-query kernels run one query per lane, so a wavefront is as fast as
// its slowest lane: random query sets make neighbouring lanes walk different
// BVH paths and different numbers of curve or patch panels.  Sorting the
// queries once by their Morton codes (10 bits per axis over the queries'
// bounding box) puts spatially close queries in the same wavefront.  The sort
// is the stable LSD radix sort of the BVH build, so the order is
// deterministic (ties by query index); non-finite queries go last.
#include <algorithm>

#include "bvh_build.hpp"
#include "kernels.hpp"

namespace wn {

namespace {

__device__ __forceinline__ unsigned ord_key(float f) {
  const unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord_float(unsigned o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// Bounding box of the finite queries as order-preserving integers:
// box[2c] = min, box[2c + 1] = max of coordinate c.  A grid-stride loop over
// few workgroups, wavefront shuffles, then one atomic per value and
// workgroup, so that the atomics on the six words do not serialise.
constexpr int kBoxBlocks = 256;

__global__ __launch_bounds__(256) void k_qbox(const float* __restrict__ qx, const float* __restrict__ qy,
                                              const float* __restrict__ qz, int64_t n, unsigned* __restrict__ box) {
  __shared__ unsigned red[6][4];
  unsigned v[6] = {0xffffffffu, 0u, 0xffffffffu, 0u, 0xffffffffu, 0u};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float p[3] = {qx[i], qy[i], qz[i]};
    if (isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))
      for (int c = 0; c < 3; ++c) {
        const unsigned k = ord_key(p[c]);
        v[2 * c] = min(v[2 * c], k);
        v[2 * c + 1] = max(v[2 * c + 1], k);
      }
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int c = 0; c < 3; ++c) {
      v[2 * c] = min(v[2 * c], (unsigned)__shfl_xor((int)v[2 * c], o, 64));
      v[2 * c + 1] = max(v[2 * c + 1], (unsigned)__shfl_xor((int)v[2 * c + 1], o, 64));
    }
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    unsigned r = red[k][0];
    for (int w = 1; w < 4; ++w) r = (k % 2 == 0) ? min(r, red[k][w]) : max(r, red[k][w]);
    if (k % 2 == 0) atomicMin(&box[k], r);
    else atomicMax(&box[k], r);
  }
}

__device__ __forceinline__ unsigned spread10(unsigned x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// Morton code of the query's cell in a (2^bits)^3 grid over the box
// (bits <= 10), or 0xffffffff for a non-finite query.
__global__ void k_qmorton(const float* __restrict__ qx, const float* __restrict__ qy, const float* __restrict__ qz,
                          int64_t n, const unsigned* __restrict__ box, int bits, unsigned* __restrict__ keys,
                          int32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float p[3] = {qx[i], qy[i], qz[i]};
  vals[i] = (int32_t)i;
  if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) {
    keys[i] = 0xffffffffu;
    return;
  }
  unsigned code = 0;
  for (int c = 0; c < 3; ++c) {
    const float lo = ord_float(box[2 * c]), hi = ord_float(box[2 * c + 1]);
    const float ext = hi - lo;
    const float t = ext > 0.f ? (p[c] - lo) / ext : 0.f;
    const float cells = (float)(1u << bits);
    const unsigned cell = (unsigned)fminf(fmaxf(t * cells, 0.f), cells - 1.f);
    code |= spread10(cell) << c;
  }
  keys[i] = code;
}

// dst row order[i] = src row i, rows of `width` 32-bit words.
__global__ void k_scatter_rows(const uint32_t* __restrict__ src, const int32_t* __restrict__ order, int64_t n,
                               int width, uint32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = order[i];
  for (int c = 0; c < width; ++c) dst[r * width + c] = src[i * width + c];
}

// Sorted copies: x[i] = qx[order[i]] (and g[i] = gw[order[i]] when gw is set).
__global__ void k_gather_queries(const float* __restrict__ qx, const float* __restrict__ qy,
                                 const float* __restrict__ qz, const float* __restrict__ gw,
                                 const int32_t* __restrict__ order, int64_t n, float* __restrict__ x,
                                 float* __restrict__ y, float* __restrict__ z, float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = order[i];
  x[i] = qx[r];
  y[i] = qy[r];
  z[i] = qz[r];
  if (gw) g[i] = gw[r];
}

hipError_t order_by_cells(const float* qx, const float* qy, const float* qz, int64_t n, int32_t* order, int bits,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t b_box = up(6 * sizeof(unsigned));
  const size_t b_keys = up((size_t)n * sizeof(unsigned));
  const size_t b_tmp = up(radix_sort_tmp_bytes(n));
  unsigned char* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, b_box + 3 * b_keys + b_tmp, s);
  if (e != hipSuccess) return e;
  unsigned* box = (unsigned*)ws;
  unsigned* keys = (unsigned*)(ws + b_box);
  unsigned* keys2 = (unsigned*)(ws + b_box + b_keys);
  int32_t* vals2 = (int32_t*)(ws + b_box + 2 * b_keys);
  void* tmp = ws + b_box + 3 * b_keys;
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    e = fill_u32(box + 2 * c, 1, 0xffffffffu, s);
    if (e == hipSuccess) e = fill_u32(box + 2 * c + 1, 1, 0u, s);
  }
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (e == hipSuccess) {
    const unsigned bb = (unsigned)std::min<int64_t>((n + 255) / 256, kBoxBlocks);
    hipLaunchKernelGGL(k_qbox, dim3(bb), dim3(256), 0, s, qx, qy, qz, n, box);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_qmorton, dim3(blocks), dim3(256), 0, s, qx, qy, qz, n, box, bits, keys, order);
    e = hipGetLastError();
  }
  // 3 * bits code bits in whole bytes, an even number of passes
  const int passes = ((3 * bits + 15) / 16) * 2;
  if (e == hipSuccess) e = radix_sort_pairs(keys, order, keys2, vals2, n, tmp, s, passes);
  const hipError_t e2 = hipFreeAsync(ws, s);
  return e != hipSuccess ? e : e2;
}

}  // namespace

hipError_t spatial_order(const float* qx, const float* qy, const float* qz, int64_t n, int32_t* order,
                         hipStream_t s) {
  return order_by_cells(qx, qy, qz, n, order, 10, s);
}

SortedQueries::~SortedQueries() {
  if (ws) (void)hipFreeAsync(ws, stream);
}

hipError_t sort_queries(const float* qx, const float* qy, const float* qz, const float* gw, int64_t n, int out_words,
                        hipStream_t s, SortedQueries* o) {
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t b = up((size_t)n * sizeof(float));
  const size_t bytes = 4 * b + (gw ? b : 0) + (size_t)out_words * b;
  hipError_t e = hipMallocAsync((void**)&o->ws, bytes, s);
  if (e != hipSuccess) {
    o->ws = nullptr;
    return e;
  }
  o->stream = s;
  unsigned char* p = o->ws;
  o->order = (int32_t*)p;
  o->x = (float*)(p + b);
  o->y = (float*)(p + 2 * b);
  o->z = (float*)(p + 3 * b);
  o->g = gw ? (float*)(p + 4 * b) : nullptr;
  o->out = (uint32_t*)(p + (gw ? 5 : 4) * b);
  o->block_words = b / sizeof(uint32_t);
  // 32^3 cells: two radix passes; about 32 queries per cell at 2^20 queries
  e = order_by_cells(qx, qy, qz, n, o->order, 5, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather_queries, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, qx, qy, qz, gw, o->order, n,
                     o->x, o->y, o->z, o->g);
  return hipGetLastError();
}

hipError_t scatter_rows(const void* src, const int32_t* order, int64_t n, int width, void* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const uint32_t*)src, order, n,
                     width, (uint32_t*)dst);
  return hipGetLastError();
}

}  // namespace wn
