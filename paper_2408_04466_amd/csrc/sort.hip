// Least-significant-digit radix sort of (uint32 key, int32 value) pairs,
// 8 bits per pass, stable, deterministic.
//
// Per pass: (1) every tile of kTile keys counts its digits in LDS and writes
// the counts digit-major, hist[d * ntiles + tile]; (2) an exclusive scan of
// that array gives every (digit, tile) its first output slot; (3) every tile
// sorts itself stably by the digit with eight one-bit splits in LDS and
// writes each key to  slot(d, tile) + (local position - local start of d).
#include "bvh_build.hpp"

namespace wn {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;   // 2048

// Exclusive scan of one value per thread over a 256-thread block; returns the
// block total through `total`.
__device__ __forceinline__ unsigned block_excl_scan(unsigned v, unsigned* total, unsigned* sm) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  unsigned x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sm[wave] = x;
  __syncthreads();
  unsigned off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const unsigned s = sm[w];
    if (w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ __launch_bounds__(kThreads) void k_hist(const unsigned* __restrict__ keys, int64_t n,
                                                   int shift, unsigned* __restrict__ hist,
                                                   int64_t ntiles) {
  __shared__ unsigned cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int j = 0; j < kItems; ++j) {
    const int64_t i = base + (int64_t)j * kThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// scan phase 1: per-chunk sums (chunks of kTile entries)
__global__ __launch_bounds__(kThreads) void k_scan_sums(const unsigned* __restrict__ in, int64_t n,
                                                        unsigned* __restrict__ sums) {
  __shared__ unsigned sm[4];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  unsigned s = 0;
  for (int j = 0; j < kItems; ++j)
    if (base + j < n) s += in[base + j];
  unsigned tot;
  block_excl_scan(s, &tot, sm);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// scan phase 2: one block scans the chunk sums in place (looping)
__global__ __launch_bounds__(kThreads) void k_scan_top(unsigned* sums, int64_t m) {
  __shared__ unsigned sm[4];
  unsigned carry = 0;
  for (int64_t c = 0; c < m; c += kThreads) {
    const int64_t i = c + threadIdx.x;
    const unsigned v = i < m ? sums[i] : 0u;
    unsigned tot;
    const unsigned ex = block_excl_scan(v, &tot, sm);
    if (i < m) sums[i] = carry + ex;
    carry += tot;
  }
}

// scan phase 3: exclusive scan inside each chunk plus the chunk offset
__global__ __launch_bounds__(kThreads) void k_scan_apply(const unsigned* __restrict__ in, int64_t n,
                                                         const unsigned* __restrict__ sums,
                                                         unsigned* __restrict__ out) {
  __shared__ unsigned sm[4];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  unsigned v[kItems];
  unsigned s = 0;
  for (int j = 0; j < kItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0u;
    s += v[j];
  }
  unsigned tot;
  unsigned run = sums[blockIdx.x] + block_excl_scan(s, &tot, sm);
  for (int j = 0; j < kItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
}

__global__ __launch_bounds__(kThreads) void k_scatter(const unsigned* __restrict__ kin,
                                                      const int32_t* __restrict__ vin, int64_t n,
                                                      int shift, const unsigned* __restrict__ offs,
                                                      int64_t ntiles, unsigned* __restrict__ kout,
                                                      int32_t* __restrict__ vout) {
  __shared__ unsigned sk[kTile];
  __shared__ int32_t svl[kTile];
  __shared__ unsigned cnt[256];
  __shared__ unsigned sm[4];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  const int64_t valid = min((int64_t)kTile, n - base);
  cnt[threadIdx.x] = 0;
  // load in order: thread t owns local positions [t*kItems, t*kItems + kItems)
  unsigned k[kItems];
  int32_t v[kItems];
  for (int j = 0; j < kItems; ++j) {
    const int p = threadIdx.x * kItems + j;
    if (p < valid) { k[j] = kin[base + p]; v[j] = vin[base + p]; }
    else { k[j] = 0xffffffffu; v[j] = -1; }   // padding sorts last, never written
  }
  __syncthreads();
  for (int j = 0; j < kItems; ++j)
    if (threadIdx.x * kItems + j < valid) atomicAdd(&cnt[(k[j] >> shift) & 255u], 1u);
  // stable local sort by the 8-bit digit: eight one-bit splits
  for (int b = 0; b < 8; ++b) {
    unsigned ones = 0;
    for (int j = 0; j < kItems; ++j) ones += (k[j] >> (shift + b)) & 1u;
    unsigned tot;
    const unsigned before = block_excl_scan(ones, &tot, sm);
    const unsigned zeros = kTile - tot;
    unsigned o = before;
    for (int j = 0; j < kItems; ++j) {
      const int p = threadIdx.x * kItems + j;
      const unsigned bit = (k[j] >> (shift + b)) & 1u;
      const int np = bit ? (int)(zeros + o) : (int)(p - o);
      o += bit;
      sk[np] = k[j];
      svl[np] = v[j];
    }
    __syncthreads();
    for (int j = 0; j < kItems; ++j) {
      const int p = threadIdx.x * kItems + j;
      k[j] = sk[p];
      v[j] = svl[p];
    }
    __syncthreads();
  }
  // local start of each digit
  unsigned tot;
  const unsigned c = cnt[threadIdx.x];
  const unsigned st = block_excl_scan(c, &tot, sm);
  __syncthreads();
  cnt[threadIdx.x] = st;
  __syncthreads();
  for (int j = 0; j < kItems; ++j) {
    const int p = threadIdx.x * kItems + j;
    if (p < valid) {
      const unsigned d = (k[j] >> shift) & 255u;
      const int64_t dst = (int64_t)offs[(int64_t)d * ntiles + blockIdx.x] + (p - (int64_t)cnt[d]);
      if (dst >= 0 && dst < n) {
        kout[dst] = k[j];
        vout[dst] = v[j];
      }
    }
  }
}

hipError_t scan_excl(const unsigned* in, unsigned* out, int64_t n, unsigned* sums, hipStream_t s) {
  const int64_t chunks = (n + kTile - 1) / kTile;
  if (chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)chunks), dim3(kThreads), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, s, sums, chunks);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)chunks), dim3(kThreads), 0, s, in, n, sums, out);
  return hipGetLastError();
}

}  // namespace

size_t radix_sort_tmp_bytes(int64_t n) {
  const int64_t ntiles = (n + kTile - 1) / kTile;
  const int64_t m = 256 * ntiles;
  const int64_t chunks = (m + kTile - 1) / kTile;
  return (size_t)(2 * m + chunks + 64) * sizeof(unsigned);
}

hipError_t radix_sort_pairs(unsigned* keys, int32_t* vals, unsigned* keys_alt, int32_t* vals_alt,
                            int64_t n, void* tmp, hipStream_t s, int passes) {
  if (n <= 1) return hipSuccess;
  const int64_t ntiles = (n + kTile - 1) / kTile;
  const int64_t m = 256 * ntiles;
  unsigned* hist = (unsigned*)tmp;
  unsigned* offs = hist + m;
  unsigned* sums = offs + m;
  unsigned* ka = keys;
  int32_t* va = vals;
  unsigned* kb = keys_alt;
  int32_t* vb = vals_alt;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)ntiles), dim3(kThreads), 0, s, ka, n, shift, hist, ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = scan_excl(hist, offs, m, sums, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)ntiles), dim3(kThreads), 0, s, ka, va, n, shift,
                       offs, ntiles, kb, vb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    unsigned* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  // an even number of passes: the result is back in (keys, vals)
  return hipSuccess;
}

}  // namespace wn
