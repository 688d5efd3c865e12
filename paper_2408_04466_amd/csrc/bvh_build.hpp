// Device buffers and helpers of the BVH build.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace wn {

constexpr int kShortStack = 8;    // traversal stack entries kept in registers

struct BuildBufs {
  RPt* Vr;              // [nv]
  float4* box;          // [nf] projected boxes (input order)
  float* zmax;          // [nf]
  float2* cen;          // [nf]
  unsigned* cbounds;    // [4] centroid bounds (ordered ints)
  unsigned* keys;       // [nf]
  int32_t* vals;        // [nf]
  unsigned* keys2;      // [nf]
  int32_t* vals2;       // [nf]
  void* sort_tmp;       // radix_sort_tmp_bytes(nf)
  TriRec* tris;         // [nf] sorted triangle records
  float4* leafbox;      // [nf]
  float* leafz;         // [nf]
  int32_t* left;        // [nf-1]
  int32_t* right;       // [nf-1]
  int32_t* parent_int;  // [nf-1]
  int32_t* parent_leaf; // [nf]
  float4* ibox;         // [nf-1] node bounds
  float* iz;            // [nf-1]
  int32_t* flags;       // [nf-1]
  BvhNode* nodes;       // [nf-1] binary tree
  BvhNode4* nodes4;     // [nf-1] four-wide tree (written at even depths)
};

size_t radix_sort_tmp_bytes(int64_t n);
// Stable LSD radix sort on the low 8 * passes bits of the keys (passes even:
// the result ends in keys, vals).
hipError_t radix_sort_pairs(unsigned* keys, int32_t* vals, unsigned* keys_alt, int32_t* vals_alt,
                            int64_t n, void* tmp, hipStream_t s, int passes = 4);
hipError_t fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t s);
hipError_t build_bvh_device(const BuildBufs& b, const Frame& F, const float* V, int32_t nv,
                            const int32_t* Fc, int32_t nf, float pad, hipStream_t s);

}  // namespace wn
