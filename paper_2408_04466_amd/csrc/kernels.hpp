// Kernel argument structures and launch helpers shared by the host API and
// the kernels (plain structs passed by value as kernel arguments).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.hpp"
#include "wn.h"

namespace wn {

// Boundary loops of one call: loop l covers vertices [off[l], off[l+1]).  Up
// to WN_MAX_LOOPS loops travel in the kernel arguments; a longer table is
// read from device memory (dev, [n + 1]; null otherwise).
struct LoopTable {
  int32_t n;
  const int32_t* dev;
  int32_t off[WN_MAX_LOOPS + 1];
};

// Binary BVH node of the build: the boxes of both children (projected x/y
// range and the largest coordinate along d) and the children (>= 0 internal
// node index, < 0 leaf ~index into the sorted triangle array).  48 bytes.
struct alignas(16) BvhNode {
  float4 lbox;   // xmin, xmax, ymin, ymax of the left child
  float4 rbox;   // same for the right child
  float lzmax, rzmax;
  int32_t left, right;
};

// Four-wide BVH node, the tree that the traversals walk: the binary tree
// with every second level folded into its parent, so that a node holds up to
// four children (its binary children, or theirs where a binary child is
// internal) and a query needs half the dependent node loads.  The children's
// boxes are 8-bit cells of an integer grid of the node: along each axis a
// coordinate v lies in cell floor(fma(v, i, m)) (grid_cell; i a power of
// two), and a child stores the cells of its float box's bounds, computed with
// that same function.  The function is monotone in v, so every point of the
// box has its cells between the stored ones: a query computes its three
// cells once per node and then needs one comparison per bound, with no
// decoding of the children's bounds.  64 bytes, one aligned half cache line.  Nodes
// keep the index of their binary node (the array is sparse: only binary nodes
// at even depth are written).
struct alignas(64) BvhNode4 {
  float ix, mx, iy, my, iz, mz;  // per axis the grid cell_i(v) = floor(fma(v, i, m)), cells 0..255 spanning the children
  uint32_t xlo, xhi;      // byte k: child k's cells of xmin and xmax (an empty slot: 255 and 0, which no cell passes)
  uint32_t ylo, yhi;
  uint32_t zhi;           // byte k: child k's cell of zmax
  int32_t child[4];       // >= 0 node index, < 0 leaf ~index into the sorted triangles
  uint32_t ties;          // bits 3k..3k+2: the edge tie signs of leaf child k (TriRec::ties); bit 12 + k: child k is a leaf
};
static_assert(sizeof(BvhNode4) == 64, "four-wide node is 64 bytes");

// Sorted triangle of the traversal, one aligned 128-byte line: the three
// rotated vertices as float32 (hi, lo) pairs.  The first three words hold
// what the projected inside test reads for every triangle the traversal
// reaches (x and y; the tree's nodes carry the edges' tie signs too); the
// heights follow, read only when the line passes through the triangle.
struct alignas(128) TriRec {
  float4 xy[3];           // vertex k: xh, xl, yh, yl
  float zch, zcl;         // zh, zl of v2
  uint32_t ties;          // bit e set: edge e (v0v1, v1v2, v2v0) starts at the lexicographically smaller vertex
  int32_t face;           // index of the triangle in the input
  float4 zab;             // zh, zl of v0 and v1
  uint32_t pad[12];
};
static_assert(sizeof(TriRec) == 128, "triangle record is one 128-byte line");

struct CrossArgs {
  Frame F;
  const BvhNode4* nodes;
  const TriRec* tris;      // sorted triangles
  const float4* leafbox;   // used when the tree is a single leaf
  const float* leafz;
  int32_t nf;
  const float* qx;
  const float* qy;
  const float* qz;
  int64_t nq;
  int32_t* chi;
};

struct BndArgs {
  Frame F;
  const float* bnd;        // [nb][3]
  int32_t nb;
  const float* qx;
  const float* qy;
  const float* qz;
  int64_t nq;
  const int32_t* chi_in;   // may alias w_out
  float* w_out;
};

struct AdjArgs {
  const float* bnd;
  int32_t nb;
  const float* qx;
  const float* qy;
  const float* qz;
  int64_t nq;
  const float* gw;
  float* gq;               // [nq][3] or null
  float* partial;          // [rows][nb][3] or null (rows = workgroups * 4)
  float* partial_loop;     // [rows][nloops][3] (with partial)
};

// host-side launchers (defined next to their kernels)
hipError_t launch_bnd3d(const BndArgs& a, const LoopTable& L, hipStream_t s);
// Fused crossing count + boundary integral (chi_out may be null).
hipError_t launch_fwd3d(const CrossArgs& c, const BndArgs& a, const LoopTable& L, int32_t* chi_out,
                        hipStream_t s);
hipError_t launch_cross3d(const CrossArgs& a, hipStream_t s);
// 3D grid mode (grid3d.hip): fused forward per query, z fastest.
hipError_t launch_patches3d(const Frame& F, const float* nets, int64_t np, const float* qx, const float* qy,
                            const float* qz, int64_t nq, int32_t* chi_out, hipStream_t s);
// Parametric surfaces (bicubic patches + boundary curves) with their own
// directions and query ranges, evaluated in one launch (psurf.hip).  The
// surfaces' patches, curves and queries are consecutive in the arrays.
struct PSurf {
  Frame F;                          // frame of the surface's direction, centre 0
  int64_t patch0, curve0, q0, blk0; // first patch, curve, query and workgroup
  int64_t nq;
  int32_t npatch, ncurve;
};
struct PBatch {
  int32_t nsurf = 0;
  int64_t npatch = 0, ncurve = 0, nq = 0, nblocks = 0;
  unsigned char* ws = nullptr;      // the one allocation: descriptors | block -> surface
  PSurf* desc = nullptr;
  int32_t* blk_surf = nullptr;
  ~PBatch();
};
// surfs: F, nq, npatch, ncurve filled in; the offsets are computed here.
hipError_t pbatch_create(const PSurf* surfs, int32_t n, hipStream_t s, PBatch* b);
hipError_t eval_pbatch(const PBatch& b, const float* nets, const float* curves, const float* qx, const float* qy,
                       const float* qz, float* w_out, int32_t* chi_out, hipStream_t s);
// One parametric surface (frame centre 0) through the same kernel: w, and chi
// when chi_out is not null.
hipError_t launch_psurf_single(const Frame& F, const float* nets, int64_t np, const float* curves, int64_t nc,
                               const float* qx, const float* qy, const float* qz, int64_t nq, float* w_out,
                               int32_t* chi_out, hipStream_t s);
// Counts over a call's outputs (diag.hip): counts[0] = non-finite queries,
// counts[1] = finite queries whose chi is WN_CHI_INVALID.
hipError_t diagnose(const float* qx, const float* qy, const float* qz, const int32_t* chi, int64_t n,
                    int64_t* counts, hipStream_t s);
// Morton-order permutation of the queries (order.hip).
hipError_t spatial_order(const float* qx, const float* qy, const float* qz, int64_t n, int32_t* order,
                         hipStream_t s);
// Sorted copies of a query set in a coarse Morton order (32^3 cells; order.hip),
// for the kernels whose lanes diverge on random query orders: order, the
// sorted coordinates (and loss weights g when given) and out_words float32 or
// int32 words per query of output space, all in one stream-ordered
// allocation released by the destructor (on the same stream).
struct SortedQueries {
  unsigned char* ws = nullptr;
  hipStream_t stream = nullptr;
  int32_t* order = nullptr;
  float *x = nullptr, *y = nullptr, *z = nullptr, *g = nullptr;
  uint32_t* out = nullptr;
  size_t block_words = 0;   // out_block(k): the k-th output array of n words
  uint32_t* out_block(int k) const { return out + (size_t)k * block_words; }
  ~SortedQueries();
};
hipError_t sort_queries(const float* qx, const float* qy, const float* qz, const float* gw, int64_t n, int out_words,
                        hipStream_t s, SortedQueries* o);
// dst row order[i] = src row i (rows of `width` 32-bit words).
hipError_t scatter_rows(const void* src, const int32_t* order, int64_t n, int width, void* dst, hipStream_t s);
// Query count from which the curve adjoint and the parametric path sort
// their queries first.
constexpr int64_t kSortQueriesMin = 1 << 16;
hipError_t backward_curves(const float* ctrl, int64_t nc, const float* qx, const float* qy, const float* qz,
                           int64_t nq, const float* gw, float* gq, float* gc, hipStream_t s);
hipError_t launch_curves3d(const CrossArgs& c, const float* ctrl, int64_t nc, const int32_t* chi_in, float* w_out,
                           int32_t* chi_out, hipStream_t s);
hipError_t launch_grid3d_fwd(const CrossArgs& c, const BndArgs& a, const LoopTable& L, const float* gx,
                             const float* gy, const float* gz, int64_t nx, int64_t ny, int64_t nz, int32_t* chi_out,
                             hipStream_t s);
int adj3d_qpl(int64_t nq);   // queries per lane the plain adjoint uses for nq queries
hipError_t launch_adj3d(const AdjArgs& a, const LoopTable& L, int64_t nblocks, int qpl, hipStream_t s);
int64_t adj3d_blocks(int64_t nq, int qpl);
int64_t adj3d_rows(int64_t nblocks);
int64_t reduce_groups(int64_t rows);
hipError_t backward_2d(int32_t dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                       const uint8_t* closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                       int64_t nx, int64_t ny, const void* gw, void* gq, void* gc, hipStream_t s);
// Most columns one workgroup of the 2D grid mode handles (wider rows are split
// into even tiles).
constexpr int kGridColTile2D = 4096;
// Batched 2D: sets with at most kRowPieces2D monotone pieces (3 per segment)
// run one wavefront per row tile of at most kRowColTile2D columns.
constexpr int kRowPieces2D = 64;
constexpr int kRowColTile2D = 512;
constexpr int kRowsPerWave2D = 8;   // rows per wavefront item (fewer if pieces x rows > 64)
// Most work items of one 2D batch launch (a launch holds fewer than 2^32
// work-items): 2^24 workgroup items, 2^26 wavefront items.
constexpr int64_t kMaxItemsG2D = (int64_t)1 << 24;
constexpr int64_t kMaxItemsW2D = (int64_t)1 << 26;
// A 2D batch: the set descriptors and loop tables on the device, and room
// for the monotone pieces of every segment.
struct Batch2D {
  int32_t dtype = 0;
  int32_t nsets_g = 0, nsets_w = 0;    // sets on the workgroup / wavefront kernel
  int64_t nseg = 0, nx = 0, ny = 0, nout = 0;
  int64_t items_g = 0, items_w = 0;    // (row, column tile) items of each kernel
  size_t lds = 0;
  unsigned char* ws = nullptr;   // the one allocation below
  unsigned char* desc_g = nullptr;
  unsigned char* desc_w = nullptr;
  unsigned char* loop_off = nullptr;
  unsigned char* loop_closed = nullptr;
  unsigned char* blk_set = nullptr;
  unsigned char* pieces = nullptr;
  ~Batch2D();
};
hipError_t batch2d_create(int32_t dtype, const wn_curveset_2d* sets, int32_t nsets, hipStream_t s, Batch2D* b);
hipError_t eval_2d_batched(const Batch2D& b, const void* ctrl, const void* x, const void* y, void* w, int32_t* chi,
                           hipStream_t s);
hipError_t eval_2d(int32_t dtype, const void* ctrl, int64_t nseg, const int64_t* loop_off,
                   const uint8_t* closed, int32_t nloops, int32_t kind, const void* x, const void* y,
                   int64_t nx, int64_t ny, void* w, int32_t* chi, hipStream_t s);
hipError_t launch_reduce_partials(const float* pv, const float* pl, int64_t rows, int32_t nb,
                                  const LoopTable& L, double* tmp, float* out, hipStream_t s);

}  // namespace wn
