// Adjoint launchers for small query counts: the boundary is split into
// ranges of whole LDS chunks, one range per workgroup row of the grid, so
// that few query tiles still fill the chip.
#pragma once

#include "kernels.hpp"

namespace wn {

// Queries per lane (1, 2 or 4) for nq queries over nb boundary vertices.
int adj3d_qpl_ranges(int64_t nq, int64_t nb);
// Number of vertex ranges for nblocks query tiles over nb boundary vertices
// (1: no split), and the range length in vertices (a multiple of the chunk).
int adj3d_parts(int64_t nblocks, int64_t nb);
int32_t adj3d_span(int64_t nb, int parts);

// carry: [rows][parts][3] shares of the vertex before each range (with
// a.partial), gq_part: [parts][nq][3] query gradients per range (with a.gq).
hipError_t launch_adj3d_split(const AdjArgs& a, const LoopTable& L, int64_t nblocks, int qpl, int parts,
                              int32_t span, float* carry, float* gq_part, hipStream_t s);
// gq[t] = sum over ranges of gq_part[p][t], in range order.
hipError_t launch_sum_parts(const float* gq_part, int parts, int64_t n, float* gq, hipStream_t s);
// launch_reduce_partials plus the carry slots of the ranges that start
// inside a loop.
hipError_t launch_reduce_partials_split(const float* pv, const float* pl, const float* carry, int parts,
                                        int32_t span, int64_t rows, int32_t nb, const LoopTable& L, double* tmp,
                                        float* out, hipStream_t s);

}  // namespace wn
