/*
 * wn.h -- C ABI of the one-shot generalized winding number library (libwn.so)
 * for AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 3, Alg. 1 of Martens & Bessmeltsev, "One-Shot Method for
 * Computing Generalized Winding Numbers"): given an oriented surface M with
 * boundary dM and query points p, return the generalized winding number
 * w_M(p) = (1/4pi) int_M dOmega(p) (2D: (1/2pi) int_C dtheta(p)).
 *
 * Method as implemented here.  One fixed unit direction d is shared by every
 * query.  Eq. wn_chi and Lemmas 1-2 give
 *
 *     w(p) = chi_d(p) + (1/2pi) * sum over boundary edges of theta_e(p)
 *
 * where chi_d(p) is the signed number of crossings of the ray p + t d,
 * t > 0, with M (Eq. chi: +1 when the ray runs along the face normal
 * (v1-v0)x(v2-v0)), and theta_e is half the signed solid angle of the
 * spherical triangle (-d, a-p, b-p) for boundary edge a->b, i.e. the region
 * areas of Eq. wn_discrete_sum written as a boundary line integral with d's
 * region as the BFS seed of Alg. 1.  2D: chi_d plus the open-curve end-point
 * angles measured from d.
 *
 * Conventions for every call
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary CPU memory read before the call returns.
 *  - Every call enqueues work on `stream` (a hipStream_t passed as void*,
 *    NULL = the null stream) and returns without synchronising; the caller
 *    keeps every buffer alive until the stream reaches that point.
 *  - Inputs are never modified.  Outputs are fully overwritten (never
 *    accumulated) and must not alias inputs.  Arrays are tightly packed,
 *    little-endian, 4-byte aligned (16-byte preferred).
 *  - Errors are returned, never thrown.  Arguments are validated on the host
 *    before anything is enqueued; on error nothing is enqueued and handles
 *    are unchanged.  wn_last_error() gives a per-thread message.
 *  - A query exactly on M or its boundary has no defined w (Sec. 3); the
 *    result there is unspecified but finite unless the query itself is
 *    non-finite, in which case w = NaN and chi = WN_CHI_INVALID.
 *  - A zero-size batch (nq == 0) is a no-op returning WN_OK.
 */
#ifndef WN_H
#define WN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wn_status;
#define WN_OK                    0
#define WN_ERR_INVALID_ARGUMENT  1
#define WN_ERR_UNSUPPORTED       2
#define WN_ERR_OUT_OF_MEMORY     3
#define WN_ERR_HIP               4
#define WN_ERR_INTERNAL          5

typedef int32_t wn_dtype;
#define WN_F32 0
#define WN_F64 1

/* chi value written for a query whose input is not finite */
#define WN_CHI_INVALID ((int32_t)0x80000000)

/* Boundary loops whose table travels in the kernel arguments.  The 3D calls
 * (wn_eval_3d, wn_eval_3d_boundary, wn_eval_3d_grid, wn_backward) and
 * wn_eval_2d take more: such a table is copied to device memory allocated on
 * the call's stream (which the call then synchronises once) and freed after
 * the launches.  wn_backward_2d and wn_backward_noalloc take at most this
 * many. */
#define WN_MAX_LOOPS 256

typedef struct wn_bvh wn_bvh;       /* opaque: frame, rotated vertices, BVH */
typedef struct wn_batch wn_batch;   /* opaque: many surfaces, one launch   */
typedef struct wn_batch2d wn_batch2d;   /* opaque: many 2D curve sets    */

/* Library version (major*10000 + minor*100 + patch). */
int32_t wn_version(void);

/* Human-readable name of a status code (static string). */
const char* wn_status_string(wn_status s);

/* Message of the last error on the calling thread ("" if none). */
const char* wn_last_error(void);

/* ---------------------------------------------------------------------------
 * wn_boundary_loops -- boundary of an oriented triangle mesh (host, topology).
 *
 * Sec. 5.1 "Multiple Boundaries" / Sec. 6.1 "Preprocessing": the boundary consists
 * of the edges used by exactly one face.  Each boundary half-edge keeps the
 * orientation it has in its face; half-edges are chained head to tail into
 * closed loops.
 *
 *  F         host [nf][3] int32 vertex indices, each in [0, nv).
 *  bnd_idx   host [cap] int32 out: boundary vertex ids, loop after loop; loop
 *            l occupies [loop_off[l], loop_off[l+1]) and has edges
 *            v_i -> v_{i+1} plus the closing edge last -> first.
 *  loop_off  host [cap + 1] int64 out.
 *  cap       capacity of bnd_idx (3*nf always suffices).
 *  nb_out, nloops_out  host out: number of boundary vertices and loops.
 * Loops are ordered by their smallest vertex id and start there.
 * Errors: INVALID_ARGUMENT for out-of-range indices, a non-manifold boundary
 * (a vertex with two outgoing boundary edges) or cap too small.
 * ------------------------------------------------------------------------- */
wn_status wn_boundary_loops(const int32_t* F, int64_t nf, int64_t nv,
                            int32_t* bnd_idx, int64_t* loop_off, int64_t cap,
                            int64_t* nb_out, int32_t* nloops_out);

/* ---------------------------------------------------------------------------
 * wn_build_bvh -- prepare a triangle mesh for chi_d (Eq. chi; the ray-casting step of Alg. 1).
 *
 * Builds, on the GPU, the rotated frame of d (rows e1, e2, d; det +1; scaled
 * by a power of two so that coordinates are O(1)), the rotated vertices and
 * a binary LBVH over the triangles' projections along d (every ray of one
 * call is parallel to d, so a node is a 2D box plus the largest coordinate
 * along d), then folds every second level of that tree into a four-wide
 * tree whose child boxes are 8-bit cells of a per-node grid, assigned with
 * the same monotone function the traversal applies to the query (no ray
 * loses a triangle).  The handle keeps that tree and one 128-byte record per sorted
 * triangle (its rotated vertices as float32 pairs); it owns its device memory
 * and does not keep V or F.
 *
 *  V    device [nv][3] float32; F device [nf][3] int32 (indices must lie in
 *       [0, nv): they are not checked on the device).
 *  dir  host [3] float64, finite and nonzero (normalised here in float64).
 *  out  receives the handle on success.
 * The build is enqueued on `stream`; the handle may be used on that stream
 * at once and on other streams after synchronising with it.
 * Errors: INVALID_ARGUMENT (null pointers with nonzero counts, bad dir,
 * nv or nf above 2^31-2), OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_build_bvh(const float* V, int64_t nv, const int32_t* F, int64_t nf,
                       const double dir[3], void* stream, wn_bvh** out);

/* Release a handle (waits for nothing; the caller synchronises first). */
wn_status wn_free_bvh(wn_bvh* bvh);

/* The unit direction (float64, host [3]) a handle was built for. */
wn_status wn_bvh_direction(const wn_bvh* bvh, double dir[3]);

/* ---------------------------------------------------------------------------
 * wn_eval_3d -- w_M(p) for triangle meshes (Alg. 1 with one shared ray
 * direction; Eq. wn_discrete_sum as a boundary line integral).
 *
 *  bvh        from wn_build_bvh for this mesh.
 *  bnd_xyz    device [nb][3] float32 boundary vertices in loop order; they
 *             must be bit-identical copies of the mesh vertices (e.g.
 *             V[bnd_idx] from wn_boundary_loops), so that the crossing count
 *             and the boundary term flip together where the ray meets dM.
 *  loop_off   host [nloops + 1] int64, nondecreasing, loop_off[0] = 0,
 *             every loop with >= 3 vertices; nb = loop_off[nloops].
 *             nloops = 0 (closed mesh) is allowed; more than WN_MAX_LOOPS
 *             loops are read from a device copy of the table.
 *  qx, qy, qz device [nq] float32 query coordinates (structure of arrays).
 *  w_out      device [nq] float32 out.
 *  chi_out    device [nq] int32 out (chi_d), or NULL.
 * Errors: INVALID_ARGUMENT, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_3d(const wn_bvh* bvh, const float* bnd_xyz,
                     const int64_t* loop_off, int32_t nloops,
                     const float* qx, const float* qy, const float* qz, int64_t nq,
                     float* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_eval_3d_grid -- w_M on a grid whose columns run along the ray: queries
 * (gx[i], gy[j], gz[k]), i < nx, j < ny, k < nz, for a BVH built for the
 * direction +z.  Sec. 5 ("Optimization"): points on one line parallel to
 * the ray share the ray.  The points of a column are consecutive lanes with
 * identical frame coordinates X, Y, so a wavefront walks the tree once for
 * its column and each point applies the exact triangle test at its own
 * height; chi and w are bit-identical to wn_eval_3d on the same float32
 * points, without materialising the point coordinates.
 *  gx, gy, gz device float32 [nx], [ny], [nz].
 *  w_out      device [nx][ny][nz] float32 out (z fastest); chi_out same
 *             layout int32, or NULL.
 * Errors: UNSUPPORTED if the BVH's direction is not +z; INVALID_ARGUMENT
 * (negative sizes, 2^32 points or more); HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_3d_grid(const wn_bvh* bvh, const float* bnd_xyz,
                          const int64_t* loop_off, int32_t nloops,
                          const float* gx, const float* gy, const float* gz,
                          int64_t nx, int64_t ny, int64_t nz,
                          float* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_eval_3d_boundary -- boundary term only: w_out = chi_in + S/(2pi), in the
 * frame of `bvh`.  Same arguments as wn_eval_3d except that chi_d comes from
 * the caller (device [nq] int32).  A WN_CHI_INVALID entry gives w = NaN.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_3d_boundary(const wn_bvh* bvh, const float* bnd_xyz,
                              const int64_t* loop_off, int32_t nloops,
                              const float* qx, const float* qy, const float* qz,
                              int64_t nq, const int32_t* chi_in, float* w_out,
                              void* stream);

/* ---------------------------------------------------------------------------
 * wn_eval_3d_curves -- w for a surface whose boundary is a set of closed
 * loops of cubic Bezier curves: w = chi_d + Theta/(2pi), Theta the line
 * integral along the curves of the form whose integral along a straight edge
 * is the polyline path's edge term (Sec. 5.1 "Exact Computations": region areas from boundary
 * integrals, Gauss-Bonnet; Bezier boundaries are integrated numerically).
 *  bvh        frame and direction d; also gives chi_d when chi_in is NULL
 *             (the BVH of the surface's tessellation).
 *  ctrl       device [ncurves][4][3] float32 control points, in the
 *             orientation the surface induces on its boundary.
 *  qx..nq     queries as in wn_eval_3d.
 *  chi_in     device [nq] int32 chi_d from the caller (for example from an
 *             exact ray-surface intersection), or NULL.
 *  w_out      device [nq] float32 out; chi_out device int32 or NULL.
 * Quadrature: per curve, dyadic panels integrated by 6-point Gauss-Legendre
 * once they lie farther than 1.5 control-polygon lengths from the query,
 * halved otherwise (at most 24 times; the chord's exact edge term then
 * stands in).  With chi_d from a tessellation whose boundary vertices lie on
 * the curves, chi_d and Theta jump at slightly different places: w can be
 * off by one where the ray passes between a boundary chord and its curve.
 * With chi_in and from 2^16 queries the call works on a copy of the queries
 * (and chi_in) in a coarse Morton order, as wn_backward_curves, and scatters
 * the results back, the same values per query; this allocates about 36
 * bytes per query on the stream.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_3d_curves(const wn_bvh* bvh, const float* ctrl, int64_t ncurves,
                            const float* qx, const float* qy, const float* qz, int64_t nq,
                            const int32_t* chi_in, float* w_out, int32_t* chi_out,
                            void* stream);

/* ---------------------------------------------------------------------------
 * wn_backward_curves -- adjoint of the curve boundary term for a loss L with
 * dL/dw = grad_w.  Away from the surface chi_d is locally constant, so
 * (as for wn_backward) the derivatives come from the boundary alone and do
 * not depend on d:
 *   dL/dp   = +(g/4pi) int (gamma - p) x gamma'(t) / |gamma - p|^3 dt,
 *   dL/dc_k = -sum_q (g_q/4pi) int B_k(t) (gamma - p) x gamma'(t) / |gamma - p|^3 dt
 * over every curve (B_k the cubic Bernstein functions), integrated on the
 * same dyadic panels as wn_eval_3d_curves (6-point Gauss-Legendre once a
 * panel is 1.5 control-polygon lengths away).
 *  ctrl       device [ncurves][4][3] float32 (world coordinates).
 *  qx..nq     queries; grad_w device [nq] float32.
 *  grad_q     device [nq][3] out, or NULL (NaN for non-finite queries).
 *  grad_ctrl  device [ncurves][4][3] out, or NULL: fixed-order sums
 *             (wavefront, workgroup, then float64 over workgroups), bitwise
 *             reproducible; allocates 48 bytes per (256 queries, curve) on
 *             the stream.  A control point shared by two curves gets one
 *             entry per curve; the caller adds them.
 * From 2^16 queries the call first puts a copy of the queries in a coarse
 * Morton order (32^3 cells over their bounding box, as wn_spatial_order
 * with 5 bits per axis), so that the lanes of a wavefront refine similar
 * panels; grad_q is scattered back and is the same per query, and
 * grad_ctrl is summed in that (deterministic) order.  This allocates about
 * 40 bytes per query more on the stream.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_backward_curves(const float* ctrl, int64_t ncurves,
                             const float* qx, const float* qy, const float* qz, int64_t nq,
                             const float* grad_w, float* grad_q, float* grad_ctrl, void* stream);

/* ---------------------------------------------------------------------------
 * wn_eval_3d_patches -- w of a parametric surface made of bicubic Bezier
 * patches, without tessellation: chi_d from the exact ray-patch crossings
 * (Eq. chi; Sec. 5.1, "Parametric Surfaces") plus the boundary integral along
 * the surface's boundary curves as in wn_eval_3d_curves.
 *  dir        host [3] ray direction d (normalised here).
 *  nets       device [npatch][4][4][3] float32 Bernstein control nets (index
 *             [i][j]: i along u, j along v); a crossing counts
 *             sign(d . (S_u x S_v)).
 *  curves     device [ncurves][4][3] float32: the surface's boundary loops
 *             as cubic Beziers, oriented as the patches induce (may be 0).
 *  qx..nq     queries as in wn_eval_3d.
 *  w_out      device [nq] float32 out, or NULL (crossings only);
 *  chi_out    device [nq] int32 out, or NULL.
 * Crossings: per query a depth-first walk over dyadic sub-squares of each
 * patch; a sub-square is dropped when its net relative to the query excludes
 * the ray (convex hull); when it lies wholly in front of the query and the
 * hull of each of its boundary edges excludes the ray, its signed crossings
 * are the winding number of its boundary's image around the ray; otherwise
 * it is split, down to level 16 (where it is dropped).  Non-finite queries
 * give NaN / WN_CHI_INVALID.  With w_out, one launch computes both terms per
 * query (the kernel of wn_eval_3d_patches_batched).  With w_out and from
 * 2^16 queries the call works on a copy of the queries in a coarse Morton
 * order (as wn_backward_curves) and scatters the results back, the same
 * values per query; this allocates about 36 bytes per query on the stream.
 * Otherwise it allocates nothing.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_3d_patches(const double dir[3], const float* nets, int64_t npatch,
                             const float* curves, int64_t ncurves,
                             const float* qx, const float* qy, const float* qz, int64_t nq,
                             float* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * Batched parametric surfaces: many surfaces, each made of bicubic Bezier
 * patches with cubic Bezier boundary curves, its own ray direction and its
 * own queries, evaluated in one launch (w = chi_d + Theta/2pi as in
 * wn_eval_3d_patches; Sec. 5.1, "Parametric Surfaces").
 *
 * One surface of such a batch: its patch, curve and query counts and its
 * direction.  The surfaces' patches are consecutive in the nets array, their
 * curves in the curves array and their queries in qx/qy/qz and the outputs,
 * in surface order.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t npatch;
  int64_t ncurves;
  int64_t nq;
  double dir[3];
} wn_patch_surface;

typedef struct wn_patch_batch wn_patch_batch;

/* ---------------------------------------------------------------------------
 * wn_patch_batch_create -- copy the surfaces' frames and a table of which
 * surface each workgroup of 256 queries belongs to to the device.
 * Synchronises `stream`.  Errors: INVALID_ARGUMENT (naming the surface:
 * negative count, non-finite or zero direction), UNSUPPORTED (more than
 * 2^31 - 1 workgroups, patches or curves beyond 32-bit indexing),
 * OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_patch_batch_create(const wn_patch_surface* surfs, int32_t nsurf, void* stream,
                                wn_patch_batch** out);
wn_status wn_patch_batch_free(wn_patch_batch* batch);

/* ---------------------------------------------------------------------------
 * wn_eval_3d_patches_batched -- wn_eval_3d_patches for every surface of the
 * batch in one launch.
 *  nets       device [sum npatch][4][4][3] float32 (or NULL if none).
 *  curves     device [sum ncurves][4][3] float32 (or NULL if none).
 *  qx..qz     device [sum nq] float32 queries.
 *  w_out      device [sum nq] float32 out, or NULL (crossings only).
 *  chi_out    device [sum nq] int32 out, or NULL; not both NULL.
 * Each result equals, bit for bit, that of wn_eval_3d_patches called for
 * the surface alone.  Allocates nothing.  Errors: INVALID_ARGUMENT, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_3d_patches_batched(const wn_patch_batch* batch, const float* nets, const float* curves,
                                     const float* qx, const float* qy, const float* qz,
                                     float* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_diagnose -- device counters over a call's outputs (not a step of the
 * method): counts_out[0] = queries with a non-finite coordinate,
 * counts_out[1] = finite queries whose chi is WN_CHI_INVALID (a traversal
 * that found the tree malformed; 0 for every tree wn_build_bvh builds).
 *  qx..qz, nq  the queries of the call; chi the chi_out it wrote.
 *  counts_out  device [2] int64 out (overwritten, not accumulated).
 * Exact integer counts (deterministic).  Errors: INVALID_ARGUMENT, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_diagnose(const float* qx, const float* qy, const float* qz, const int32_t* chi, int64_t nq,
                      int64_t* counts_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_device_info -- compute units and peak shader clock (kHz) of the
 * current HIP device, as the runtime reports them.
 * Errors: INVALID_ARGUMENT, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_device_info(int32_t* cu_count, int32_t* clock_khz);

/* ---------------------------------------------------------------------------
 * wn_spatial_order -- a query order that groups nearby queries into the same
 * wavefront (a utility, not a step of the method).  Every query kernel runs
 * one query per lane, so a wavefront waits for its slowest lane; queries in
 * this order walk similar BVH paths and similar panel refinements.
 *  qx..nq     queries as in wn_eval_3d (nq <= INT32_MAX).
 *  order_out  device [nq] int32 out: a permutation of 0..nq-1 sorting the
 *             queries by the Morton code of their cell in a 1024^3 grid over
 *             the finite queries' bounding box; ties keep index order, so
 *             the result is deterministic; non-finite queries come last.
 * Evaluating q[order] gives w[order] bit for bit: results depend on the
 * query alone, not on its position.  Allocates about 13 bytes per query on
 * the stream for the keys and the radix sort.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_spatial_order(const float* qx, const float* qy, const float* qz, int64_t nq,
                           int32_t* order_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_crossings_3d -- chi_d only (Eq. chi; the ray-casting step of Alg. 1) through the BVH.
 *  chi_out device [nq] int32 out.
 * ------------------------------------------------------------------------- */
wn_status wn_crossings_3d(const wn_bvh* bvh, const float* qx, const float* qy,
                          const float* qz, int64_t nq, int32_t* chi_out,
                          void* stream);

/* ---------------------------------------------------------------------------
 * wn_backward -- adjoint of w with respect to the query points and the
 * boundary vertices for a loss L with dL/dw = grad_w.  chi_d is piecewise
 * constant, so only the boundary integral contributes; its derivatives are
 * the Biot-Savart field of dM and its hat-weighted edge integrals, which do
 * not depend on d.
 *
 *  bnd_xyz, loop_off, nloops as in wn_eval_3d (nloops = 0: all outputs 0).
 *  grad_w     device [nq] float32 (dL/dw per query).
 *  grad_q     device [nq][3] float32 out: dL/dp, or NULL.
 *  grad_bnd   device [nb][3] float32 out: dL/d(bnd_xyz), or NULL.  Reduced
 *             over queries in a fixed order (float64 partial sums), so the
 *             result is bitwise reproducible.
 * Few queries over a boundary of more than 512 vertices (fewer than 2048
 * workgroups of 256 threads) split the boundary into ranges of whole
 * 512-vertex chunks, one grid row per range.  grad_q is then summed over the
 * ranges in a fixed order, from a workspace of ranges x nq x 12 bytes, so it
 * stays bitwise reproducible.  It can differ from a call that does not split
 * the boundary in the last bits.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, OUT_OF_MEMORY (workspace), HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_backward(const float* bnd_xyz, const int64_t* loop_off, int32_t nloops,
                      const float* qx, const float* qy, const float* qz, int64_t nq,
                      const float* grad_w, float* grad_q, float* grad_bnd,
                      void* stream);

/* ---------------------------------------------------------------------------
 * wn_backward_noalloc -- wn_backward for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops or harnesses that
 * forbid allocation).  Same arguments, kernels, results (bit for bit) and
 * errors as wn_backward; the call makes no device allocation or free.
 *
 * Its workspace (per-workgroup vertex partials, first-stage float64 sums,
 * per-range query gradients) lives in one library-held device array of
 * WN_NOALLOC_SCRATCH_BYTES bytes.  Each GPU holds its own copy until the
 * process ends; its address is looked up on the first call on that device.
 * A call whose workspace does not fit, or whose loop table has more than
 * WN_MAX_LOOPS loops (a longer table would need device memory), returns
 * WN_ERR_UNSUPPORTED and enqueues nothing (the workspace of 2^20 queries
 * over 512 boundary vertices is about 7 MB, of 2^18 queries over 2048
 * vertices about 20 MB).
 * Every call on one GPU uses that GPU's array: calls that overlap in time on
 * one GPU (other streams, other host threads) race and must be serialised
 * by the caller.  The array keeps the last call's contents; every entry a
 * call reads was written by that call first.
 * ------------------------------------------------------------------------- */
#define WN_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
wn_status wn_backward_noalloc(const float* bnd_xyz, const int64_t* loop_off, int32_t nloops,
                              const float* qx, const float* qy, const float* qz, int64_t nq,
                              const float* grad_w, float* grad_q, float* grad_bnd,
                              void* stream);

/* ---------------------------------------------------------------------------
 * wn_eval_2d -- w_C(p) for loops of cubic Bezier curves (Sec. 3 2D
 * definition; Sec. 7 "2D Parametric Geometry").  The ray direction is +x.
 *
 *  dtype      WN_F32 or WN_F64: type of ctrl, the query coordinates and w.
 *  ctrl       device [nseg][4][2] control points; the segments of a loop are
 *             C0-joined (segment i's last point equals segment i+1's first,
 *             bit for bit).
 *  loop_off   host [nloops + 1] int64 segment offsets; loop_closed host
 *             [nloops] uint8 (nonzero: the loop's last point equals its
 *             first point; zero: open, its two end points add
 *             (phi(end-p) - phi(start-p))/(2pi), phi in [0, 2pi) measured
 *             counter-clockwise from +x).  Any number of loops (more than
 *             WN_MAX_LOOPS: a device copy of the table, see there).
 *  kind       0 = points: x[n], y[n] (n = nx, ny ignored);
 *             1 = grid: x[nx] ascending, y[ny]; outputs row-major [ny][nx]
 *             (one ray per row, the paper's one-shot reuse of Sec. 5).
 *  w_out      device out, dtype, [n] or [ny][nx]; chi_out device int32 or NULL.
 * A point on the ray's line counts as lying above it, so chi and the end
 * point angles change together where a row passes exactly through a joint.
 * Errors: INVALID_ARGUMENT, UNSUPPORTED, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_2d(wn_dtype dtype, const void* ctrl, int64_t nseg,
                     const int64_t* loop_off, const uint8_t* loop_closed, int32_t nloops,
                     int32_t kind, const void* x, const void* y, int64_t nx, int64_t ny,
                     void* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * Batched 2D grid mode: many independent curve sets, each on its own grid,
 * in one launch (the 2D experiment of Sec. 7 evaluates 1000 random cubics,
 * each on a 250 x 250 grid over its bounding box).
 *
 * One set of a batch: nseg segments (taken from the batch's ctrl array in set
 * order), its loop table as in wn_eval_2d (host arrays, offsets relative to
 * the set's first segment) and its grid size nx by ny.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t nseg;
  const int64_t* loop_off;
  const uint8_t* loop_closed;
  int32_t nloops;
  int64_t nx, ny;
} wn_curveset_2d;

/* ---------------------------------------------------------------------------
 * wn_batch2d_create -- copy the set descriptors and loop tables to the
 * device and reserve room for the monotone pieces of every segment
 * (192 (f32) or 384 (f64) bytes per segment).  `sets` is read during the
 * call only.  A loop table of any length is accepted (no WN_MAX_LOOPS
 * limit).  Sets of at most 21 segments run one wavefront per (row, tile of
 * at most 512 columns), larger sets one workgroup per (row, tile of at most
 * 4096 columns).  Synchronises `stream`.  Errors: INVALID_ARGUMENT (naming
 * the set), UNSUPPORTED (a grid side over 2^31 - 1, or more than 2^24
 * workgroup tiles or 2^26 wavefront tiles in one batch), OUT_OF_MEMORY,
 * HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_batch2d_create(wn_dtype dtype, const wn_curveset_2d* sets, int32_t nsets,
                            void* stream, wn_batch2d** out);

/* Release a 2D batch (the caller synchronises first). */
wn_status wn_batch2d_free(wn_batch2d* batch);

/* ---------------------------------------------------------------------------
 * wn_eval_2d_batched -- wn_eval_2d in grid mode (kind 1) for every set of
 * the batch: one launch splits every segment, then one launch per kernel
 * kind runs the (set, row, column tile) items; every output equals the
 * single-set wn_eval_2d grid call bit for bit.
 *  ctrl    device [sum nseg][4][2] of the batch's dtype, the sets' segments
 *          concatenated (may change between calls; the pieces are rebuilt).
 *  x, y    device [sum nx], [sum ny]: each set's axes concatenated in set
 *          order, each x axis ascending.
 *  w_out   device [sum nx*ny] out: each set's [ny][nx] grid, row-major,
 *          concatenated in set order; chi_out the same in int32, or NULL.
 * A set without segments gets w = 0, chi = 0.  No allocation, no host
 * copies: the call only enqueues the two kernels on `stream`; calls that
 * overlap on one batch race on its piece buffer.  Errors: INVALID_ARGUMENT,
 * HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_eval_2d_batched(const wn_batch2d* batch, const void* ctrl, const void* x,
                             const void* y, void* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_backward_2d -- adjoint of wn_eval_2d for a loss L with dL/dw = grad_w.
 * Away from the curves the crossing count is locally constant, so w moves
 * only with the open loops' end-point angles (the 2D boundary of Sec. 4):
 * with A(v) = (-v_y, v_x)/|v|^2 and c = grad_w/(2 pi) per query,
 *   dL/dp = c (A(s - p) - A(e - p)) summed over open loops,
 *   dL/ds = -sum_q c A(s - p),  dL/de = sum_q c A(e - p),
 * s = ctrl[first segment][0], e = ctrl[last segment][3] of each open loop;
 * every other control point gets 0.
 *  Curves, loop table, kind, x, y, nx, ny as in wn_eval_2d.
 *  grad_w     device [n] (points: n = nx; grid: [ny][nx]) of dtype.
 *  grad_q     device [n][2] of dtype out, or NULL (NaN for non-finite
 *             queries).
 *  grad_ctrl  device [nseg][4][2] of dtype out (fully written), or NULL.
 * The end-point sums are reduced in float64 in a fixed order (wavefront
 * butterfly, workgroup, chunks of workgroups, chunks; bitwise
 * reproducible).  Allocates about 32 bytes per (open loop, 256 queries) on
 * the stream.  Errors as wn_eval_2d.
 * ------------------------------------------------------------------------- */
wn_status wn_backward_2d(wn_dtype dtype, const void* ctrl, int64_t nseg,
                         const int64_t* loop_off, const uint8_t* loop_closed,
                         int32_t nloops, int32_t kind, const void* x, const void* y,
                         int64_t nx, int64_t ny, const void* grad_w, void* grad_q,
                         void* grad_ctrl, void* stream);

/* ---------------------------------------------------------------------------
 * Batched evaluation: many surfaces of uneven size, each with its own query
 * set, evaluated in one persistent launch replayed from a hipGraph.
 *
 * One surface of a batch.  V, F, bnd_xyz are device pointers as in
 * wn_build_bvh / wn_eval_3d (bnd_xyz bit-identical copies of boundary
 * vertices of V); loop_off is a host array [nloops + 1]; nq is the number of
 * this surface's queries.  The batch copies what it needs at creation.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* V;
  int64_t nv;
  const int32_t* F;
  int64_t nf;
  const float* bnd_xyz;
  const int64_t* loop_off;
  int32_t nloops;
  int64_t nq;
} wn_surface;

/* ---------------------------------------------------------------------------
 * wn_batch_create -- build the BVH of every surface (one shared ray direction
 * `dir`), a descriptor table, the boundary arena and a work list of
 * (surface, query tile) items in longest-processing-time-first order.
 *  tune_mode  0: default tile (1024 queries), 4 workgroups per compute
 *             unit, fused forward; 1: quick autotune, 2: full autotune of
 *             (tile, workgroups per CU, fused or split forward), run on the
 *             first wn_eval_batched with its real inputs; results are cached
 *             in the JSON file named by $WN_TUNE_CACHE.
 * Synchronises `stream`.  Errors: INVALID_ARGUMENT (naming the surface),
 * UNSUPPORTED, OUT_OF_MEMORY, HIP.
 * ------------------------------------------------------------------------- */
wn_status wn_batch_create(const wn_surface* surfs, int32_t ns, const double dir[3],
                          int32_t tune_mode, void* stream, wn_batch** out);

/* Release a batch (the caller synchronises first). */
wn_status wn_batch_free(wn_batch* batch);

/* ---------------------------------------------------------------------------
 * wn_eval_batched -- w (and chi) for every query of every surface.
 *  qx, qy, qz  device [sum nq] float32, the surfaces' queries concatenated in
 *              surface order.
 *  w_out       device [sum nq] float32 out; chi_out device int32 or NULL.
 * The first call captures a counter-reset kernel and the persistent
 * kernel(s) into a hipGraph (after autotuning when requested); later calls
 * replay it, patching the kernel arguments when the pointers change.  With
 * autotuning the graph is kept only if its replay is not slower than direct
 * launches of the same kernels (wn_batch_info reports which is in use).  The
 * split forward without chi_out keeps the crossing counts in a buffer the
 * batch allocates on first use (4 bytes per query).  Set
 * $WN_FORCE_NO_GRAPH to launch directly (identical results).
 * ------------------------------------------------------------------------- */
wn_status wn_eval_batched(wn_batch* batch, const float* qx, const float* qy, const float* qz,
                          float* w_out, int32_t* chi_out, void* stream);

/* ---------------------------------------------------------------------------
 * wn_backward_batched -- adjoint of the batch for dL/dw = grad_w (device
 * [sum nq]): grad_q device [sum nq][3] or NULL; grad_bnd device
 * [sum nb][3] or NULL, the surfaces' boundary vertices concatenated in
 * surface order.  Fixed-order float64 reduction (bitwise reproducible).
 * ------------------------------------------------------------------------- */
wn_status wn_backward_batched(wn_batch* batch, const float* qx, const float* qy, const float* qz,
                              const float* grad_w, float* grad_q, float* grad_bnd, void* stream);

/* info[0..8] = total queries, total boundary vertices, total (query, edge)
 * pairs, forward work items, tile size, workgroups per CU (0: one
 * workgroup per item instead of a persistent grid), graph in use
 * (0/1), autotuning time in microseconds, forward mode (0: fused kernel,
 * 1: crossing kernel then boundary kernel). */
wn_status wn_batch_info(const wn_batch* batch, int64_t info[9]);

#ifdef __cplusplus
}
#endif

#endif /* WN_H */
