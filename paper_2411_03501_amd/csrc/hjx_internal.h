// Internal interface between the host engine (hjx_api.cpp) and the HIP
// kernels (hjx_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hjx_fastdiv.h"

namespace hjx {

constexpr int kMaxDim = 4;

// Per-axis device tables: for axis d, node coordinates and their cosine and
// sine (used by Hamiltonians with an angle axis), each n[d] values of T.
template <typename T>
struct AxisTables {
    const T *coord[kMaxDim];
    const T *cosv[kMaxDim];
    const T *sinv[kMaxDim];
};

// Geometry of a dense row-major grid (last axis fastest).
struct GridGeom {
    int dim;
    int n[kMaxDim];
    int stride[kMaxDim];
    unsigned periodic;  // bit d: axis d periodic
    int plane;          // nodes in the plane of the last two axes (last axis for dim 1)
    int slow;           // product of the remaining axes
};

// Launch shape of the stage kernel.  A block covers tx nodes of the fastest
// axis by ty nodes of the second-fastest ("plane tile", staged in LDS with its
// halo) and, in 3-D and 4-D, marches over `march` consecutive nodes of axis 0.
// tx * ty <= 256 in 1-D and 2-D; in 3-D and 4-D the tile kernel runs 512
// threads over tx * ty <= 512 nodes.  The steps variant (1-D, 2-D) takes
// `march` whole RK steps of a tx x ty output tile per launch.
struct Tile {
    int tx, ty, march;
    int variant;  // kVariantPlaneMarch, kVariantDirect or kVariantSteps
};

// Stage-kernel variants (the same arithmetic, bit for bit):
//   plane-march: the tiling above, each interval evaluated once and shared;
//   direct: one thread per node, gathering its stencils through the caches
//           and evaluating both halves at the node (no LDS, no barriers);
//   steps: several whole RK steps per launch (below); single stages of such
//          a problem take the direct variant.
enum : int { kVariantPlaneMarch = 0, kVariantDirect = 1, kVariantSteps = 2 };

// One fused stage: out = ca * phi_n + cb * (phi_in + dt * L(phi_in)),
// then out = min(out, target) if target != nullptr; with rhs_only the
// kernel writes L(phi_in) itself.  L is clipped first when clip != 0.
template <typename T>
struct StageArgs {
    const T *phi_in;
    const T *phi_n;   // read only when ca != 0
    const T *target;  // nullable
    T *out;
    GridGeom g;
    AxisTables<T> tab;
    T inv_dx[kMaxDim];
    T dx[kMaxDim];
    T alpha[kMaxDim];
    T hp[8];
    T dt, ca, cb;
    int rhs_only;
    int clip;  // restricted update: 0 none, -1 L <- min(L, 0), +1 L <- max(L, 0) (not with rhs_only)
    int diss;  // 0: Lax-Friedrichs with alpha[d]; 1: with alpha_d at the node; 2: Godunov (normal motion)
    Tile tile;
    unsigned char *mask;  // nullable (replay for the adjoint): bit 0 where the target was the smaller, bit 1 where L was clipped
    T *dp_out;            // nullable: p-_d at dp_out + 2d dp_stride, p+_d at dp_out + (2d+1) dp_stride
    int dp_stride;
};

// ---------------------------------------------------------------- adjoint
// Per-block accumulators of the adjoint (doubles per block):
enum : int {
    kAccDhMain = 0,   // dL/dh summed over every step but the last
    kAccDhLast = 1,   // dL/dh of the last (clamped) step
    kAccAlpha = 2,    // dL/dalpha_d, d < 4
    kAccTheta = 6,    // dL/dtheta_m at fixed alpha, m < 8
    kAccCount = 16
};

// Reverse of one stage out = ca phi_n + cb (phi_in + h L(phi_in)) (then
// min with the target), given lam_out = dL/dout.  `mask` (nullable) holds
// the replay's decisions per node: bit 0 where the target was kept, bit 1
// where a restricted update clipped L to 0.
//   lam_out' = lam_out where the evolved value was kept (the rest goes to
//              the target's adjoint),
//   lam_in  (=, or += when in_mode) cb lam_out' (+ the transposed spatial
//              operator, added afterwards by the per-axis kernels from the
//              seeds written here),
//   lam_n   (=, or += when n_mode == 2) ca lam_out' when n_mode != 0,
//   seeds   s-_d = w dL/dp-_d, s+_d = w dL/dp+_d with w = cb h lam_out'
//              (0 where L was clipped),
//   acc     dL/dh += cb lam_out' . L (unclipped nodes), dL/dalpha_d,
//              dL/dtheta (per block).
template <typename T>
struct AdjSeedArgs {
    StageArgs<T> st;  // forward evaluation at st.phi_in (alpha, tables, parameters)
    const T *lam_out;
    const unsigned char *mask;
    T *lam_target;
    T *seed_m[kMaxDim];
    T *seed_p[kMaxDim];
    T *lam_in;
    int in_mode;
    T *lam_n;
    int n_mode;
    T ca, cb, h;
    double *acc;
    int h_slot;
    const T *dp_in;            // nullable: p-, p+ stored by the replay (layout of StageArgs::dp_out)
    int dp_stride;
    const T *lam_add[kMaxDim]; // lam_out is lam_out + lam_add[0] + ... (added in that order)
    int n_add;
};

// lam += transposed derivative intervals along axis d, from the seeds of
// that axis (line tiles of tl nodes along d by tw along the cross axis c).
template <typename T>
struct AdjAxisArgs {
    const T *phi;
    const T *seed_m, *seed_p;
    T *lam;
    GridGeom g;
    int d, c;        // line axis; cross axis or -1
    int rest[2];     // remaining axes, or -1
    T inv_dx, dx;
    int tl, tw;
    T *out;          // nullable: write the contribution here instead of adding it to lam
    // filled in by the launcher: line tiles per line and the divisors below
    // as multipliers for udiv()
    int tiles_d;
    unsigned m_tiles, m_rest1;
};

// x / d for a uniform divisor d, from m = fast_div_multiplier(d, bound)
// (hjx_fastdiv.h): m = 0 means d = 1; m = 1 means plain division; otherwise
// the high half of x m, exact for 0 <= x < bound.
__device__ __forceinline__ int udiv(int x, int d, unsigned m)
{
    if (m == 0) return x;
    if (m == 1) return x / d;
    return (int)__umulhi((unsigned)x, m);
}

// The transposes of several axes in one launch (start and gx are filled in
// by the launcher).
template <typename T>
struct AdjAxesArgs {
    AdjAxisArgs<T> ax[kMaxDim];
    int nax;
    int start[kMaxDim + 1];
    int gx[kMaxDim];
    unsigned m_gx[kMaxDim];
};

// lam += c[0] + ... + c[n-1], in that order
template <typename T>
struct AdjCombineArgs {
    const T *c[kMaxDim];
    int n;
};

// ---------------------------------------------------------------- batch
// One instance of a batched solve.  Its solution lives in phi (the caller's
// output array); ws0 and ws1 are its stage buffers (ws1 for RK3 only).
template <typename T>
struct BatchInst {
    StageArgs<T> st;   // geometry, tables, alpha, parameters (stage pointers set in the kernel)
    const T *phi0;     // initial data, copied into phi first
    const T *target;   // nullable
    T *phi, *ws0, *ws1;
    T dt, dt_last;     // CFL step; the last (clamped) step
    int steps;         // RK steps of this instance
    int ham;
    int total;         // nodes
    int item0;         // first work item of this instance
};

// Batch launch modes (BatchArgs::stage): RK stages are 0..rk-1; the others
// are whole-batch passes.
enum : int {
    kBatchCopyIn = -1,     // phi = phi0
    kBatchCopyOut = -2,    // RK1 with an odd step count: phi = ws0
    kBatchCheckIn = -3,    // flags[k] = 1 if phi0 of instance k holds NaN/Inf
    kBatchCheckOut = -4    // the same for phi
};

// One launch: `items` work items (item_nodes consecutive nodes of one
// instance each) of the first n_active instances (instances sorted by
// decreasing step count), for stage `stage` of global step s.
template <typename T>
struct BatchArgs {
    const BatchInst<T> *inst;
    int *flags;
    int n_active, items, s, stage, rk, item_nodes;
    int clip;  // some instance has a restricted update
    int ext;   // some instance plays the rockets game or takes the local dissipation or Godunov's Hamiltonian
};

hipError_t launch_batch_f32(const BatchArgs<float> &a, int scheme, int blocks, hipStream_t s);
hipError_t launch_batch_f64(const BatchArgs<double> &a, int scheme, int blocks, hipStream_t s);
// resident blocks of the batch kernel on one CU (occupancy); clip: the
// kernel for batches with a restricted update
int batch_blocks_per_cu(int dtype_f64, int scheme, int clip, int ext);

// The seed pass; with rep (nullable) one forward stage of the replay (same
// grid; p-, p+ kept exactly when a.dp_in is set) runs in the same launch.
hipError_t launch_adj_seed_f32(const AdjSeedArgs<float> &a, const StageArgs<float> *rep, int scheme, int ham,
                               hipStream_t s);
hipError_t launch_adj_seed_f64(const AdjSeedArgs<double> &a, const StageArgs<double> *rep, int scheme, int ham,
                               hipStream_t s);
hipError_t launch_adj_axes_f32(const AdjAxesArgs<float> &a, int scheme, hipStream_t s);
hipError_t launch_adj_axes_f64(const AdjAxesArgs<double> &a, int scheme, hipStream_t s);
hipError_t launch_combine_f32(float *lam, const AdjCombineArgs<float> &c, int n, hipStream_t s);
hipError_t launch_combine_f64(double *lam, const AdjCombineArgs<double> &c, int n, hipStream_t s);
int adj_seed_blocks(const GridGeom &g);
// out[k] = sum over blocks of acc[block * kAccCount + k]
hipError_t launch_acc_reduce(const double *acc, int blocks, double *out, hipStream_t s);
// x[i] = 0 for i < n (a kernel, not a memset)
hipError_t launch_zero_f32(float *x, int n, hipStream_t s);
hipError_t launch_zero_f64(double *x, int n, hipStream_t s);
hipError_t launch_zero_f64acc(double *x, int n, hipStream_t s);
// smoothed-volume loss: out[0] = vol * sum s(-phi/eps); grad (nullable) =
// its derivative; partial holds `blocks` doubles
hipError_t launch_loss_f32(const float *phi, int n, double eps, double vol, float *grad, double *partial, int blocks,
                           double *out, hipStream_t s);
hipError_t launch_loss_f64(const double *phi, int n, double eps, double vol, double *grad, double *partial,
                           int blocks, double *out, hipStream_t s);

// Dissipation reduction over all nodes (first pass: one partial per block).
template <typename T>
struct AlphaArgs {
    GridGeom g;
    AxisTables<T> tab;
    T hp[8];
    int ham;
    double *partial;  // [blocks][kMaxDim]
    int total;
};

// LDS of one stage block: the staged plane with a 3-node halo on both plane
// axes, and the right-biased derivatives exchanged along each plane axis.
inline size_t stage_lds_bytes(const Tile &t, size_t elem)
{
    return elem * ((size_t)(t.ty + 6) * (t.tx + 6) + (size_t)t.ty * (t.tx + 1) + (size_t)(t.ty + 1) * t.tx);
}

// The tile kernel of 3-D and 4-D grids: the decomposition of its blocks
// (tiles along the fastest axis and the second, chunks of the marched axis 0,
// and in 4-D the nodes of the gathered axis 1, which varies fastest) and its
// LDS: the staged tile with its halo and four one-sided values per node.
constexpr int kTileNodes = 512;  // nodes of one tile of the 3-D and 4-D tile kernel, at most

struct TileLaunch {
    int tiles_f, tiles_m, chunks, outer;
    int blocks;  // tiles_f * tiles_m * chunks * outer (the grid is padded to a multiple of 8)
    int y_first; // 4-D interior launch: axis-1 node of its first line (3)
};

// The 4-D tile kernel's lines of the gathered axis 1: every line (a 3-D grid,
// or a 4-D grid with too few lines for an interior), the lines whose
// seven-plane stencil lies inside the grid, or the six lines within three of
// its ends, non-periodic (ghost planes extrapolated from planes the line
// loads anyway) or periodic (wrapped).  The kinds are separate launches with
// separate register allocations: the ghost rules of the end lines need block
// constants that would otherwise stay live, spilled, through every interior
// block.
enum : int { kTileLinesAll = 0, kTileLinesInterior = 1, kTileLinesEnds = 2, kTileLinesEndsWrap = 3 };

inline size_t tile_lds_bytes(const Tile &t, size_t elem)
{
    return elem * ((size_t)(t.ty + 6) * (t.tx + 6) + 4 * (size_t)t.tx * t.ty);
}

enum : int { kSchemeFirst = 1, kSchemeEno2 = 2, kSchemeEno3 = 3, kSchemeWeno5 = 5 };

// Nodes each side of a node that one stage of the scheme reads along an axis.
constexpr int scheme_radius(int scheme) { return scheme == kSchemeFirst ? 1 : (scheme == kSchemeEno2 ? 2 : 3); }

// Several whole RK steps of a 1-D or 2-D grid in one launch (the steps
// variant).  Each block owns a tx x ty tile of the output (ty along axis 0,
// tx along the fastest axis; ty = 1 in 1-D) and loads it into LDS with a halo
// of H = k * rk * radius nodes on every side that is not a non-periodic end
// of the grid; every stage is then evaluated on the whole region that still
// holds valid values, which shrinks by the radius on those sides, so after k
// steps the tile itself is exact.  The halo work is done again by the
// neighbouring blocks: it buys k - 1 fewer dependent launches per k steps,
// which is what small grids are bound by.
struct StepsLaunch {
    int k, rk;           // whole steps in this launch, RK order
    double dt, dt_last;  // size of every step of the launch but its last, and of its last
    int tx, ty;          // output tile
    int tiles_x;         // tiles along the fastest axis (blocks: tiles_x * tiles along axis 0)
    int area_max;        // LDS values per buffer (the largest region of any block)
    int *flag_in;        // nullable: set to 1 if a value loaded from the input is NaN or Inf
    int *flag_out;       // nullable: set to 1 if a value stored is NaN or Inf
};

// LDS buffers of the steps variant: the stage input and phi^n, plus a third
// for the middle stage of RK3.
constexpr int steps_buffers(int rk) { return rk == 3 ? 3 : 2; }

// The largest region of one block (values per LDS buffer) for tile (tx, ty)
// and halo H on a grid of n_x x n_y (n_y = 1 in 1-D): a region never spans
// more than a non-periodic axis holds.
inline long steps_area(long tx, long ty, long H, long nx, long ny, bool per_x, bool per_y, bool two_d)
{
    long wx = (tx < nx ? tx : nx) + 2 * H, wy = two_d ? (ty < ny ? ty : ny) + 2 * H : 1;
    if (!per_x && wx > nx) wx = nx;
    if (two_d && !per_y && wy > ny) wy = ny;
    return wx * wy;
}
constexpr size_t kStepsLdsMax = 64 * 1024;  // bytes of LDS per block, so that two blocks share a CU
enum : int { kHamNormal = 0, kHamDubins3 = 1, kHamDubins4 = 2, kHamRockets = 3 };
// normal motion with Godunov's numerical Hamiltonian instead of Lax-Friedrichs
// (a template tag of the stage kernels, chosen by StageArgs::diss)
enum : int { kHamNormalGodunov = 4 };

// Launchers (return hipSuccess or the launch error).
hipError_t launch_stage_f32(const StageArgs<float> &a, int scheme, int ham, hipStream_t s);
hipError_t launch_stage_f64(const StageArgs<double> &a, int scheme, int ham, hipStream_t s);
// l.k whole RK steps from a.phi_in into a.out (different arrays), with
// a.target (nullable) taken after the last stage of every step (hjx_steps.hip)
hipError_t launch_steps_f32(const StageArgs<float> &a, const StepsLaunch &l, int scheme, int ham, hipStream_t s);
hipError_t launch_steps_f64(const StageArgs<double> &a, const StepsLaunch &l, int scheme, int ham, hipStream_t s);

// alpha[d] = max over nodes (written to alpha_out[0..dim-1] on the device);
// partial must hold alpha_blocks() * kMaxDim doubles.
int alpha_blocks(int total);
hipError_t launch_alpha_f32(const AlphaArgs<float> &a, double *alpha_out, hipStream_t s);
hipError_t launch_alpha_f64(const AlphaArgs<double> &a, double *alpha_out, hipStream_t s);

// flag |= 1 if any of the n values is NaN or Inf (flag must be cleared first).
hipError_t launch_nonfinite_f32(const float *x, int n, int *flag, hipStream_t s);
hipError_t launch_nonfinite_f64(const double *x, int n, int *flag, hipStream_t s);

// ---------------------------------------------------------------- conservation laws
// One Lax-Friedrichs step of v_t + sum_d f_d(v)_{x_d} = 0 (hjx_claw.hip):
// out = inv_2n sum_d (v_{+d} + v_{-d}) - sum_d half_lam[d] (f_d(v_{+d}) - f_d(v_{-d}))
// with half_lam[d] = dt / (2 dx_d) and inv_2n = 1 / (2 dim).
enum : int { kFluxLinear = 0, kFluxBurgers = 1 };

template <typename T>
struct ClawArgs {
    const T *v;
    T *out;
    int dim;
    int n[kMaxDim];
    int stride[kMaxDim];
    unsigned periodic;  // bit d: axis d periodic (else the edge value continues)
    int rows;           // nodes / n[dim - 1]
    T c[kMaxDim];       // f_d(v) = c_d v (linear) or c_d v^2 / 2 (Burgers)
    T half_lam[kMaxDim];
    T inv_2n;
};

hipError_t launch_claw_f32(const ClawArgs<float> &a, int flux, hipStream_t s);
hipError_t launch_claw_f64(const ClawArgs<double> &a, int flux, hipStream_t s);
// *out = max |v_i| as the bits of a double (cleared first by the launcher)
hipError_t launch_maxabs_f32(const float *v, int n, unsigned long long *out, hipStream_t s);
hipError_t launch_maxabs_f64(const double *v, int n, unsigned long long *out, hipStream_t s);

// ---------------------------------------------------------------- shapes
// An implicit surface over a grid (hjx_shapes.hip).
enum : int { kShapeBall = 0, kShapeEllipsoid = 1 };
enum : int { kOpUnion = 0, kOpIntersection = 1, kOpComplement = 2, kOpSubtraction = 3 };

struct ShapeArgs {
    int dim, kind;
    unsigned mask;      // bit d: axis d takes part
    int n[kMaxDim];
    int rows;           // nodes / n[dim - 1]
    long total;
    double gmin[kMaxDim], dx[kMaxDim];
    double center[kMaxDim], weights[kMaxDim];
    double radius;
};

// One member of a batched construction: its shape and output.
struct ShapeMember {
    ShapeArgs a;
    void *out;
};

// hjx_shape_batch_noalloc's descriptor array (a file-scope device array of
// this many members per GPU) and its device address on the current device
constexpr int kShapeNoAllocMax = 1024;
hipError_t shape_noalloc_scratch(ShapeMember **out);

hipError_t launch_shape_f32(const ShapeArgs &a, float *out, hipStream_t s);
// members: device array of nm (<= 65535) members; largest: the most nodes of one member
hipError_t launch_shape_batch_f32(const ShapeMember *members, int nm, long largest, hipStream_t s);
hipError_t launch_shape_batch_f64(const ShapeMember *members, int nm, long largest, hipStream_t s);
hipError_t launch_shape_f64(const ShapeArgs &a, double *out, hipStream_t s);
hipError_t launch_shape_op_f32(int op, const float *a, const float *b, float *out, long n, hipStream_t s);
hipError_t launch_shape_op_f64(int op, const double *a, const double *b, double *out, long n, hipStream_t s);

// plain element copy (used where a stage result must land in another buffer)
hipError_t launch_copy_f32(const float *src, float *dst, int n, hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, int n, hipStream_t s);

}  // namespace hjx
