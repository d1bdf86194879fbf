// Internal interface between the host engine (hjx_api.cpp) and the HIP
// kernels (hjx_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
// halo) and marches over `march` consecutive nodes of the third-fastest axis
// (dim >= 3).  tx * ty <= 256.
struct Tile {
    int tx, ty, march;
    int variant;  // kVariantPlaneMarch or kVariantDirect
};

// Stage-kernel variants (the same arithmetic, bit for bit):
//   plane-march: the tiling above, each interval evaluated once and shared;
//   direct: one thread per node, gathering its stencils through the caches
//           and evaluating both halves at the node (no LDS, no barriers).
enum : int { kVariantPlaneMarch = 0, kVariantDirect = 1 };

// One fused stage: out = ca * phi_n + cb * (phi_in + dt * L(phi_in)),
// then out = min(out, target) if target != nullptr; with rhs_only the
// kernel writes L(phi_in) itself.
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
    Tile tile;
};

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

enum : int { kSchemeFirst = 1, kSchemeEno2 = 2, kSchemeEno3 = 3, kSchemeWeno5 = 5 };
enum : int { kHamNormal = 0, kHamDubins3 = 1, kHamDubins4 = 2 };

// Launchers (return hipSuccess or the launch error).
hipError_t launch_stage_f32(const StageArgs<float> &a, int scheme, int ham, hipStream_t s);
hipError_t launch_stage_f64(const StageArgs<double> &a, int scheme, int ham, hipStream_t s);

// alpha[d] = max over nodes (written to alpha_out[0..dim-1] on the device);
// partial must hold alpha_blocks() * kMaxDim doubles.
int alpha_blocks(int total);
hipError_t launch_alpha_f32(const AlphaArgs<float> &a, double *alpha_out, hipStream_t s);
hipError_t launch_alpha_f64(const AlphaArgs<double> &a, double *alpha_out, hipStream_t s);

// flag |= 1 if any of the n values is NaN or Inf (flag must be cleared first).
hipError_t launch_nonfinite_f32(const float *x, int n, int *flag, hipStream_t s);
hipError_t launch_nonfinite_f64(const double *x, int n, int *flag, hipStream_t s);

// plain element copy (used where a stage result must land in another buffer)
hipError_t launch_copy_f32(const float *src, float *dst, int n, hipStream_t s);
hipError_t launch_copy_f64(const double *src, double *dst, int n, hipStream_t s);

}  // namespace hjx
