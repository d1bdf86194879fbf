// Batched solve on gfx950: many instances of uneven sizes, Hamiltonians and
// parameters advanced together.  Every RK stage of every global step is ONE
// launch of persistent blocks that stride over a work list of (instance,
// run of nodes) items; instances are ordered by decreasing step count so
// that those still active at step s are a prefix of the list, and each
// instance uses its own CFL step and clamped last step.  The per-node
// arithmetic is the direct variant of the single-instance stage kernel
// (LevelSetPy, arXiv 2411.03501, Sec. IV-V), so every instance gets the same
// bits as its own hjx_solve.  The host captures the launches of one horizon
// in a hipGraph and replays it.
#include "hjx_device.h"

namespace hjx {
namespace {

using namespace dev;

constexpr int kBatchThreads = 256;

// Stage pointers and coefficients of RK stage `stage` of step s (the same
// ones hjx_solve uses for this instance).
template <typename T>
__device__ __forceinline__ StageArgs<T> batch_stage(const BatchInst<T> &I, int s, int stage, int rk)
{
    StageArgs<T> a = I.st;
    a.dt = s == I.steps - 1 ? I.dt_last : I.dt;
    a.rhs_only = 0;
    a.mask = nullptr;
    a.dp_out = nullptr;
    a.phi_n = nullptr;
    a.ca = T(0);
    a.cb = T(1);
    a.target = stage == rk - 1 ? I.target : nullptr;
    if (rk == 1) {  // forward Euler alternates between phi and ws0
        a.phi_in = (s & 1) ? I.ws0 : I.phi;
        a.out = (s & 1) ? I.phi : I.ws0;
    } else if (stage == 0) {  // phi + h L(phi)
        a.phi_in = I.phi;
        a.out = I.ws0;
    } else if (rk == 2) {  // 1/2 phi^n + 1/2 (phi1 + h L(phi1))
        a.phi_in = I.ws0;
        a.phi_n = I.phi;
        a.out = I.phi;
        a.ca = T(0.5);
        a.cb = T(0.5);
    } else if (stage == 1) {  // 3/4 phi^n + 1/4 (phi1 + h L(phi1))
        a.phi_in = I.ws0;
        a.phi_n = I.phi;
        a.out = I.ws1;
        a.ca = T(0.75);
        a.cb = T(0.25);
    } else {  // 1/3 phi^n + 2/3 (phi_half + h L(phi_half))
        a.phi_in = I.ws1;
        a.phi_n = I.phi;
        a.out = I.phi;
        a.ca = T(1.0 / 3.0);
        a.cb = T(2.0 / 3.0);
    }
    return a;
}

// Nodes [f0, f1) of one instance; flat index -> grid index by multiplying
// with a rounded reciprocal of n and correcting by one either way.
template <typename T, int D, int SCHEME, int HAM, int MODE>
__device__ __forceinline__ void batch_run(const StageArgs<T> &a, int f0, int f1)
{
    double rn[kMaxDim];
#pragma unroll
    for (int d = 1; d < D; ++d) rn[d] = 1.0 / (double)a.g.n[d];
    for (int f = f0 + (int)threadIdx.x; f < f1; f += kBatchThreads) {
        int j[kMaxDim] = {0, 0, 0, 0};
        int rem = f;
#pragma unroll
        for (int d = D - 1; d >= 1; --d) {
            const int n = a.g.n[d];
            int q = (int)((double)rem * rn[d]);
            int r = rem - q * n;
            if (r < 0) {
                --q;
                r += n;
            } else if (r >= n) {
                ++q;
                r -= n;
            }
            j[d] = r;
            rem = q;
        }
        j[0] = rem;
        direct_node<T, D, SCHEME, HAM, MODE>(a, j);
    }
}

// CLIP: some instance has a restricted update (each applies its own a.clip,
// which may be 0); batches without one never compile the clip.  EXT: some
// instance plays the rockets game or takes the local dissipation or
// Godunov's Hamiltonian (a.diss); batches without one never compile those,
// whose registers would set the occupancy of every batch.
template <typename T, int SCHEME, bool CLIP, bool EXT>
__global__ __launch_bounds__(kBatchThreads) void batch_kernel(const BatchInst<T> *__restrict__ inst, BatchArgs<T> b)
{
    constexpr int M = CLIP ? kNodeClip : kNodePlain;
    // XCD-aware order: the hardware deals consecutive blocks round-robin to
    // the 8 XCDs; renumber so that each XCD walks a contiguous run of items
    // (neighbouring nodes of an instance share halo lines in that XCD's L2).
    const int G = (int)gridDim.x;
    int vb = (int)blockIdx.x;
    if ((G & 7) == 0) vb = (vb & 7) * (G >> 3) + (vb >> 3);
    for (int item = vb; item < b.items; item += G) {
        // the instance owning this item: the last one with item0 <= item
        int lo = 0, hi = b.n_active - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (inst[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchInst<T> &I = inst[lo];
        const int f0 = (item - I.item0) * b.item_nodes;
        const int f1 = min(I.total, f0 + b.item_nodes);
        if (b.stage < 0) {
            if (b.stage == kBatchCopyIn) {
                for (int f = f0 + (int)threadIdx.x; f < f1; f += kBatchThreads) I.phi[f] = I.phi0[f];
            } else if (b.stage == kBatchCopyOut) {
                if (I.steps & 1)
                    for (int f = f0 + (int)threadIdx.x; f < f1; f += kBatchThreads) I.phi[f] = I.ws0[f];
            } else {
                const T *x = b.stage == kBatchCheckIn ? I.phi0 : I.phi;
                bool bad = false;
                for (int f = f0 + (int)threadIdx.x; f < f1; f += kBatchThreads) bad |= !__builtin_isfinite(x[f]);
                if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(b.flags + lo, 1);
            }
            continue;
        }
        const StageArgs<T> a = batch_stage(I, b.s, b.stage, b.rk);
        if constexpr (EXT) {
            if (a.diss == 2) {  // Godunov's Hamiltonian for normal motion
                switch (a.g.dim) {
                case 1: batch_run<T, 1, SCHEME, kHamNormalGodunov, M>(a, f0, f1); break;
                case 2: batch_run<T, 2, SCHEME, kHamNormalGodunov, M>(a, f0, f1); break;
                case 3: batch_run<T, 3, SCHEME, kHamNormalGodunov, M>(a, f0, f1); break;
                default: batch_run<T, 4, SCHEME, kHamNormalGodunov, M>(a, f0, f1); break;
                }
                continue;
            }
            if (a.diss == 1) {  // alpha_d at the node
                constexpr int ML = M | kNodeLocal;
                if (I.ham == kHamDubins3) {
                    batch_run<T, 3, SCHEME, kHamDubins3, ML>(a, f0, f1);
                } else if (I.ham == kHamDubins4) {
                    batch_run<T, 4, SCHEME, kHamDubins4, ML>(a, f0, f1);
                } else if (I.ham == kHamRockets) {
                    batch_run<T, 3, SCHEME, kHamRockets, ML>(a, f0, f1);
                } else {
                    switch (a.g.dim) {
                    case 1: batch_run<T, 1, SCHEME, kHamNormal, ML>(a, f0, f1); break;
                    case 2: batch_run<T, 2, SCHEME, kHamNormal, ML>(a, f0, f1); break;
                    case 3: batch_run<T, 3, SCHEME, kHamNormal, ML>(a, f0, f1); break;
                    default: batch_run<T, 4, SCHEME, kHamNormal, ML>(a, f0, f1); break;
                    }
                }
                continue;
            }
            if (I.ham == kHamRockets) {
                batch_run<T, 3, SCHEME, kHamRockets, M>(a, f0, f1);
                continue;
            }
        }
        if (I.ham == kHamDubins3) {
            batch_run<T, 3, SCHEME, kHamDubins3, M>(a, f0, f1);
        } else if (I.ham == kHamDubins4) {
            batch_run<T, 4, SCHEME, kHamDubins4, M>(a, f0, f1);
        } else {
            switch (a.g.dim) {
            case 1: batch_run<T, 1, SCHEME, kHamNormal, M>(a, f0, f1); break;
            case 2: batch_run<T, 2, SCHEME, kHamNormal, M>(a, f0, f1); break;
            case 3: batch_run<T, 3, SCHEME, kHamNormal, M>(a, f0, f1); break;
            default: batch_run<T, 4, SCHEME, kHamNormal, M>(a, f0, f1); break;
            }
        }
    }
}

template <typename T, int SCHEME, bool CLIP, bool EXT>
int occupancy()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<T, SCHEME, CLIP, EXT>, kBatchThreads, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <typename T, bool CLIP, bool EXT>
int occupancy_t(int scheme)
{
    switch (scheme) {
    case kSchemeFirst: return occupancy<T, kSchemeFirst, CLIP, EXT>();
    case kSchemeEno2: return occupancy<T, kSchemeEno2, CLIP, EXT>();
    case kSchemeEno3: return occupancy<T, kSchemeEno3, CLIP, EXT>();
    default: return occupancy<T, kSchemeWeno5, CLIP, EXT>();
    }
}

template <typename T, bool CLIP, bool EXT>
hipError_t launch_batch_t(const BatchArgs<T> &a, int scheme, dim3 grid, hipStream_t s)
{
    switch (scheme) {
    case kSchemeFirst:
        hipLaunchKernelGGL((batch_kernel<T, kSchemeFirst, CLIP, EXT>), grid, dim3(kBatchThreads), 0, s, a.inst, a);
        break;
    case kSchemeEno2:
        hipLaunchKernelGGL((batch_kernel<T, kSchemeEno2, CLIP, EXT>), grid, dim3(kBatchThreads), 0, s, a.inst, a);
        break;
    case kSchemeEno3:
        hipLaunchKernelGGL((batch_kernel<T, kSchemeEno3, CLIP, EXT>), grid, dim3(kBatchThreads), 0, s, a.inst, a);
        break;
    case kSchemeWeno5:
        hipLaunchKernelGGL((batch_kernel<T, kSchemeWeno5, CLIP, EXT>), grid, dim3(kBatchThreads), 0, s, a.inst, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch(const BatchArgs<T> &a, int scheme, int blocks, hipStream_t s)
{
    if (a.items <= 0) return hipSuccess;
    const dim3 grid(blocks < a.items ? blocks : a.items);
    if (a.ext) return a.clip ? launch_batch_t<T, true, true>(a, scheme, grid, s)
                             : launch_batch_t<T, false, true>(a, scheme, grid, s);
    return a.clip ? launch_batch_t<T, true, false>(a, scheme, grid, s) : launch_batch_t<T, false, false>(a, scheme, grid, s);
}

}  // namespace

hipError_t launch_batch_f32(const BatchArgs<float> &a, int scheme, int blocks, hipStream_t s)
{
    return launch_batch<float>(a, scheme, blocks, s);
}
hipError_t launch_batch_f64(const BatchArgs<double> &a, int scheme, int blocks, hipStream_t s)
{
    return launch_batch<double>(a, scheme, blocks, s);
}
int batch_blocks_per_cu(int dtype_f64, int scheme, int clip, int ext)
{
    if (ext) {
        if (clip) return dtype_f64 ? occupancy_t<double, true, true>(scheme) : occupancy_t<float, true, true>(scheme);
        return dtype_f64 ? occupancy_t<double, false, true>(scheme) : occupancy_t<float, false, true>(scheme);
    }
    if (clip) return dtype_f64 ? occupancy_t<double, true, false>(scheme) : occupancy_t<float, true, false>(scheme);
    return dtype_f64 ? occupancy_t<double, false, false>(scheme) : occupancy_t<float, false, false>(scheme);
}

}  // namespace hjx
