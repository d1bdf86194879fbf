// HIP kernels for gfx950: the fused level-set stage (upwind derivatives along
// every axis -> Lax-Friedrichs Hamiltonian -> TVD-RK combination ->
// min-with-target), the dissipation reduction and small helpers.
//
// Method: LevelSetPy (arXiv 2411.03501).  Derivatives: Sec. IV-A (first
// order), Sec. IV-B (ENO2/ENO3), Sec. IV-C (WENO5); Lax-Friedrichs
// Hamiltonian and its global dissipation: Sec. IV-D with Listing 4
// (termLaxFriedrichs, artificialDissipationGLF); stage combinations: Sec. V
// (odeCFL1/2/3); min-with-target: Sec. VI (variational HJ PDE).
//
// Layout: row-major, last axis fastest.  The fastest axis runs along the
// lanes of a wave, so every row load is coalesced; see the stage kernel for
// the tiling.
#include "hjx_device.h"
#include "hjx_tile.h"

#include <cstdint>
#include <type_traits>

namespace hjx {
namespace {

using namespace dev;

// threads per block of the tile kernel (one node each at 512)
constexpr int kTileThreads = 512;

// ---------------------------------------------------------------- stage kernel
//
// A block owns a plane tile of TX x TY nodes (fastest axis x second-fastest
// axis) and marches over `march` consecutive nodes of the third axis.  Per
// marched plane:
//   1. the tile and a 3-node halo on both plane axes are staged in LDS, ghost
//      cells filled (periodic wrap or linear extrapolation);
//   2. every thread evaluates ONE interval per plane axis (the one to the left
//      of its node): it yields the node's left-biased derivative and the
//      right-biased derivative of the node to its left, which goes through
//      LDS; the last node of each row/column gets its interval from an extra
//      evaluation;
//   3. along the marched axis a register queue of 7 values does the same
//      with no exchange: the interval right of the node is evaluated and its
//      left-biased half is kept for the next plane;
//   4. the fourth axis (dim 4) is gathered from global memory, both sides at
//      the node;
//   5. Hamiltonian, LF dissipation, RK combination, min with target, store.
// Each interval is evaluated by exactly the same arithmetic whichever thread
// or tile evaluates it, so results do not depend on the launch shape.
// MODE: kNodePlain, or kNodeClip and kNodeLocal bits (hjx_device.h).


template <typename T, int D, int SCHEME, int HAM, int MODE>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs<T> a)
{
    constexpr int AF = D - 1;  // fastest axis: along the lanes
    constexpr int AM = D - 2;  // second axis: tile rows (dim >= 2)
    constexpr int AK = D - 3;  // third axis: marched (dim >= 3)
    extern __shared__ unsigned char smem_raw[];

    const int TX = blockDim.x, TY = blockDim.y;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx, nthr = TX * TY;
    const int LW = TX + 6;                    // staged row pitch
    T *S = reinterpret_cast<T *>(smem_raw);   // (TY + 6) x LW staged plane
    T *PPf = S + (TY + 6) * LW;               // TY x (TX + 1): right-biased, fast axis
    T *PPm = PPf + TY * (TX + 1);             // (TY + 1) x TX: right-biased, second axis

    const T *__restrict__ phi = a.phi_in;
    const int nf = a.g.n[AF];
    const int nm = D >= 2 ? a.g.n[AM] : 1;
    const int sm = D >= 2 ? a.g.stride[AM] : 0;
    const bool per_f = (a.g.periodic >> AF) & 1u;
    const bool per_m = D >= 2 && ((a.g.periodic >> AM) & 1u);
    const int tiles_f = (nf + TX - 1) / TX;
    const int jf0 = (blockIdx.x % tiles_f) * TX, jm0 = (blockIdx.x / tiles_f) * TY;
    const int jf = jf0 + tx, jm = jm0 + ty;
    const bool valid = jf < nf && jm < nm;
    const int off = jm * sm + jf;  // node offset inside its plane

    int k0 = 0, k1 = 1, nk = 1, sk = 0, jd = 0, base_d = 0;
    bool per_k = false;
    if constexpr (D >= 3) {
        nk = a.g.n[AK];
        sk = a.g.stride[AK];
        per_k = (a.g.periodic >> AK) & 1u;
        const int M = a.tile.march;
        const int nchunks = (nk + M - 1) / M;
        k0 = (blockIdx.y % nchunks) * M;
        k1 = min(k0 + M, nk);
        if constexpr (D == 4) {
            jd = blockIdx.y / nchunks;
            base_d = jd * a.g.stride[0];
        }
    }

    // phi at (plane base, second-axis index y, fast-axis index x) with ghosts
    // in the plane; a cell outside on both axes is never read
    auto plane_at = [&](int base, int y, int x) -> T {
        const bool xo = x < 0 || x >= nf, yo = y < 0 || y >= nm;
        if (xo && yo) return T(0);
        if (xo) {
            if (per_f) return phi[base + y * sm + wrap_index<T>(x, nf)];
            const int e = x < 0 ? 0 : nf - 1, e2 = x < 0 ? 1 : nf - 2;
            const T c = T(x < 0 ? -x : x - (nf - 1));
            const T p0 = phi[base + y * sm + e], p1 = phi[base + y * sm + e2];
            return fmaT(c, p0 - p1, p0);
        }
        if (yo) {
            if (per_m) return phi[base + wrap_index<T>(y, nm) * sm + x];
            const int e = y < 0 ? 0 : nm - 1, e2 = y < 0 ? 1 : nm - 2;
            const T c = T(y < 0 ? -y : y - (nm - 1));
            const T p0 = phi[base + e * sm + x], p1 = phi[base + e2 * sm + x];
            return fmaT(c, p0 - p1, p0);
        }
        return phi[base + y * sm + x];
    };
    // phi at marched index k of this thread's node (k may be a ghost; k is
    // the same for the whole block, so the branches do not diverge)
    auto march_at = [&](int k) -> T {
        if (k >= 0 && k < nk) return phi[base_d + k * sk + off];
        if (per_k) return phi[base_d + wrap_index<T>(k, nk) * sk + off];
        const int e = k < 0 ? 0 : nk - 1, e2 = k < 0 ? 1 : nk - 2;
        const T c = T(k < 0 ? -k : k - (nk - 1));
        const T p0 = phi[base_d + e * sk + off], p1 = phi[base_d + e2 * sk + off];
        return fmaT(c, p0 - p1, p0);
    };

    // per-node Hamiltonian coordinates that do not change while marching
    int j[kMaxDim] = {0, 0, 0, 0};
    j[AF] = jf;
    if constexpr (D >= 2) j[AM] = jm;
    if constexpr (D == 4) j[0] = jd;

    T q[7];            // marched axis: phi at k-3 .. k+3
    T pm_k = T(0);     // left-biased derivative of the current node along the marched axis
    if constexpr (D >= 3) {
        if (valid) {
#pragma unroll
            for (int i = 0; i < 7; ++i) q[i] = march_at(k0 - 3 + i);
            T unused;
            interval<T, SCHEME>(q, a.inv_dx[AK], a.dx[AK], pm_k, unused);
        }
    }

    for (int k = k0; k < k1; ++k) {
        const int base = base_d + k * sk;
        // 1. stage the plane tile with its halo
        T center;
        if constexpr (D >= 3)
            center = valid ? q[3] : plane_at(base, jm, jf);
        else
            center = plane_at(base, jm, jf);
        S[(ty + 3) * LW + tx + 3] = center;
        if constexpr (D >= 2) {
            for (int r = ty; r < 6; r += TY) {
                const int ly = r < 3 ? r : TY + r;
                S[ly * LW + tx + 3] = plane_at(base, jm0 + ly - 3, jf);
            }
        }
        for (int c = tx; c < 6; c += TX) {
            const int lx = c < 3 ? c : TX + c;
            S[(ty + 3) * LW + lx] = plane_at(base, jm, jf0 + lx - 3);
        }
        __syncthreads();

        // 2. one interval per plane axis
        T pm_f = T(0), pm_m = T(0);
        if (jm < nm && jf <= nf) {
            T ppl;
            interval<T, SCHEME>(&S[(ty + 3) * LW + tx], a.inv_dx[AF], a.dx[AF], pm_f, ppl);
            PPf[ty * (TX + 1) + tx] = ppl;
        }
        if (tid < TY) {  // interval right of the last node of row tid
            const int r = tid;
            if (jm0 + r < nm && jf0 + TX - 1 < nf) {
                T pmx, ppl;
                interval<T, SCHEME>(&S[(r + 3) * LW + TX], a.inv_dx[AF], a.dx[AF], pmx, ppl);
                PPf[r * (TX + 1) + TX] = ppl;
            }
        }
        if constexpr (D >= 2) {
            if (jf < nf && jm <= nm) {
                T v[6], ppl;
#pragma unroll
                for (int i = 0; i < 6; ++i) v[i] = S[(ty + i) * LW + tx + 3];
                interval<T, SCHEME>(v, a.inv_dx[AM], a.dx[AM], pm_m, ppl);
                PPm[ty * TX + tx] = ppl;
            }
            const int c = tid - (nthr - TX);  // interval below the last node of column c
            if (c >= 0 && jf0 + c < nf && jm0 + TY - 1 < nm) {
                T v[6], pmx, ppl;
#pragma unroll
                for (int i = 0; i < 6; ++i) v[i] = S[(TY + i) * LW + c + 3];
                interval<T, SCHEME>(v, a.inv_dx[AM], a.dx[AM], pmx, ppl);
                PPm[TY * TX + c] = ppl;
            }
        }

        // 3. marched axis: interval right of the node
        T pp_k = T(0), pm_kk = pm_k;
        if constexpr (D >= 3) {
            if (valid) {
                T pm_next;
                interval<T, SCHEME>(q + 1, a.inv_dx[AK], a.dx[AK], pm_next, pp_k);
                pm_k = pm_next;
            }
        }
        __syncthreads();

        if (valid) {
            T pm[D], pp[D];
            pm[AF] = pm_f;
            pp[AF] = PPf[ty * (TX + 1) + tx + 1];
            if constexpr (D >= 2) {
                pm[AM] = pm_m;
                pp[AM] = PPm[(ty + 1) * TX + tx];
            }
            if constexpr (D >= 3) {
                pm[AK] = pm_kk;
                pp[AK] = pp_k;
                j[AK] = k;
            }
            const int idx = base + off;
            if constexpr (D == 4) {  // 4. the slowest axis, both sides at the node
                T v[7];
                gather7(phi, idx, jd, a.g.n[0], a.g.stride[0], a.g.periodic & 1u, v);
                node_derivs<T, SCHEME>(v, a.inv_dx[0], a.dx[0], pm[0], pp[0]);
            }
            // 5. LF Hamiltonian and the stage combination
            a.out[idx] = stage_result<T, D, HAM, MODE>(a, j, pm, pp, center, idx);
        }

        if constexpr (D >= 3) {  // advance the marched queue
            if (valid && k + 1 < k1) {
#pragma unroll
                for (int i = 0; i < 6; ++i) q[i] = q[i + 1];
                q[6] = march_at(k + 4);
            }
        }
    }
}

// The direct variant: one thread per node, all axes gathered through the
// caches (fastest axis along the lanes), both halves evaluated at the node.
// Best for grids of a few million nodes, where the plane-march tiling cannot
// keep enough waves in flight.
// Whether the direct kernel gives each thread two neighbouring planes of
// axis 0 (direct_pair) instead of one node: in 2-D and 3-D, for FP64 (fewer
// quarter-rate reciprocals outweigh the registers) and, in FP32, for every
// scheme but WENO5 (fewer loads and shared axis-0 windows at 60 VGPRs,
// still 8 waves: ENO2 9.67 -> 8.76 us and ENO3 12.09 -> 11.33 us per stage
// on dubins3d 101^3).  FP32 WENO5 keeps one node per thread: pairs cost it
// occupancy.
template <typename T, int D, int SCHEME>
constexpr bool direct_pairs()
{
    return (D == 2 || D == 3) && (sizeof(T) == 8 || SCHEME != kSchemeWeno5);
}

// With pairs, 2-D: thread q takes rows 2 (q / n1) and 2 (q / n1) + 1 of
// column q % n1; 3-D: block row by takes planes 2 by and 2 by + 1.
template <typename T, int D, int SCHEME, int HAM, int MODE>
__device__ __forceinline__ void direct_stage(const StageArgs<T> &a)
{
    constexpr bool PAIR = direct_pairs<T, D, SCHEME>();
    // XCD-aware order: the hardware deals consecutive blocks round-robin to
    // the 8 XCDs, each with its own L2.  Renumber the blocks so that each
    // XCD takes a contiguous run of them: the rows a block's stencils reach
    // along the second-fastest axis then mostly sit in the same L2.
    const int G = (int)(gridDim.x * gridDim.y);
    int lb = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if ((G & 7) == 0) lb = (lb & 7) * (G >> 3) + (lb >> 3);
    const int bx = lb % (int)gridDim.x, by = lb / (int)gridDim.x;
    const int q = bx * 256 + threadIdx.x;
    if constexpr (D == 2 && PAIR) {
        const int n1 = a.g.n[1];
        if (q >= ((a.g.n[0] + 1) / 2) * n1) return;
        int pr = (int)((double)q / (double)n1);
        int jl = q - pr * n1;
        if (jl < 0) {
            --pr;
            jl += n1;
        } else if (jl >= n1) {
            ++pr;
            jl -= n1;
        }
        int j[kMaxDim] = {2 * pr, jl, 0, 0};
        if (j[0] + 1 < a.g.n[0]) direct_pair<T, D, SCHEME, HAM, MODE>(a, j);
        else direct_node<T, D, SCHEME, HAM, MODE>(a, j);
        return;
    }
    if (q >= a.g.plane) return;
    int j[kMaxDim] = {0, 0, 0, 0};
    if constexpr (D == 1) {
        j[0] = q;
    } else {
        const int nl = a.g.n[D - 1];
        int jm = (int)((double)q / (double)nl);
        int jl = q - jm * nl;
        if (jl < 0) {
            --jm;
            jl += nl;
        } else if (jl >= nl) {
            ++jm;
            jl -= nl;
        }
        j[D - 2] = jm;
        j[D - 1] = jl;
    }
    if constexpr (D <= 2) {  // one plane: no loop over the slow axes
        direct_node<T, D, SCHEME, HAM, MODE>(a, j);
        return;
    }
    if constexpr (D == 3 && PAIR) {
        for (int sp = by; 2 * sp < a.g.slow; sp += gridDim.y) {
            j[0] = 2 * sp;
            if (j[0] + 1 < a.g.n[0]) direct_pair<T, D, SCHEME, HAM, MODE>(a, j);
            else direct_node<T, D, SCHEME, HAM, MODE>(a, j);
        }
        return;
    }
    for (int sy = by; sy < a.g.slow; sy += gridDim.y) {
        if constexpr (D == 3) j[0] = sy;
        if constexpr (D == 4) {
            j[0] = sy / a.g.n[1];
            j[1] = sy - j[0] * a.g.n[1];
        }
        direct_node<T, D, SCHEME, HAM, MODE>(a, j);
    }
}

// FP32: at most 96 scalar registers, so that 8 waves fit on a SIMD (the
// vector registers allow 8; the compiler's own choice, about 106 scalar
// registers, allows 7).  The few scalar values over the cap live in vector
// lanes: a handful of lane moves per thread, against an eighth more waves
// to hide latency (about 2% faster at 101^3).  WENO keeps one node per
// thread: pairs need 75 vector registers (6 waves) and were 2% slower.
template <typename T, int D, int SCHEME, int HAM, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_num_sgpr(96))) void stage_direct_kernel(StageArgs<T> a)
{
    direct_stage<T, D, SCHEME, HAM, MODE>(a);
}

// FP64: the vector registers bound the occupancy, so no cap.  Pairs of
// axis-0 planes: in 3-D WENO a quarter fewer axis-0 windows, and so fewer
// quarter-rate FP64 reciprocals, outweigh 4 waves per SIMD instead of 5
// (29.0 -> 27.3 us per stage at 101^3); first order in 2-D reads 4 values
// per node instead of 5 (4.4 -> 4.8 TB/s at 4096^2).
template <typename T, int D, int SCHEME, int HAM, int MODE>
__global__ __launch_bounds__(256) void stage_direct_kernel_f64(StageArgs<T> a)
{
    direct_stage<T, D, SCHEME, HAM, MODE>(a);
}

// First order in 2-D, two x-neighbours per thread, for an even row length
// and arrays aligned to two elements: the two nodes' own values and those of
// the rows above and below come in as one vector access each, the two x
// halo values as scalars (5 loads for 2 nodes), and the results leave as one
// vector store.  Each node is assembled into the stencils direct_node would
// gather and goes through the same node_derivs and stage_result, so the
// bits are direct_node's; threads with a node on the grid's edge take
// direct_node itself.
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

template <typename T, int HAM, int MODE>
__global__ __launch_bounds__(256) void stage_x2_kernel(StageArgs<T> a)
{
    using T2 = typename Vec2<T>::type;
    const int ny = a.g.n[0], nx = a.g.n[1], hx = nx >> 1;
    const long q = (long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long)ny * hx) return;
    const int y = (int)(q / hx), x0 = 2 * (int)(q - (long)y * hx);
    int j[kMaxDim] = {y, x0, 0, 0};
    if (y < 1 || y > ny - 2 || x0 < 1 || x0 + 2 > nx - 1) {
        direct_node<T, 2, kSchemeFirst, HAM, MODE>(a, j);
        j[1] = x0 + 1;
        direct_node<T, 2, kSchemeFirst, HAM, MODE>(a, j);
        return;
    }
    const int idx = y * nx + x0;
    const T2 c = *reinterpret_cast<const T2 *>(a.phi_in + idx);
    const T2 up = *reinterpret_cast<const T2 *>(a.phi_in + (idx - nx));
    const T2 dn = *reinterpret_cast<const T2 *>(a.phi_in + (idx + nx));
    const T xl = ld32(a.phi_in, idx - 1), xr = ld32(a.phi_in, idx + 2);
    // the stencils gather7 would give (first order reads positions 2..4)
    T v0[7] = {T(0), T(0), up.x, c.x, dn.x, T(0), T(0)}, v1[7] = {T(0), T(0), xl, c.x, c.y, T(0), T(0)};
    T w0[7] = {T(0), T(0), up.y, c.y, dn.y, T(0), T(0)}, w1[7] = {T(0), T(0), c.x, c.y, xr, T(0), T(0)};
    T pm[2], pp[2], pm2[2], pp2[2];
    node_derivs<T, kSchemeFirst>(v0, a.inv_dx[0], a.dx[0], pm[0], pp[0]);
    node_derivs<T, kSchemeFirst>(v1, a.inv_dx[1], a.dx[1], pm[1], pp[1]);
    node_derivs<T, kSchemeFirst>(w0, a.inv_dx[0], a.dx[0], pm2[0], pp2[0]);
    node_derivs<T, kSchemeFirst>(w1, a.inv_dx[1], a.dx[1], pm2[1], pp2[1]);
    if constexpr ((MODE & kNodeKeep) != 0) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            at32(a.dp_out + (size_t)(2 * d) * (size_t)a.dp_stride, idx) = pm[d];
            at32(a.dp_out + (size_t)(2 * d + 1) * (size_t)a.dp_stride, idx) = pp[d];
            at32(a.dp_out + (size_t)(2 * d) * (size_t)a.dp_stride, idx + 1) = pm2[d];
            at32(a.dp_out + (size_t)(2 * d + 1) * (size_t)a.dp_stride, idx + 1) = pp2[d];
        }
    }
    const T r0 = stage_result<T, 2, HAM, MODE>(a, j, pm, pp, c.x, idx);
    j[1] = x0 + 1;
    const T r1 = stage_result<T, 2, HAM, MODE>(a, j, pm2, pp2, c.y, idx + 1);
    T2 r;
    r.x = r0;
    r.y = r1;
    *reinterpret_cast<T2 *>(a.out + idx) = r;
}

// whether stage_x2_kernel applies: 2-D first order, an even row length, and
// every array the stage reads or writes aligned to two elements
template <typename T, int D, int SCHEME>
bool x2_applies(const StageArgs<T> &a)
{
    if constexpr (D != 2 || SCHEME != kSchemeFirst) {
        return false;
    } else {
        auto al = [](const void *p) { return p == nullptr || ((uintptr_t)p % (2 * sizeof(T))) == 0; };
        return (a.g.n[1] % 2) == 0 && al(a.phi_in) && al(a.out) && (a.ca == T(0) || al(a.phi_n)) && al(a.target);
    }
}

// One stage launch in node mode M (bits of kNodeKeep, kNodeClip, kNodeLocal, kNodeMark).
template <typename T, int D, int SCHEME, int HAM, int M>
hipError_t launch_mode(const StageArgs<T> &a, hipStream_t s)
{
    const Tile t = a.tile;
    const int nf = a.g.n[D - 1], nm = D >= 2 ? a.g.n[D - 2] : 1;
    const int tiles = ((nf + t.tx - 1) / t.tx) * ((nm + t.ty - 1) / t.ty);
    int gy = 1;
    if (D >= 3) gy = (a.g.n[D - 3] + t.march - 1) / t.march;
    if (D == 4) gy *= a.g.n[0];
    if (D <= 2 && t.variant == kVariantPlaneMarch &&
        (t.tx < 1 || t.ty < 1 || t.tx * t.ty > 256 || (D == 1 && t.ty != 1) || t.march < 1 || gy > 65535))
        return hipErrorInvalidConfiguration;
    // only the direct variant keeps p-, p+ and marks clips; single stages of
    // a problem whose solves take the steps variant run direct
    if (t.variant == kVariantDirect || t.variant == kVariantSteps || (M & (kNodeKeep | kNodeMark)) != 0) {
        if (x2_applies<T, D, SCHEME>(a)) {
            const long threads = (long)a.g.n[0] * (a.g.n[1] / 2);
            const dim3 grid((unsigned)((threads + 255) / 256));
            hipLaunchKernelGGL((stage_x2_kernel<T, HAM, M>), grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
        // with pairs: half the planes (3-D) or half the rows (2-D)
        constexpr bool pairs = direct_pairs<T, D, SCHEME>();
        const int rows = D == 3 && pairs ? (a.g.slow + 1) / 2 : a.g.slow;
        const long cols = D == 2 && pairs ? (long)((a.g.n[0] + 1) / 2) * a.g.n[1] : (long)a.g.plane;
        dim3 grid((unsigned)((cols + 255) / 256), rows < 65535 ? rows : 65535);
        if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL((stage_direct_kernel<T, D, SCHEME, HAM, M>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((stage_direct_kernel_f64<T, D, SCHEME, HAM, M>), grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if constexpr ((M & (kNodeKeep | kNodeMark)) == 0) {
        if constexpr (D >= 3) {  // the tile kernel: 256 threads, up to 512 nodes of the plane tile
            if (t.tx < 1 || t.ty < 1 || t.tx * t.ty > 512 || t.march < 1) return hipErrorInvalidConfiguration;
            TileLaunch tl{};
            tl.tiles_f = (nf + t.tx - 1) / t.tx;
            tl.tiles_m = (nm + t.ty - 1) / t.ty;
            tl.chunks = (a.g.n[0] + t.march - 1) / t.march;  // the marched axis is axis 0
            const size_t lds = tile_lds_bytes(t, sizeof(T));
            // one launch over `lines` lines of the gathered axis (4-D), from y_first
            auto go = [&](auto kind, int lines, int y_first) -> hipError_t {
                constexpr int LINES = decltype(kind)::value;
                tl.outer = lines;
                tl.y_first = y_first;
                const long blocks = (long)tl.tiles_f * tl.tiles_m * tl.chunks * tl.outer;
                if (blocks > (1l << 30)) return hipErrorInvalidConfiguration;
                tl.blocks = (int)blocks;
                const unsigned grid = (unsigned)((blocks + 7) / 8 * 8);
                hipLaunchKernelGGL((stage_tile_kernel<T, D, SCHEME, HAM, M, kTileThreads, LINES>), dim3(grid),
                                   dim3(kTileThreads), lds, s, a, tl);
                return hipGetLastError();
            };
            using AllT = std::integral_constant<int, kTileLinesAll>;
            if constexpr (D == 3) {
                return go(AllT{}, 1, 0);
            } else {
                const int ng = a.g.n[1];
                if (ng < 7) return go(AllT{}, ng, 0);  // no line has its stencil inside
                const hipError_t e = go(std::integral_constant<int, kTileLinesInterior>{}, ng - 6, 3);
                if (e != hipSuccess) return e;
                if ((a.g.periodic >> 1) & 1u) return go(std::integral_constant<int, kTileLinesEndsWrap>{}, 6, 0);
                return go(std::integral_constant<int, kTileLinesEnds>{}, 6, 0);
            }
        } else {
            const size_t lds = stage_lds_bytes(t, sizeof(T));
            hipLaunchKernelGGL((stage_kernel<T, D, SCHEME, HAM, M>), dim3(tiles, gy), dim3(t.tx, t.ty), lds, s, a);
            return hipGetLastError();
        }
    }
    return hipErrorInvalidValue;
}

// The node mode of a stage: the replay for the adjoint keeps p-, p+ (when
// the tape stores them) and, for a restricted update, marks its clips in the
// mask; a clipped stage with a mask is such a replay (solves pass no mask).
// The local dissipation combines with all of these.  The right-hand side
// alone is never clipped.  Plain stages run the kernels without any of them.
template <typename T, int D, int SCHEME, int HAM>
hipError_t launch_one(const StageArgs<T> &a, hipStream_t s)
{
    const bool clip = !a.rhs_only && a.clip != 0;
    const int mode = (a.dp_out ? kNodeKeep : 0) | (clip ? kNodeClip : 0) | (clip && a.mask ? kNodeMark : 0) |
                     (a.diss == 1 ? kNodeLocal : 0);
    if constexpr (HAM == kHamNormalGodunov) {  // no alpha, so no local form
        switch (mode) {
        case kNodePlain: return launch_mode<T, D, SCHEME, HAM, kNodePlain>(a, s);
        case kNodeClip: return launch_mode<T, D, SCHEME, HAM, kNodeClip>(a, s);
        case kNodeKeep: return launch_mode<T, D, SCHEME, HAM, kNodeKeep>(a, s);
        case kNodeClip | kNodeMark: return launch_mode<T, D, SCHEME, HAM, kNodeClip | kNodeMark>(a, s);
        case kNodeKeep | kNodeClip | kNodeMark:
            return launch_mode<T, D, SCHEME, HAM, kNodeKeep | kNodeClip | kNodeMark>(a, s);
        }
        return hipErrorInvalidValue;
    }
    switch (mode) {
    case kNodePlain: return launch_mode<T, D, SCHEME, HAM, kNodePlain>(a, s);
    case kNodeKeep: return launch_mode<T, D, SCHEME, HAM, kNodeKeep>(a, s);
    case kNodeClip: return launch_mode<T, D, SCHEME, HAM, kNodeClip>(a, s);
    case kNodeClip | kNodeMark: return launch_mode<T, D, SCHEME, HAM, kNodeClip | kNodeMark>(a, s);
    case kNodeKeep | kNodeClip | kNodeMark:
        return launch_mode<T, D, SCHEME, HAM, kNodeKeep | kNodeClip | kNodeMark>(a, s);
    case kNodeLocal: return launch_mode<T, D, SCHEME, HAM, kNodeLocal>(a, s);
    case kNodeLocal | kNodeClip: return launch_mode<T, D, SCHEME, HAM, kNodeLocal | kNodeClip>(a, s);
    case kNodeKeep | kNodeLocal: return launch_mode<T, D, SCHEME, HAM, kNodeKeep | kNodeLocal>(a, s);
    case kNodeLocal | kNodeClip | kNodeMark:
        return launch_mode<T, D, SCHEME, HAM, kNodeLocal | kNodeClip | kNodeMark>(a, s);
    case kNodeKeep | kNodeLocal | kNodeClip | kNodeMark:
        return launch_mode<T, D, SCHEME, HAM, kNodeKeep | kNodeLocal | kNodeClip | kNodeMark>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D, int HAM>
hipError_t launch_scheme(const StageArgs<T> &a, int scheme, hipStream_t s)
{
    switch (scheme) {
    case kSchemeFirst: return launch_one<T, D, kSchemeFirst, HAM>(a, s);
    case kSchemeEno2: return launch_one<T, D, kSchemeEno2, HAM>(a, s);
    case kSchemeEno3: return launch_one<T, D, kSchemeEno3, HAM>(a, s);
    case kSchemeWeno5: return launch_one<T, D, kSchemeWeno5, HAM>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stage(const StageArgs<T> &a, int scheme, int ham, hipStream_t s)
{
    if (ham == kHamDubins3) {
        if (a.g.dim != 3) return hipErrorInvalidValue;
        return launch_scheme<T, 3, kHamDubins3>(a, scheme, s);
    }
    if (ham == kHamDubins4) {
        if (a.g.dim != 4) return hipErrorInvalidValue;
        return launch_scheme<T, 4, kHamDubins4>(a, scheme, s);
    }
    if (ham == kHamRockets) {
        if (a.g.dim != 3) return hipErrorInvalidValue;
        return launch_scheme<T, 3, kHamRockets>(a, scheme, s);
    }
    if (a.diss == 2) {  // Godunov's numerical Hamiltonian for normal motion
        switch (a.g.dim) {
        case 1: return launch_scheme<T, 1, kHamNormalGodunov>(a, scheme, s);
        case 2: return launch_scheme<T, 2, kHamNormalGodunov>(a, scheme, s);
        case 3: return launch_scheme<T, 3, kHamNormalGodunov>(a, scheme, s);
        case 4: return launch_scheme<T, 4, kHamNormalGodunov>(a, scheme, s);
        }
        return hipErrorInvalidValue;
    }
    switch (a.g.dim) {
    case 1: return launch_scheme<T, 1, kHamNormal>(a, scheme, s);
    case 2: return launch_scheme<T, 2, kHamNormal>(a, scheme, s);
    case 3: return launch_scheme<T, 3, kHamNormal>(a, scheme, s);
    case 4: return launch_scheme<T, 4, kHamNormal>(a, scheme, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- dissipation

constexpr int kAlphaThreads = 256;
constexpr int kAlphaMaxBlocks = 1024;

template <typename T>
__device__ __forceinline__ double partial_bound(const AlphaArgs<T> &a, const int *j, int d)
{
    if (a.ham == kHamNormal) return (double)vabs(a.hp[0]);
    if (a.ham == kHamDubins3) {
        const T ve = a.hp[0], vp = a.hp[1], we = a.hp[2], wp = a.hp[3];
        if (d == 0) return (double)(vabs(-ve + vp * a.tab.cosv[2][j[2]]) + we * vabs(a.tab.coord[1][j[1]]));
        if (d == 1) return (double)(vabs(vp * a.tab.sinv[2][j[2]]) + we * vabs(a.tab.coord[0][j[0]]));
        return (double)(we + wp);
    }
    if (a.ham == kHamRockets) {
        const T ac = a.hp[0], g = a.hp[1], ue = a.hp[2], up = a.hp[3];
        const T ax = vabs(a.tab.coord[0][j[0]]);
        if (d == 0) return (double)(vabs(ac * a.tab.cosv[2][j[2]]) + ue * ax);
        if (d == 1) return (double)(vabs(ac * a.tab.sinv[2][j[2]] + ac - g) + up * ax);
        return (double)(ue + up);
    }
    const T v = a.tab.coord[3][j[3]];
    if (d == 0) return (double)vabs(v * a.tab.cosv[2][j[2]]);
    if (d == 1) return (double)vabs(v * a.tab.sinv[2][j[2]]);
    if (d == 2) return (double)a.hp[0];
    return (double)a.hp[1];
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(x, off, 64);
        x = o > x ? o : x;
    }
    return x;
}

template <typename T>
__global__ __launch_bounds__(kAlphaThreads) void alpha_partial_kernel(AlphaArgs<T> a)
{
    double m[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
    for (int f = blockIdx.x * kAlphaThreads + threadIdx.x; f < a.total; f += gridDim.x * kAlphaThreads) {
        int j[kMaxDim];
        int r = f;
        for (int d = a.g.dim - 1; d >= 0; --d) {
            j[d] = r % a.g.n[d];
            r /= a.g.n[d];
        }
        for (int d = 0; d < a.g.dim; ++d) {
            const double b = partial_bound(a, j, d);
            m[d] = b > m[d] ? b : m[d];
        }
    }
    __shared__ double red[kAlphaThreads / 64][kMaxDim];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 0; d < kMaxDim; ++d) {
        const double w = wave_max(m[d]);
        if (lane == 0) red[wave][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < kMaxDim) {
        double b = red[0][threadIdx.x];
        for (int w = 1; w < kAlphaThreads / 64; ++w) b = red[w][threadIdx.x] > b ? red[w][threadIdx.x] : b;
        a.partial[blockIdx.x * kMaxDim + threadIdx.x] = b;
    }
}

__global__ __launch_bounds__(kAlphaThreads) void alpha_final_kernel(const double *partial, int blocks, int dim,
                                                                  double *alpha_out)
{
    double m[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < blocks; b += kAlphaThreads)
        for (int d = 0; d < kMaxDim; ++d) {
            const double x = partial[b * kMaxDim + d];
            m[d] = x > m[d] ? x : m[d];
        }
    __shared__ double red[kAlphaThreads / 64][kMaxDim];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 0; d < kMaxDim; ++d) {
        const double w = wave_max(m[d]);
        if (lane == 0) red[wave][d] = w;
    }
    __syncthreads();
    if (threadIdx.x < dim) {
        double b = red[0][threadIdx.x];
        for (int w = 1; w < kAlphaThreads / 64; ++w) b = red[w][threadIdx.x] > b ? red[w][threadIdx.x] : b;
        alpha_out[threadIdx.x] = b;
    }
}

template <typename T>
hipError_t launch_alpha(const AlphaArgs<T> &a, double *alpha_out, hipStream_t s)
{
    const int blocks = alpha_blocks(a.total);
    hipLaunchKernelGGL(alpha_partial_kernel<T>, dim3(blocks), dim3(kAlphaThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(alpha_final_kernel, dim3(1), dim3(kAlphaThreads), 0, s, a.partial, blocks, a.g.dim,
                       alpha_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- helpers

template <typename T>
__global__ __launch_bounds__(256) void nonfinite_kernel(const T *x, int n, int *flag)
{
    bool bad = false;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) bad |= !__builtin_isfinite(x[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

template <typename T>
__global__ __launch_bounds__(256) void copy_kernel(const T *src, T *dst, int n)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = src[i];
}

int stream_blocks(int n)
{
    const int b = (n + 255) / 256;
    return b < 4096 ? (b > 0 ? b : 1) : 4096;
}

}  // namespace

int alpha_blocks(int total)
{
    const int b = (total + kAlphaThreads - 1) / kAlphaThreads;
    return b < kAlphaMaxBlocks ? (b > 0 ? b : 1) : kAlphaMaxBlocks;
}

hipError_t launch_stage_f32(const StageArgs<float> &a, int scheme, int ham, hipStream_t s)
{
    return launch_stage<float>(a, scheme, ham, s);
}
hipError_t launch_stage_f64(const StageArgs<double> &a, int scheme, int ham, hipStream_t s)
{
    return launch_stage<double>(a, scheme, ham, s);
}
hipError_t launch_alpha_f32(const AlphaArgs<float> &a, double *alpha_out, hipStream_t s)
{
    return launch_alpha<float>(a, alpha_out, s);
}
hipError_t launch_alpha_f64(const AlphaArgs<double> &a, double *alpha_out, hipStream_t s)
{
    return launch_alpha<double>(a, alpha_out, s);
}
hipError_t launch_nonfinite_f32(const float *x, int n, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(stream_blocks(n)), dim3(256), 0, s, x, n, flag);
    return hipGetLastError();
}
hipError_t launch_nonfinite_f64(const double *x, int n, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(stream_blocks(n)), dim3(256), 0, s, x, n, flag);
    return hipGetLastError();
}
hipError_t launch_copy_f32(const float *src, float *dst, int n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel<float>, dim3(stream_blocks(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
hipError_t launch_copy_f64(const double *src, double *dst, int n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel<double>, dim3(stream_blocks(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace hjx
