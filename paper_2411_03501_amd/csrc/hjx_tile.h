// The tile kernel of 3-D and 4-D grids (the plane-march variant of the stage
// kernel there).  Method: LevelSetPy (arXiv 2411.03501), Sec. IV-A..IV-D
// (upwind derivatives, Lax-Friedrichs Hamiltonian), Sec. V (TVD-RK stages),
// Sec. VI (min-with-target); the per-interval and per-node arithmetic is
// hjx_device.h's, shared with every other variant.
#pragma once

#include "hjx_device.h"

namespace hjx {
namespace dev {

// ---------------------------------------------------------------- raw buffer access
//
// A raw buffer resource (stride 0) over `bytes` bytes from p: the base and the
// range sit in scalar registers and every load takes a 32-bit vector byte
// offset plus a 32-bit scalar byte offset, so a load costs no vector
// address arithmetic.  A load at or beyond the range reads zero instead of
// faulting.  The fourth word is the gfx9 family's
// raw-access format (32-bit data).
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, size_t bytes)
{
    const unsigned n = bytes < 0xFFFFFFFFull ? (unsigned)bytes : 0xFFFFFFFFu;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, kBufWord3);
}

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned vbyte, unsigned sbyte);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned vbyte, unsigned sbyte)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vbyte, sbyte, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned vbyte, unsigned sbyte)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vbyte, sbyte, 0));
}

// ---------------------------------------------------------------- tile kernel (3-D and 4-D)
//
// The seven planes of the gathered axis for one of the six end lines of a
// non-periodic axis 1 (CASE 0..2: lines 0..2; 3..5: lines n-3..n-1): the
// planes inside the grid through one buffer, then each ghost plane by
// gather7's linear extrapolation from the two end planes, which are among
// those just loaded (the same arithmetic, so the same bits).
template <typename T, int CASE>
__device__ __forceinline__ void end_line_planes(const T *pk, int jd, int sg, size_t pbytes, int off, T (&v)[7])
{
    constexpr bool low = CASE < 3;
    constexpr int first = low ? 3 - CASE : 0, last = low ? 6 : 5 - (CASE - 3);  // planes inside the grid
    const __amdgpu_buffer_rsrc_t r =
        buf_rsrc(pk + (ptrdiff_t)(jd - 3 + first) * (ptrdiff_t)sg, (size_t)(last - first + 1) * pbytes);
#pragma unroll
    for (int m = first; m <= last; ++m)
        v[m] = buf_ld<T>(r, (unsigned)off * sizeof(T), (unsigned)((m - first) * sg) * sizeof(T));
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        if (m < first) v[m] = fmaT(T(first - m), v[first] - v[first + 1], v[first]);
        if (m > last) v[m] = fmaT(T(m - last), v[last] - v[last - 1], v[last]);
    }
}

// FP32: at least six waves per SIMD (at most 80 vector registers); left to
// itself the compiler takes 81 for the 4-D WENO5 kernel, which allows five.
template <typename T>
constexpr int tile_min_waves() { return sizeof(T) == 4 ? 6 : 1; }

// NT threads own a tile of TX x TY nodes of the plane of the two fastest
// axes (AF along the lanes, AM across; TX * TY <= 512, so at most 512 / NT
// nodes per thread) and march over `march` consecutive nodes of the slowest axis
// AK = 0.  In 4-D axis 1 is gathered node by node from seven planes that lie
// one plane of AM x AF apart, close enough to share one L2.  Per marched
// plane:
//   1. the tile's halo, three nodes beyond it on both plane axes, is staged
//      in LDS (ghosts filled; the tile's corners are never read and never
//      staged), and every thread writes its own nodes from its marched queue;
//   2. every interval of the tile along AF (TY rows of TX + 1) and along AM
//      (TY + 1 rows of TX) is evaluated exactly once, the items dealt evenly
//      over the NT threads, and its two one-sided values go to LDS;
//   3. each thread finishes its nodes: the marched axis from a register
//      queue of seven values (the interval right of the node, its left half
//      kept for the next plane), axis 1 in 4-D (both sides at the node), then
//      the plane axes' values from LDS, the Hamiltonian, the stage
//      combination, the store.
// Each interval goes through the same interval() arithmetic as in every
// other variant, so the bits do not depend on the launch shape.  Addresses
// are 32-bit offsets inside one plane (seven planes for the gathered axis)
// from a 64-bit base that is the same for the whole block (the host checks
// that they fit in 4 GiB).
// Blocks are renumbered so that each XCD takes a contiguous run of them with
// axis 1 varying fastest (4-D): the planes a node's axis-1 stencil reads are
// then read by neighbouring blocks of the same XCD, through its L2.
// In 4-D a stage is two launches (LINES): the lines of axis 1 whose seven
// planes all lie inside the grid, which read them through one buffer
// resource, and the six end lines, whose ghost planes are extrapolated
// (end_line_planes) or wrapped; a grid with fewer than seven lines takes one
// launch over all of them.
template <typename T, int D, int SCHEME, int HAM, int MODE, int NT, int LINES>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(tile_min_waves<T>())))
void stage_tile_kernel(StageArgs<T> a, TileLaunch tl)
{
    constexpr int NPT = kTileNodes / NT;  // nodes per thread
    static_assert(D == 3 || D == 4, "the tile kernel marches axis 0 of a 3-D or 4-D grid");
    static_assert((MODE & kNodeKeep) == 0, "kept p-, p+ (and the target mask) come from the direct variant");
    constexpr int AF = D - 1, AM = D - 2, AK = 0, AG = 1;  // AG: the gathered axis of a 4-D grid
    extern __shared__ unsigned char smem_raw[];
    const int TX = a.tile.tx, TY = a.tile.ty, LW = TX + 6;
    T *S = reinterpret_cast<T *>(smem_raw);  // (TY + 6) x LW: the plane tile and its halo
    T *PMf = S + (TY + 6) * LW;              // TY x TX one-sided values of each node, AF and AM
    T *PPf = PMf + TX * TY;
    T *PMm = PPf + TX * TY;
    T *PPm = PMm + TX * TY;

    const int b = (int)blockIdx.x;
    const int lb = (b & 7) * ((int)gridDim.x >> 3) + (b >> 3);
    if (lb >= tl.blocks) return;  // padding to a multiple of 8 blocks (whole block)
    int rest = lb;
    int jd = 0;
    if constexpr (D == 4) {
        jd = rest % tl.outer;
        rest /= tl.outer;
        if constexpr (LINES == kTileLinesInterior) jd += tl.y_first;
        if constexpr (LINES == kTileLinesEnds || LINES == kTileLinesEndsWrap) jd = jd < 3 ? jd : a.g.n[AG] - 6 + jd;
    }
    const int tf = rest % tl.tiles_f;
    rest /= tl.tiles_f;
    const int tm = rest % tl.tiles_m;
    const int kc = rest / tl.tiles_m;

    const int nf = a.g.n[AF], nm = a.g.n[AM], nk = a.g.n[AK];
    const int sm = a.g.stride[AM];
    const size_t sk = (size_t)a.g.stride[AK];
    const bool per_f = (a.g.periodic >> AF) & 1u, per_m = (a.g.periodic >> AM) & 1u;
    const bool per_k = (a.g.periodic >> AK) & 1u;
    const int jf0 = tf * TX, jm0 = tm * TY;
    const int txv = min(TX, nf - jf0), tyv = min(TY, nm - jm0);  // the tile's nodes inside the grid
    const int k0 = kc * a.tile.march, k1 = min(k0 + a.tile.march, nk);
    const size_t slab = D == 4 ? (size_t)jd * (size_t)a.g.stride[AG] : 0;

    // bytes of one plane of the tile's two axes: what one buffer range covers
    const size_t pbytes = (size_t)(D == 4 ? a.g.stride[AG] : a.g.stride[AK]) * sizeof(T);
    const T *__restrict__ phi = a.phi_in + slab;

    // phi at plane kk (a ghost plane beyond a non-periodic end is
    // extrapolated linearly from the two end planes; kk is within three of
    // [0, nk), so one wrap suffices on a periodic axis)
    auto march_at = [&](int kk, int off) -> T {
        if (kk >= 0 && kk < nk) return ld32(phi + (size_t)kk * sk, off);
        if (per_k) return ld32(phi + (size_t)(kk < 0 ? kk + nk : kk - nk) * sk, off);
        const int e = kk < 0 ? 0 : nk - 1, e2 = kk < 0 ? 1 : nk - 2;
        const T c = T(kk < 0 ? -kk : kk - (nk - 1));
        const T p0 = ld32(phi + (size_t)e * sk, off), p1 = ld32(phi + (size_t)e2 * sk, off);
        return fmaT(c, p0 - p1, p0);
    };

    // the thread's nodes: n = t + NT i of the tile, row n / TX, column n % TX
    const int t = (int)threadIdx.x;
    // index reciprocals: one-ulp rcp keeps the floors below exact (indices < 2^20)
    const float rtx = __builtin_amdgcn_rcpf((float)TX);
    bool valid[NPT];
    int rr[NPT], cc[NPT], off[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int n = t + NT * i;
        int r = (int)(((float)n + 0.5f) * rtx);  // exact: the fraction stays 0.5/TX from an integer
        const int c = n - r * TX;
        rr[i] = r;
        cc[i] = c;
        valid[i] = n < TX * TY && r < tyv && c < txv;
        off[i] = (jm0 + r) * sm + jf0 + c;
    }

    T q[NPT][7];        // marched axis: phi at k-3 .. k+3 of each node
    T pm_k[NPT];  // left-biased derivative of each node along AK at the current plane
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        pm_k[i] = T(0);
        if (valid[i]) {
#pragma unroll
            for (int m = 0; m < 7; ++m) q[i][m] = march_at(k0 - 3 + m, off[i]);
            T unused;
            interval<T, SCHEME>(q[i], a.inv_dx[AK], a.dx[AK], pm_k[i], unused);
        }
    }

    const int band = 6 * txv, side = 6 * tyv;
    const float rtxv = __builtin_amdgcn_rcpf((float)txv), rtx1 = __builtin_amdgcn_rcpf((float)(txv + 1));
    const int items_f = tyv * (txv + 1), items_m = (tyv + 1) * txv;

    // the gathered axis of a 4-D grid: all seven planes inside the grid for
    // every block of an interior launch (one buffer over them), ghost rules
    // otherwise
    constexpr bool YIN = D == 3 || LINES == kTileLinesInterior;
    for (int k = k0; k < k1; ++k) {
        const T *base = phi + (size_t)k * sk;
        // 1. halo: three rows above and below the tile (inside its columns)
        for (int h = t; h < band; h += NT) {
            const int bi = (int)(((float)h + 0.5f) * rtxv);
            const int c = h - bi * txv;
            const int r = bi < 3 ? bi : tyv + bi;  // S rows 0..2 and tyv+3..tyv+5
            const int y = jm0 + r - 3, x = jf0 + c;
            T v;
            if (y >= 0 && y < nm) {
                v = ld32(base, y * sm + x);
            } else if (per_m) {
                v = ld32(base, (y < 0 ? y + nm : y - nm) * sm + x);
            } else {
                const int e = y < 0 ? 0 : nm - 1, e2 = y < 0 ? 1 : nm - 2;
                const T cf = T(y < 0 ? -y : y - (nm - 1));
                const T p0 = ld32(base, e * sm + x), p1 = ld32(base, e2 * sm + x);
                v = fmaT(cf, p0 - p1, p0);
            }
            S[r * LW + c + 3] = v;
        }
        //    and three columns left and right of it (inside its rows)
        for (int h = t; h < side; h += NT) {
            const int r = 3 + h / 6, ci = h - (h / 6) * 6;
            const int c = ci < 3 ? ci : txv + ci;  // S columns 0..2 and txv+3..txv+5
            const int y = jm0 + r - 3, x = jf0 + c - 3;
            T v;
            if (x >= 0 && x < nf) {
                v = ld32(base, y * sm + x);
            } else if (per_f) {
                v = ld32(base, y * sm + (x < 0 ? x + nf : x - nf));
            } else {
                const int e = x < 0 ? 0 : nf - 1, e2 = x < 0 ? 1 : nf - 2;
                const T cf = T(x < 0 ? -x : x - (nf - 1));
                const T p0 = ld32(base, y * sm + e), p1 = ld32(base, y * sm + e2);
                v = fmaT(cf, p0 - p1, p0);
            }
            S[r * LW + c] = v;
        }
        //    and the tile itself, from the marched queues
#pragma unroll
        for (int i = 0; i < NPT; ++i)
            if (valid[i]) S[(rr[i] + 3) * LW + cc[i] + 3] = q[i][3];
        __syncthreads();

        // 2. every interval of the tile, once: along AF between columns c-1
        //    and c of row r (c = 0 .. txv), along AM between rows r-1 and r of
        //    column c (r = 0 .. tyv)
        for (int e = t; e < items_f; e += NT) {
            const int r = (int)(((float)e + 0.5f) * rtx1);
            const int c = e - r * (txv + 1);
            T pm, pp;
            interval<T, SCHEME>(&S[(r + 3) * LW + c], a.inv_dx[AF], a.dx[AF], pm, pp);
            if (c < txv) PMf[r * TX + c] = pm;
            if (c > 0) PPf[r * TX + c - 1] = pp;
        }
        for (int e = t; e < items_m; e += NT) {
            const int r = (int)(((float)e + 0.5f) * rtxv);
            const int c = e - r * txv;
            T v[6], pm, pp;
#pragma unroll
            for (int m = 0; m < 6; ++m) v[m] = S[(r + m) * LW + c + 3];
            interval<T, SCHEME>(v, a.inv_dx[AM], a.dx[AM], pm, pp);
            if (r < tyv) PMm[r * TX + c] = pm;
            if (r > 0) PPm[(r - 1) * TX + c] = pp;
        }
        __syncthreads();

        // 3. the thread's nodes (this plane's arrays: uniform bases, 32-bit offsets)
        const size_t po = slab + (size_t)k * sk;
        const T *phin_p = a.phi_n ? a.phi_n + po : nullptr;
        const T *tgt_p = a.target ? a.target + po : nullptr;
        T *outp = a.out + po;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            if (!valid[i]) continue;
            const int n = t + NT * i;
            T pm[D], pp[D];
            T pm_next;
            interval<T, SCHEME>(q[i] + 1, a.inv_dx[AK], a.dx[AK], pm_next, pp[AK]);
            pm[AK] = pm_k[i];
            pm_k[i] = pm_next;
            // the marched axis done before the gathered axis' loads are issued
            // and before the scheduler may start on them: fewer registers live
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
            int j[kMaxDim] = {0, 0, 0, 0};
            j[AF] = jf0 + cc[i];
            j[AM] = jm0 + rr[i];
            j[AK] = k;
            if constexpr (D == 4) {  // axis 1: seven planes, both sides at the node
                j[AG] = jd;
                const int ng = a.g.n[AG], sg = a.g.stride[AG];
                const T *pk = a.phi_in + (size_t)k * sk;
                T v[7];
                if constexpr (YIN) {  // one buffer over the seven planes
                    const __amdgpu_buffer_rsrc_t ry = buf_rsrc(pk + (size_t)(jd - 3) * (size_t)sg, 7 * pbytes);
#pragma unroll
                    for (int m = 0; m < 7; ++m)
                        v[m] = buf_ld<T>(ry, (unsigned)off[i] * sizeof(T), (unsigned)(m * sg) * sizeof(T));
                } else if constexpr (LINES == kTileLinesEnds) {  // block-uniform: which end line
                    const int line = jd < 3 ? jd : jd - (ng - 6);
                    switch (line) {
                    case 0: end_line_planes<T, 0>(pk, jd, sg, pbytes, off[i], v); break;
                    case 1: end_line_planes<T, 1>(pk, jd, sg, pbytes, off[i], v); break;
                    case 2: end_line_planes<T, 2>(pk, jd, sg, pbytes, off[i], v); break;
                    case 3: end_line_planes<T, 3>(pk, jd, sg, pbytes, off[i], v); break;
                    case 4: end_line_planes<T, 4>(pk, jd, sg, pbytes, off[i], v); break;
                    default: end_line_planes<T, 5>(pk, jd, sg, pbytes, off[i], v); break;
                    }
                } else
#pragma unroll
                for (int m = 0; m < 7; ++m) {  // yy is the same for the whole block
                    const int yy = jd + m - 3;
                    if (yy >= 0 && yy < ng) {
                        v[m] = ld32(pk + (size_t)yy * (size_t)sg, off[i]);
                    } else if ((a.g.periodic >> AG) & 1u) {
                        v[m] = ld32(pk + (size_t)(yy < 0 ? yy + ng : yy - ng) * (size_t)sg, off[i]);
                    } else {
                        const int e = yy < 0 ? 0 : ng - 1, e2 = yy < 0 ? 1 : ng - 2;
                        const T cf = T(yy < 0 ? -yy : yy - ng + 1);
                        const T p0 = ld32(pk + (size_t)e * (size_t)sg, off[i]);
                        const T p1 = ld32(pk + (size_t)e2 * (size_t)sg, off[i]);
                        v[m] = fmaT(cf, p0 - p1, p0);
                    }
                }
                node_derivs<T, SCHEME>(v, a.inv_dx[AG], a.dx[AG], pm[AG], pp[AG]);
            }
            pm[AF] = PMf[n];  // the plane axes' values last: short live ranges
            pp[AF] = PPf[n];
            pm[AM] = PMm[n];
            pp[AM] = PPm[n];
            at32(outp, off[i]) =
                stage_result_at<T, D, HAM, MODE>(a, phin_p, tgt_p, nullptr, j, pm, pp, q[i][3], off[i]);
            // a further node's loads and arithmetic after this node's store:
            // two nodes' temporaries are never live together
            asm volatile("" ::: "memory");
        }

        if (k + 1 < k1) {  // advance the marched queues
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                if (!valid[i]) continue;
#pragma unroll
                for (int m = 0; m < 6; ++m) q[i][m] = q[i][m + 1];
                q[i][6] = march_at(k + 4, off[i]);
            }
        }
    }
}

}  // namespace dev
}  // namespace hjx
