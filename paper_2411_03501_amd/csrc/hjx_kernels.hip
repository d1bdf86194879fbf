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
#include "hjx_internal.h"

namespace hjx {
namespace {

// ---------------------------------------------------------------- arithmetic

template <typename T>
struct Arith;

template <>
struct Arith<float> {
    // one-ulp reciprocal: the WENO weights only need relative accuracy
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    // floor of the WENO epsilon: 1e-99 is zero in binary32; (1e-18)^2 is normal
    static constexpr float kEpsFloor = 1e-18f;
};

template <>
struct Arith<double> {
    // hardware reciprocal estimate refined by two Newton-Raphson steps
    // (r <- r + r (1 - x r)), each of which roughly doubles the correct bits:
    // a few ulp, against the ten-instruction IEEE division sequence.  The
    // operands here are sums of squares plus eps >= 1e-99, far from the
    // exponent range where the estimate needs pre-scaling.
    static __device__ __forceinline__ double rcp(double x)
    {
        double r = __builtin_amdgcn_rcp(x);
        double e = __builtin_fma(-x, r, 1.0);
        r = __builtin_fma(r, e, r);
        e = __builtin_fma(-x, r, 1.0);
        return __builtin_fma(r, e, r);
    }
    static __device__ __forceinline__ double div(double a, double b) { return a * rcp(b); }
    static constexpr double kEpsFloor = 1e-99;
};

template <typename T>
__device__ __forceinline__ T sq(T x) { return x * x; }

template <typename T>
__device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }

template <typename T>
__device__ __forceinline__ T vabs(T a) { return a < T(0) ? -a : a; }

// ---------------------------------------------------------------- derivatives

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Load base[i] through a 32-bit byte offset from a uniform base pointer, so
// the address is one scalar base plus one vector offset (arrays < 4 GiB; the
// host only launches the direct variant on such arrays).
template <typename T>
__device__ __forceinline__ T ld32(const T *base, int i)
{
    const unsigned off = (unsigned)i * (unsigned)sizeof(T);
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// Gather phi at offsets -3..3 along one axis of node idx (coordinate j of n,
// stride s), filling ghosts: periodic wrap, else linear extrapolation from
// the two end nodes.
template <typename T>
__device__ __forceinline__ void gather7(const T *__restrict__ phi, int idx, int j, int n, int s, bool per, T (&v)[7])
{
    if (j >= 3 && j < n - 3) {
#pragma unroll
        for (int k = 0; k < 7; ++k) v[k] = ld32(phi, idx + (k - 3) * s);
        return;
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        int jj = j + k - 3;
        if (per) {  // n >= 3 and |jj - j| <= 3, so one wrap lands in [0, n)
            jj = jj < 0 ? jj + n : (jj >= n ? jj - n : jj);
            v[k] = ld32(phi, idx + (jj - j) * s);
        } else if (jj < 0) {
            const T p0 = ld32(phi, idx - j * s), p1 = ld32(phi, idx + (1 - j) * s);
            v[k] = fmaT(T(-jj), p0 - p1, p0);
        } else if (jj >= n) {
            const T p0 = ld32(phi, idx + (n - 1 - j) * s), p1 = ld32(phi, idx + (n - 2 - j) * s);
            v[k] = fmaT(T(jj - n + 1), p0 - p1, p0);
        } else {
            v[k] = ld32(phi, idx + (k - 3) * s);
        }
    }
}

// WENO5 (Sec. IV-C) on one window of five one-sided differences u0..u4
// (D+ phi at I-2 .. I+2, I being the interval between nodes I and I+1).
// The left-biased value of node I+1 reads the window in order; the
// right-biased value of node I is its mirror image and reads it backwards.
// The smoothness indicators of the reversed window are those of the window
// itself, so both directions share S_k, eps and q_k = 1/(S_k + eps)^2, with
// the weights d = (0.1, 0.6, 0.3) on (q0, q1, q2) forwards and on
// (q2, q1, q0) backwards.
//
// Contraction is off and every fused multiply-add is written out, so the
// rounding of each value is fixed by the source: a value computed at any call
// site, by any kernel variant or tile, has the same bits.
template <typename T>
__device__ __forceinline__ void weno5_q(T u0, T u1, T u2, T u3, T u4, T &q0, T &q1, T &q2)
{
#pragma clang fp contract(off)
    const T k1312 = T(13.0 / 12.0), k14 = T(0.25);
    const T A0 = fmaT(T(-2), u1, u0 + u2), B0 = fmaT(T(-4), u1, fmaT(T(3), u2, u0));
    const T A1 = fmaT(T(-2), u2, u1 + u3), B1 = u1 - u3;
    const T A2 = fmaT(T(-2), u3, u2 + u4), B2 = fmaT(T(-4), u3, fmaT(T(3), u2, u4));
    const T s0 = fmaT(k1312 * A0, A0, k14 * B0 * B0);
    const T s1 = fmaT(k1312 * A1, A1, k14 * B1 * B1);
    const T s2 = fmaT(k1312 * A2, A2, k14 * B2 * B2);
    const T m = vmax(vmax(vmax(u0 * u0, u1 * u1), vmax(u2 * u2, u3 * u3)), u4 * u4);
    const T eps = fmaT(T(1e-6), m, Arith<T>::kEpsFloor);
    const T r0 = Arith<T>::rcp(s0 + eps), r1 = Arith<T>::rcp(s1 + eps), r2 = Arith<T>::rcp(s2 + eps);
    q0 = r0 * r0;
    q1 = r1 * r1;
    q2 = r2 * r2;
}

template <typename T>
__device__ __forceinline__ T weno5_fwd(T u0, T u1, T u2, T u3, T u4, T q0, T q1, T q2)
{
#pragma clang fp contract(off)
    const T c13 = T(1.0 / 3.0), c16 = T(1.0 / 6.0), c56 = T(5.0 / 6.0), c76 = T(7.0 / 6.0), c116 = T(11.0 / 6.0);
    const T f0 = fmaT(c13, u0, fmaT(-c76, u1, c116 * u2));
    const T f1 = fmaT(-c16, u1, fmaT(c56, u2, c13 * u3));
    const T f2 = fmaT(c13, u2, fmaT(c56, u3, -c16 * u4));
    const T a0 = T(0.1) * q0, a1 = T(0.6) * q1, a2 = T(0.3) * q2;
    return Arith<T>::div(fmaT(a0, f0, fmaT(a1, f1, a2 * f2)), a0 + a1 + a2);
}

template <typename T>
__device__ __forceinline__ T weno5_rev(T u0, T u1, T u2, T u3, T u4, T q0, T q1, T q2)
{
#pragma clang fp contract(off)
    const T c13 = T(1.0 / 3.0), c16 = T(1.0 / 6.0), c56 = T(5.0 / 6.0), c76 = T(7.0 / 6.0), c116 = T(11.0 / 6.0);
    const T g0 = fmaT(c13, u4, fmaT(-c76, u3, c116 * u2));
    const T g1 = fmaT(-c16, u3, fmaT(c56, u2, c13 * u1));
    const T g2 = fmaT(c13, u2, fmaT(c56, u1, -c16 * u0));
    const T b0 = T(0.1) * q2, b1 = T(0.6) * q1, b2 = T(0.3) * q0;
    return Arith<T>::div(fmaT(b0, g0, fmaT(b1, g1, b2 * g2)), b0 + b1 + b2);
}

template <typename T>
__device__ __forceinline__ void weno5_pair(T u0, T u1, T u2, T u3, T u4, T &fwd, T &rev)
{
    T q0, q1, q2;
    weno5_q(u0, u1, u2, u3, u4, q0, q1, q2);
    fwd = weno5_fwd(u0, u1, u2, u3, u4, q0, q1, q2);
    rev = weno5_rev(u0, u1, u2, u3, u4, q0, q1, q2);
}

// The interval I between nodes I and I+1 along one axis, from v[0..5] = phi
// at I-2 .. I+3: pm = left-biased derivative of node I+1, pp = right-biased
// derivative of node I.  Both start from the same divided difference
// D^1_{I+1/2}; ENO grows the same stencil for both (Sec. IV-B) and only the
// evaluation point differs; WENO5 uses the same window in both directions.
template <typename T, int SCHEME>
__device__ __forceinline__ void interval(const T *v, T inv_dx, T dx, T &pm, T &pp)
{
#pragma clang fp contract(off)
    if constexpr (SCHEME == kSchemeFirst) {
        pm = pp = (v[3] - v[2]) * inv_dx;
    } else if constexpr (SCHEME == kSchemeWeno5) {
        T u[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) u[k] = (v[k + 1] - v[k]) * inv_dx;
        weno5_pair(u[0], u[1], u[2], u[3], u[4], pm, pp);
    } else {
        T d1[5];  // D^1 at (I-2+k)+1/2
#pragma unroll
        for (int k = 0; k < 5; ++k) d1[k] = (v[k + 1] - v[k]) * inv_dx;
        const T h2 = T(0.5) * inv_dx;
        T d2[5];  // D^2 at node I-2+k, k = 1..4
#pragma unroll
        for (int k = 1; k < 5; ++k) d2[k] = (d1[k] - d1[k - 1]) * h2;
        // ENO2: the smaller |D^2| of D^2_I and D^2_{I+1}; ties go left
        const bool left = vabs(d2[2]) <= vabs(d2[3]);
        const T c = left ? d2[2] : d2[3];
        // Q2'(x_i) = c (2(i-k) - 1) dx with k = I: +c dx at I+1, -c dx at I
        pm = d1[2] + c * dx;
        pp = d1[2] - c * dx;
        if constexpr (SCHEME == kSchemeEno3) {
            // k* = I-1 after a left choice, else I; candidates D^3 at k*+1/2
            // and k*+3/2; Q3' multiplier 3m^2 - 6m + 2 with m = i - k*
            const T h3 = inv_dx * T(1.0 / 3.0);
            const T lo = left ? (d2[2] - d2[1]) * h3 : (d2[3] - d2[2]) * h3;
            const T hi = left ? (d2[3] - d2[2]) * h3 : (d2[4] - d2[3]) * h3;
            const T cs = vabs(lo) <= vabs(hi) ? lo : hi;
            const T dx2 = dx * dx;
            pm = pm + cs * (left ? T(2) : T(-1)) * dx2;   // m = 2 or 1 at node I+1
            pp = pp + cs * (left ? T(-1) : T(2)) * dx2;   // m = 1 or 0 at node I
        }
    }
}

// Both derivative approximations at node j from v[0..6] = phi at j-3 .. j+3:
// pm from the interval left of the node, pp from the interval right of it,
// with exactly the arithmetic interval() uses for that half.
template <typename T, int SCHEME>
__device__ __forceinline__ void node_derivs(const T *v, T inv_dx, T dx, T &pm, T &pp)
{
    if constexpr (SCHEME == kSchemeWeno5) {
#pragma clang fp contract(off)
        T u[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) u[k] = (v[k + 1] - v[k]) * inv_dx;
        T q0, q1, q2;
        weno5_q(u[0], u[1], u[2], u[3], u[4], q0, q1, q2);
        pm = weno5_fwd(u[0], u[1], u[2], u[3], u[4], q0, q1, q2);
        weno5_q(u[1], u[2], u[3], u[4], u[5], q0, q1, q2);
        pp = weno5_rev(u[1], u[2], u[3], u[4], u[5], q0, q1, q2);
    } else {
        T unused;
        interval<T, SCHEME>(v, inv_dx, dx, pm, unused);
        interval<T, SCHEME>(v + 1, inv_dx, dx, unused, pp);
    }
}

// ---------------------------------------------------------------- Hamiltonians

template <typename T, int D, int HAM>
__device__ __forceinline__ T ham_value(const StageArgs<T> &a, const int *j, const T *p)
{
#pragma clang fp contract(off)
    if constexpr (HAM == kHamNormal) {  // a |p|
        T s = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) s = fmaT(p[d], p[d], s);
        return a.hp[0] * sqrt(s);
    } else if constexpr (HAM == kHamDubins3) {
        // -[p1(-v_e + v_p cos th) + p2 v_p sin th + wbar_e |p1 y - p2 x - p3| - wbar_p |p3|]
        const T x = a.tab.coord[0][j[0]], y = a.tab.coord[1][j[1]];
        const T c = a.tab.cosv[2][j[2]], sn = a.tab.sinv[2][j[2]];
        const T ve = a.hp[0], vp = a.hp[1], we = a.hp[2], wp = a.hp[3];
        const T drift = fmaT(p[0], fmaT(vp, c, -ve), p[1] * (vp * sn));
        const T arg = fmaT(p[0], y, -fmaT(p[1], x, p[2]));
        return -fmaT(we, vabs(arg), fmaT(-wp, vabs(p[2]), drift));
    } else {
        // -v (p1 cos th + p2 sin th) + wbar |p3| + abar |p4|
        const T c = a.tab.cosv[2][j[2]], sn = a.tab.sinv[2][j[2]];
        const T v = a.tab.coord[3][j[3]];
        return fmaT(-v, fmaT(p[0], c, p[1] * sn), fmaT(a.hp[0], vabs(p[2]), a.hp[1] * vabs(p[3])));
    }
}

// LF Hamiltonian (Sec. IV-D) and the stage combination (Sec. V, Sec. VI):
// L = -(H(x, pbar) - sum_d alpha_d (p+_d - p-_d)/2); the result is L itself
// (rhs_only) or ca phi_n + cb (phi + dt L), then min with the target.
template <typename T, int D, int HAM>
__device__ __forceinline__ T stage_result(const StageArgs<T> &a, const int *j, const T *pm, const T *pp, T center,
                                          int idx)
{
#pragma clang fp contract(off)
    T pbar[D];
#pragma unroll
    for (int d = 0; d < D; ++d) pbar[d] = T(0.5) * (pm[d] + pp[d]);
    T hhat = ham_value<T, D, HAM>(a, j, pbar);
#pragma unroll
    for (int d = 0; d < D; ++d) hhat = fmaT(-a.alpha[d], T(0.5) * (pp[d] - pm[d]), hhat);
    const T L = -hhat;
    if (a.rhs_only) return L;
    T res = a.cb * fmaT(a.dt, L, center);
    if (a.ca != T(0)) res = fmaT(a.ca, ld32(a.phi_n, idx), res);
    if (a.target) {
        const T tg = ld32(a.target, idx);
        res = tg < res ? tg : res;
    }
    return res;
}

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

template <typename T>
__device__ __forceinline__ int wrap_index(int j, int n)
{
    j %= n;
    return j < 0 ? j + n : j;
}

template <typename T, int D, int SCHEME, int HAM>
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
            a.out[idx] = stage_result<T, D, HAM>(a, j, pm, pp, center, idx);
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
template <typename T, int D, int SCHEME, int HAM>
__global__ __launch_bounds__(256) void stage_direct_kernel(StageArgs<T> a)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
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
    for (int sy = blockIdx.y; sy < a.g.slow; sy += gridDim.y) {
        if constexpr (D == 3) j[0] = sy;
        if constexpr (D == 4) {
            j[0] = sy / a.g.n[1];
            j[1] = sy - j[0] * a.g.n[1];
        }
        int idx = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) idx += j[d] * a.g.stride[d];
        T pm[D], pp[D], center = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T v[7];
            gather7(a.phi_in, idx, j[d], a.g.n[d], a.g.stride[d], (a.g.periodic >> d) & 1u, v);
            center = v[3];
            node_derivs<T, SCHEME>(v, a.inv_dx[d], a.dx[d], pm[d], pp[d]);
        }
        *reinterpret_cast<T *>(reinterpret_cast<char *>(a.out) + (unsigned)idx * (unsigned)sizeof(T)) =
            stage_result<T, D, HAM>(a, j, pm, pp, center, idx);
    }
}

template <typename T, int D, int SCHEME, int HAM>
hipError_t launch_one(const StageArgs<T> &a, hipStream_t s)
{
    const Tile t = a.tile;
    const int nf = a.g.n[D - 1], nm = D >= 2 ? a.g.n[D - 2] : 1;
    const int tiles = ((nf + t.tx - 1) / t.tx) * ((nm + t.ty - 1) / t.ty);
    int gy = 1;
    if (D >= 3) gy = (a.g.n[D - 3] + t.march - 1) / t.march;
    if (D == 4) gy *= a.g.n[0];
    if (t.variant == kVariantPlaneMarch &&
        (t.tx < 1 || t.ty < 1 || t.tx * t.ty > 256 || (D == 1 && t.ty != 1) || t.march < 1 || gy > 65535))
        return hipErrorInvalidConfiguration;
    if (t.variant == kVariantDirect) {
        dim3 grid((a.g.plane + 255) / 256, a.g.slow < 65535 ? a.g.slow : 65535);
        hipLaunchKernelGGL((stage_direct_kernel<T, D, SCHEME, HAM>), grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const size_t lds = stage_lds_bytes(t, sizeof(T));
    hipLaunchKernelGGL((stage_kernel<T, D, SCHEME, HAM>), dim3(tiles, gy), dim3(t.tx, t.ty), lds, s, a);
    return hipGetLastError();
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
