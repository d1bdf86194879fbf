// Device arithmetic of the forward stage (also used by the adjoint): reciprocal
// and FMA helpers, ghost-cell gathers, the upwind derivative intervals
// (first order, ENO2, ENO3, WENO5), the built-in Hamiltonians and the
// Lax-Friedrichs stage epilogue.  The adjoint's own helpers are in
// hjx_adjoint_device.h.  Method: LevelSetPy (arXiv 2411.03501),
// Sec. IV-A..IV-D, Sec. V, Sec. VI.
#pragma once

#include "hjx_internal.h"

// No implicit contraction in any kernel that includes this header: every
// fused multiply-add is written out (fmaT), so the rounding of each value is
// fixed by the source and is the same in every kernel, variant, tile and
// template instantiation that computes it.  (The functions below also carry
// the pragma locally, which states the same thing where it matters most.)
#pragma clang fp contract(off)

namespace hjx {
namespace dev {

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

// the larger of |a| and |b| in one instruction (abs is a source modifier)
__device__ __forceinline__ float absmax(float a, float b) { return __builtin_fmaxf(__builtin_fabsf(a), __builtin_fabsf(b)); }
__device__ __forceinline__ double absmax(double a, double b) { return __builtin_fmax(__builtin_fabs(a), __builtin_fabs(b)); }

// ---------------------------------------------------------------- derivatives

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// j modulo n in [0, n), for ghost indices any distance outside the grid
template <typename T>
__device__ __forceinline__ int wrap_index(int j, int n)
{
    j %= n;
    return j < 0 ? j + n : j;
}

// Load base[i] through a 32-bit byte offset from a uniform base pointer, so
// the address is one scalar base plus one vector offset (arrays < 4 GiB; the
// host only launches the direct variant on such arrays).
template <typename T>
__device__ __forceinline__ T ld32(const T *base, int i)
{
    const unsigned off = (unsigned)i * (unsigned)sizeof(T);
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// The same addressing for an element that is written.
template <typename T>
__device__ __forceinline__ T &at32(T *base, int i)
{
    const unsigned off = (unsigned)i * (unsigned)sizeof(T);
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
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

// gather7 along the fastest axis (stride 1).  That axis runs along the lanes
// of a wave, so nodes within three of a row's ends sit in most waves; on a
// periodic axis the wrap is then done with selects for every lane instead of
// the boundary branch that the lanes of a wave would otherwise take in turn.
// The same loads, so the same values as gather7.
// Gather phi at offsets -3 .. N-4 along one axis of node idx, with the ghost
// rules of gather7 (the same value for every position both cover).  With
// N > 7 the node must be at least N - 7 from the axis end (direct_pair's
// first node, j <= n - 2, for N = 8).
template <typename T, int N>
__device__ __forceinline__ void gatherN(const T *__restrict__ phi, int idx, int j, int n, int s, bool per, T (&v)[N])
{
    if (j >= 3 && j + (N - 4) < n) {
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = ld32(phi, idx + (k - 3) * s);
        return;
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int jj = j + k - 3;
        if (per) {  // -3 <= jj - j <= N - 4 and j <= n - 1 - (N - 7), n >= 3: one wrap lands in [0, n)
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

template <typename T>
__device__ __forceinline__ void gather7_row(const T *__restrict__ phi, int idx, int j, int n, bool per, T (&v)[7])
{
    if (per) {
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            const int jj = j + k - 3;
            const int o = (k - 3) + (jj < 0 ? n : 0) - (jj >= n ? n : 0);
            v[k] = ld32(phi, idx + o);
        }
        return;
    }
    gather7(phi, idx, j, n, 1, false, v);
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
    // max_k u_k^2 as (max_k |u_k|)^2: squaring is monotone in |u| and so is
    // its rounding, so the two are the same bits; four one-instruction
    // maxima on |u| replace five squares and four compare-and-selects
    const T am = absmax(absmax(absmax(u0, u1), absmax(u2, u3)), u4);
    const T m = am * am;
    const T eps = fmaT(T(1e-6), m, Arith<T>::kEpsFloor);
    const T r0 = Arith<T>::rcp(s0 + eps), r1 = Arith<T>::rcp(s1 + eps), r2 = Arith<T>::rcp(s2 + eps);
    q0 = r0 * r0;
    q1 = r1 * r1;
    q2 = r2 * r2;
}

// FP64: q_k up to a common factor, without reciprocals.  With t_k = S_k + eps,
// the normalised weights d_k t_k^-2 / sum_j d_j t_j^-2 equal
// d_k P_k / sum_j d_j P_j, P_k being the product of the other two t_j^2;
// weno5_fwd and weno5_rev normalise, so q_k = P_k serves.  The t_k are first
// scaled by the power of two of eps (exact): S_k <= (13/12 16 + 16) max u^2
// < 34 max u^2 and eps >= 1e-6 max u^2 put them in [1/2, 3.4e7), so every P_k
// lies in [1/16, 1.4e30).  Three quarter-rate reciprocals, each refined by
// two Newton steps, become six multiplications.
template <>
__device__ __forceinline__ void weno5_q<double>(double u0, double u1, double u2, double u3, double u4, double &q0,
                                                double &q1, double &q2)
{
#pragma clang fp contract(off)
    const double k1312 = 13.0 / 12.0, k14 = 0.25;
    const double A0 = fmaT(-2.0, u1, u0 + u2), B0 = fmaT(-4.0, u1, fmaT(3.0, u2, u0));
    const double A1 = fmaT(-2.0, u2, u1 + u3), B1 = u1 - u3;
    const double A2 = fmaT(-2.0, u3, u2 + u4), B2 = fmaT(-4.0, u3, fmaT(3.0, u2, u4));
    const double s0 = fmaT(k1312 * A0, A0, k14 * B0 * B0);
    const double s1 = fmaT(k1312 * A1, A1, k14 * B1 * B1);
    const double s2 = fmaT(k1312 * A2, A2, k14 * B2 * B2);
    const double am = absmax(absmax(absmax(u0, u1), absmax(u2, u3)), u4);
    const double eps = fmaT(1e-6, am * am, Arith<double>::kEpsFloor);
    const int e = __builtin_amdgcn_frexp_exp(eps);
    const double t0 = __builtin_amdgcn_ldexp(s0 + eps, -e), t1 = __builtin_amdgcn_ldexp(s1 + eps, -e),
                 t2 = __builtin_amdgcn_ldexp(s2 + eps, -e);
    const double p12 = t1 * t2, p02 = t0 * t2, p01 = t0 * t1;
    q0 = p12 * p12;
    q1 = p02 * p02;
    q2 = p01 * p01;
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

// node_derivs for two neighbouring nodes j and j+1 of one axis, from
// v[0..7] = phi at j-3 .. j+4: the interval between them is evaluated once
// and gives the right-biased value of the first and the left-biased value of
// the second, with exactly the arithmetic node_derivs uses for each.
template <typename T, int SCHEME>
__device__ __forceinline__ void pair_derivs(const T *v, T inv_dx, T dx, T &pm1, T &pp1, T &pm2, T &pp2)
{
    if constexpr (SCHEME == kSchemeWeno5) {
#pragma clang fp contract(off)
        T u[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) u[k] = (v[k + 1] - v[k]) * inv_dx;
        T q0, q1, q2;
        weno5_q(u[0], u[1], u[2], u[3], u[4], q0, q1, q2);
        pm1 = weno5_fwd(u[0], u[1], u[2], u[3], u[4], q0, q1, q2);
        weno5_q(u[1], u[2], u[3], u[4], u[5], q0, q1, q2);
        pp1 = weno5_rev(u[1], u[2], u[3], u[4], u[5], q0, q1, q2);
        pm2 = weno5_fwd(u[1], u[2], u[3], u[4], u[5], q0, q1, q2);
        weno5_q(u[2], u[3], u[4], u[5], u[6], q0, q1, q2);
        pp2 = weno5_rev(u[2], u[3], u[4], u[5], u[6], q0, q1, q2);
    } else {
        T unused;
        interval<T, SCHEME>(v, inv_dx, dx, pm1, unused);
        interval<T, SCHEME>(v + 1, inv_dx, dx, pm2, pp1);
        interval<T, SCHEME>(v + 2, inv_dx, dx, unused, pp2);
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
    } else if constexpr (HAM == kHamRockets) {
        // -[a p1 cos th + p2 (a sin th + a - g) + ubar_e |p1 x - p3| - ubar_p |p2 x + p3|]
        const T x = a.tab.coord[0][j[0]];
        const T c = a.tab.cosv[2][j[2]], sn = a.tab.sinv[2][j[2]];
        const T ac = a.hp[0], g = a.hp[1], ue = a.hp[2], up = a.hp[3];
        const T drift = fmaT(p[0], ac * c, p[1] * (fmaT(ac, sn, ac) - g));
        const T e = fmaT(p[0], x, -p[2]), q = fmaT(p[1], x, p[2]);
        return -fmaT(ue, vabs(e), fmaT(-up, vabs(q), drift));
    } else {
        // -v (p1 cos th + p2 sin th) + wbar |p3| + abar |p4|
        const T c = a.tab.cosv[2][j[2]], sn = a.tab.sinv[2][j[2]];
        const T v = a.tab.coord[3][j[3]];
        return fmaT(-v, fmaT(p[0], c, p[1] * sn), fmaT(a.hp[0], vabs(p[2]), a.hp[1] * vabs(p[3])));
    }
}

// What a stage node does besides its stage value, as bits: keep p-, p+ in
// a.dp_out (the replay of the adjoint), clip the rate by a.clip (a restricted
// update; a.clip may be 0 where one kernel serves clipped and unclipped
// problems), take alpha_d at the node (local Lax-Friedrichs), and mark in
// a.mask where the rate was clipped (the replay of a restricted update; bit 1
// of the mask byte, beside bit 0 for a kept target).  Solves that use none
// of them never compile them.
enum : int { kNodePlain = 0, kNodeKeep = 1, kNodeClip = 2, kNodeLocal = 4, kNodeMark = 8 };

// Bound on |dH/dp_d| over the controls at node j (the local dissipation
// coefficient; its grid maximum is the global alpha_d).
template <typename T, int D, int HAM>
__device__ __forceinline__ T node_bound(const StageArgs<T> &a, const int *j, int d)
{
    if constexpr (HAM == kHamNormal || HAM == kHamNormalGodunov) {
        return vabs(a.hp[0]);
    } else if constexpr (HAM == kHamDubins3) {
        const T ve = a.hp[0], vp = a.hp[1], we = a.hp[2], wp = a.hp[3];
        if (d == 0) return vabs(-ve + vp * a.tab.cosv[2][j[2]]) + we * vabs(a.tab.coord[1][j[1]]);
        if (d == 1) return vabs(vp * a.tab.sinv[2][j[2]]) + we * vabs(a.tab.coord[0][j[0]]);
        return we + wp;
    } else if constexpr (HAM == kHamRockets) {
        const T ac = a.hp[0], g = a.hp[1], ue = a.hp[2], up = a.hp[3];
        const T ax = vabs(a.tab.coord[0][j[0]]);
        if (d == 0) return vabs(ac * a.tab.cosv[2][j[2]]) + ue * ax;
        if (d == 1) return vabs(ac * a.tab.sinv[2][j[2]] + ac - g) + up * ax;
        return ue + up;
    } else {
        const T v = a.tab.coord[3][j[3]];
        if (d == 0) return vabs(v * a.tab.cosv[2][j[2]]);
        if (d == 1) return vabs(v * a.tab.sinv[2][j[2]]);
        return d == 2 ? a.hp[0] : a.hp[1];
    }
}

// LF Hamiltonian (Sec. IV-D) and the stage combination (Sec. V, Sec. VI):
// L = -(H(x, pbar) - sum_d alpha_d (p+_d - p-_d)/2); the result is L itself
// (rhs_only) or ca phi_n + cb (phi + dt L), then min with the target.  With
// kNodeClip in MODE, a restricted update (Sec. VI): L is first clipped to
// min(L, 0) (a.clip < 0) or max(L, 0) (a.clip > 0).  With kNodeLocal, alpha_d
// is node_bound at the node instead of the grid maximum a.alpha[d].
// phi_n, target and mask are read (written) at idx: those of `a`, or the same
// arrays rebased to where idx counts from (stage_result_at).
//
// stage_rate: L alone (clipped under kNodeClip unless a.rhs_only).
template <typename T, int D, int HAM, int MODE = kNodePlain>
__device__ __forceinline__ T stage_rate(const StageArgs<T> &a, const int *j, const T *pm, const T *pp)
{
#pragma clang fp contract(off)
    T pbar[D];
#pragma unroll
    for (int d = 0; d < D; ++d) pbar[d] = T(0.5) * (pm[d] + pp[d]);
    T hhat;
    if constexpr (HAM == kHamNormalGodunov) {
        // Godunov for a|p|: per axis the extremum of |p| over the interval
        // between p- and p+ (the minimum for a >= 0, the maximum for a < 0)
        T s = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T q;
            if (a.hp[0] >= T(0)) {
                const T up = pm[d] > T(0) ? pm[d] : T(0), dn = pp[d] < T(0) ? -pp[d] : T(0);
                q = dn > up ? dn : up;
            } else {
                const T dn = pm[d] < T(0) ? -pm[d] : T(0), up = pp[d] > T(0) ? pp[d] : T(0);
                q = up > dn ? up : dn;
            }
            s = fmaT(q, q, s);
        }
        hhat = a.hp[0] * sqrt(s);
    } else {
        hhat = ham_value<T, D, HAM>(a, j, pbar);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T al = a.alpha[d];
            if constexpr ((MODE & kNodeLocal) != 0) al = node_bound<T, D, HAM>(a, j, d);
            hhat = fmaT(-al, T(0.5) * (pp[d] - pm[d]), hhat);
        }
    }
    T L = -hhat;
    if (a.rhs_only) return L;
    if constexpr ((MODE & kNodeClip) != 0) {
        if (a.clip < 0) L = L > T(0) ? T(0) : L;
        if (a.clip > 0) L = L < T(0) ? T(0) : L;
    }
    return L;
}

template <typename T, int D, int HAM, int MODE = kNodePlain>
__device__ __forceinline__ T stage_result_at(const StageArgs<T> &a, const T *phi_n, const T *target,
                                             unsigned char *mask, const int *j, const T *pm, const T *pp, T center,
                                             int idx)
{
#pragma clang fp contract(off)
    if constexpr ((MODE & kNodeMark) != 0) {
        // the replay of a restricted update: the same value as under
        // kNodeClip, with the clip and the target recorded in the mask byte
        T L = stage_rate<T, D, HAM, MODE & ~kNodeClip>(a, j, pm, pp);
        if (a.rhs_only) return L;
        const bool clipped = (a.clip < 0 && L > T(0)) || (a.clip > 0 && L < T(0));
        if (clipped) L = T(0);
        T res = a.cb * fmaT(a.dt, L, center);
        if (a.ca != T(0)) res = fmaT(a.ca, ld32(phi_n, idx), res);
        bool kept = false;
        if (target) {
            const T tg = ld32(target, idx);
            kept = tg < res;
            res = kept ? tg : res;
        }
        if (mask) mask[idx] = (unsigned char)((kept ? 1 : 0) | (clipped ? 2 : 0));
        return res;
    } else {
        const T L = stage_rate<T, D, HAM, MODE>(a, j, pm, pp);
        if (a.rhs_only) return L;
        T res = a.cb * fmaT(a.dt, L, center);
        if (a.ca != T(0)) res = fmaT(a.ca, ld32(phi_n, idx), res);
        if (target) {
            const T tg = ld32(target, idx);
            if (mask) mask[idx] = tg < res;
            res = tg < res ? tg : res;
        }
        return res;
    }
}

template <typename T, int D, int HAM, int MODE = kNodePlain>
__device__ __forceinline__ T stage_result(const StageArgs<T> &a, const int *j, const T *pm, const T *pp, T center,
                                          int idx)
{
    return stage_result_at<T, D, HAM, MODE>(a, a.phi_n, a.target, a.mask, j, pm, pp, center, idx);
}

// One node of the direct variant: gather every axis through the caches,
// both derivative halves at the node, LF Hamiltonian, stage combination.
// MODE: the node-mode bits (above).
template <typename T, int D, int SCHEME, int HAM, int MODE = kNodePlain>
__device__ __forceinline__ void direct_node(const StageArgs<T> &a, const int *j)
{
    int idx = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) idx += j[d] * a.g.stride[d];
    T pm[D], pp[D], center = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        T v[7];
        if (d == D - 1) gather7_row(a.phi_in, idx, j[d], a.g.n[d], (a.g.periodic >> d) & 1u, v);
        else gather7(a.phi_in, idx, j[d], a.g.n[d], a.g.stride[d], (a.g.periodic >> d) & 1u, v);
        center = v[3];
        node_derivs<T, SCHEME>(v, a.inv_dx[d], a.dx[d], pm[d], pp[d]);
    }
    if constexpr ((MODE & kNodeKeep) != 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            at32(a.dp_out + (size_t)(2 * d) * (size_t)a.dp_stride, idx) = pm[d];
            at32(a.dp_out + (size_t)(2 * d + 1) * (size_t)a.dp_stride, idx) = pp[d];
        }
    }
    *reinterpret_cast<T *>(reinterpret_cast<char *>(a.out) + (unsigned)idx * (unsigned)sizeof(T)) =
        stage_result<T, D, HAM, MODE>(a, j, pm, pp, center, idx);
}

// The rest of one node of the direct variant once its axis-0 derivatives
// (pm0, pp0) and its own value are known: axes 1 .. D-1, the LF Hamiltonian,
// the stage combination, the store.
template <typename T, int D, int SCHEME, int HAM, int MODE>
__device__ __forceinline__ void direct_rest(const StageArgs<T> &a, const int *j, int idx, T pm0, T pp0, T center)
{
    T pm[D], pp[D];
    pm[0] = pm0;
    pp[0] = pp0;
#pragma unroll
    for (int d = 1; d < D; ++d) {
        T v[7];
        if (d == D - 1) gather7_row(a.phi_in, idx, j[d], a.g.n[d], (a.g.periodic >> d) & 1u, v);
        else gather7(a.phi_in, idx, j[d], a.g.n[d], a.g.stride[d], (a.g.periodic >> d) & 1u, v);
        node_derivs<T, SCHEME>(v, a.inv_dx[d], a.dx[d], pm[d], pp[d]);
    }
    if constexpr ((MODE & kNodeKeep) != 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            at32(a.dp_out + (size_t)(2 * d) * (size_t)a.dp_stride, idx) = pm[d];
            at32(a.dp_out + (size_t)(2 * d + 1) * (size_t)a.dp_stride, idx) = pp[d];
        }
    }
    *reinterpret_cast<T *>(reinterpret_cast<char *>(a.out) + (unsigned)idx * (unsigned)sizeof(T)) =
        stage_result<T, D, HAM, MODE>(a, j, pm, pp, center, idx);
}

// Two nodes of the direct variant: j and its neighbour one step along axis 0
// (j[0] + 1 < n[0]).  Along axis 0 they share one 8-point gather and the
// interval between them; then each node finishes on its own, the first
// before the second.  Each node gets the bits direct_node would give it.
template <typename T, int D, int SCHEME, int HAM, int MODE = kNodePlain>
__device__ __forceinline__ void direct_pair(const StageArgs<T> &a, const int *j)
{
    static_assert(D >= 2, "pairs run along axis 0 of a grid of two or more axes");
    int idx = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) idx += j[d] * a.g.stride[d];
    T pm1, pp1, pm2, pp2, c1, c2;
    {
        T v[8];
        gatherN<T, 8>(a.phi_in, idx, j[0], a.g.n[0], a.g.stride[0], a.g.periodic & 1u, v);
        c1 = v[3];
        c2 = v[4];
        pair_derivs<T, SCHEME>(v, a.inv_dx[0], a.dx[0], pm1, pp1, pm2, pp2);
    }
    asm volatile("" ::: "memory");
    direct_rest<T, D, SCHEME, HAM, MODE>(a, j, idx, pm1, pp1, c1);
    // the second node's memory work after the first node's store
    asm volatile("" ::: "memory");
    const int j2[kMaxDim] = {j[0] + 1, j[1], D > 2 ? j[2] : 0, D > 3 ? j[3] : 0};
    direct_rest<T, D, SCHEME, HAM, MODE>(a, j2, idx + a.g.stride[0], pm2, pp2, c2);
}

}  // namespace dev
}  // namespace hjx
