// Device helpers of the reverse sweep only: the gradient of the built-in
// Hamiltonians and the transpose of one derivative interval.  Method:
// LevelSetPy (arXiv 2411.03501), Sec. IV-A..IV-D; the adjoint itself has no
// counterpart in the paper.
#pragma once

#include "hjx_device.h"

namespace hjx {
namespace dev {

template <typename T>
__device__ __forceinline__ T vsign(T a) { return a > T(0) ? T(1) : (a < T(0) ? T(-1) : T(0)); }

// The per-node table values a Hamiltonian reads (coordinates, cosine and
// sine of the angle axis), loaded apart from its arithmetic.
template <typename T>
struct HamTab {
    T x, y, c, s, v;
};

template <typename T, int D, int HAM>
__device__ __forceinline__ HamTab<T> ham_tab(const StageArgs<T> &a, const int *j)
{
    HamTab<T> t{T(0), T(0), T(0), T(0), T(0)};
    if constexpr (HAM == kHamDubins3) {
        t.x = a.tab.coord[0][j[0]];
        t.y = a.tab.coord[1][j[1]];
        t.c = a.tab.cosv[2][j[2]];
        t.s = a.tab.sinv[2][j[2]];
    } else if constexpr (HAM == kHamRockets) {
        t.x = a.tab.coord[0][j[0]];
        t.c = a.tab.cosv[2][j[2]];
        t.s = a.tab.sinv[2][j[2]];
    } else if constexpr (HAM == kHamDubins4) {
        t.c = a.tab.cosv[2][j[2]];
        t.s = a.tab.sinv[2][j[2]];
        t.v = a.tab.coord[3][j[3]];
    }
    return t;
}

// H at p with its gradient in p (dHdp[d]) and the gradient of -H in the
// Hamiltonian parameters (dmH[m]); |.| has derivative sign(.) with
// sign(0) = 0.  tb: the node's table values (ham_tab).
template <typename T, int D, int HAM>
__device__ __forceinline__ T ham_grad(const StageArgs<T> &a, const HamTab<T> &tb, const T *p, T *dHdp, T *dmH)
{
#pragma clang fp contract(off)
    if constexpr (HAM == kHamNormal) {  // H = a |p|
        T s = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) s = fmaT(p[d], p[d], s);
        const T n = sqrt(s);
        const T inv = n > T(0) ? T(1) / n : T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) dHdp[d] = a.hp[0] * p[d] * inv;
        dmH[0] = -n;
        return a.hp[0] * n;
    } else if constexpr (HAM == kHamDubins3) {
        const T x = tb.x, y = tb.y;
        const T c = tb.c, sn = tb.s;
        const T ve = a.hp[0], vp = a.hp[1], we = a.hp[2], wp = a.hp[3];
        const T drift = fmaT(p[0], fmaT(vp, c, -ve), p[1] * (vp * sn));
        const T arg = fmaT(p[0], y, -fmaT(p[1], x, p[2]));
        const T sa = vsign(arg), s3 = vsign(p[2]);
        dHdp[0] = -fmaT(we * sa, y, fmaT(vp, c, -ve));
        dHdp[1] = -fmaT(-we * sa, x, vp * sn);
        dHdp[2] = fmaT(we, sa, wp * s3);
        dmH[0] = -p[0];                        // d(-H)/dv_e
        dmH[1] = fmaT(p[0], c, p[1] * sn);     // d(-H)/dv_p
        dmH[2] = vabs(arg);                    // d(-H)/dwbar_e
        dmH[3] = -vabs(p[2]);                  // d(-H)/dwbar_p
        return -fmaT(we, vabs(arg), fmaT(-wp, vabs(p[2]), drift));
    } else if constexpr (HAM == kHamRockets) {
        // H = -[a p1 cos th + p2 (a sin th + a - g) + ubar_e |p1 x - p3| - ubar_p |p2 x + p3|]
        const T x = tb.x, c = tb.c, sn = tb.s;
        const T ac = a.hp[0], g = a.hp[1], ue = a.hp[2], up = a.hp[3];
        const T k1 = fmaT(ac, sn, ac) - g;  // the p2 drift
        const T e = fmaT(p[0], x, -p[2]), q = fmaT(p[1], x, p[2]);
        const T se = vsign(e), sq = vsign(q);
        dHdp[0] = -fmaT(ue * se, x, ac * c);
        dHdp[1] = -fmaT(-up * sq, x, k1);
        dHdp[2] = fmaT(ue, se, up * sq);
        dmH[0] = fmaT(p[0], c, p[1] * (sn + T(1)));  // d(-H)/da
        dmH[1] = -p[1];                               // d(-H)/dg
        dmH[2] = vabs(e);                             // d(-H)/dubar_e
        dmH[3] = -vabs(q);                            // d(-H)/dubar_p
        return -fmaT(ue, vabs(e), fmaT(-up, vabs(q), fmaT(p[0], ac * c, p[1] * k1)));
    } else {
        const T c = tb.c, sn = tb.s;
        const T v = tb.v;
        dHdp[0] = -v * c;
        dHdp[1] = -v * sn;
        dHdp[2] = a.hp[0] * vsign(p[2]);
        dHdp[3] = a.hp[1] * vsign(p[3]);
        dmH[0] = -vabs(p[2]);                  // d(-H)/dwbar
        dmH[1] = -vabs(p[3]);                  // d(-H)/dabar
        return fmaT(-v, fmaT(p[0], c, p[1] * sn), fmaT(a.hp[0], vabs(p[2]), a.hp[1] * vabs(p[3])));
    }
}

// alpha_d at the node (the local dissipation coefficient, node_bound) and
// its gradient in the Hamiltonian parameters (dbnd[m]), from the node's
// table values; d|s|/ds = sign(s) as in ham_grad.
template <typename T, int D, int HAM>
__device__ __forceinline__ T bound_grad(const StageArgs<T> &a, const HamTab<T> &tb, int d, T (&dbnd)[8])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int m = 0; m < 8; ++m) dbnd[m] = T(0);
    if constexpr (HAM == kHamNormal) {  // |a|
        dbnd[0] = vsign(a.hp[0]);
        return vabs(a.hp[0]);
    } else if constexpr (HAM == kHamDubins3) {
        // |-v_e + v_p cos th| + wbar_e |y|,  |v_p sin th| + wbar_e |x|,  wbar_e + wbar_p
        const T ve = a.hp[0], vp = a.hp[1], we = a.hp[2], wp = a.hp[3];
        if (d == 0) {
            const T u = -ve + vp * tb.c, su = vsign(u);
            dbnd[0] = -su;
            dbnd[1] = su * tb.c;
            dbnd[2] = vabs(tb.y);
            return vabs(u) + we * vabs(tb.y);
        }
        if (d == 1) {
            const T u = vp * tb.s;
            dbnd[1] = vsign(u) * tb.s;
            dbnd[2] = vabs(tb.x);
            return vabs(u) + we * vabs(tb.x);
        }
        dbnd[2] = T(1);
        dbnd[3] = T(1);
        return we + wp;
    } else if constexpr (HAM == kHamRockets) {
        // |a cos th| + ubar_e |x|,  |a sin th + a - g| + ubar_p |x|,  ubar_e + ubar_p
        const T ac = a.hp[0], g = a.hp[1], ue = a.hp[2], up = a.hp[3];
        const T ax = vabs(tb.x);
        if (d == 0) {
            const T u = ac * tb.c;
            dbnd[0] = vsign(u) * tb.c;
            dbnd[2] = ax;
            return vabs(u) + ue * ax;
        }
        if (d == 1) {
            const T u = ac * tb.s + ac - g, su = vsign(u);
            dbnd[0] = su * (tb.s + T(1));
            dbnd[1] = -su;
            dbnd[3] = ax;
            return vabs(u) + up * ax;
        }
        dbnd[2] = T(1);
        dbnd[3] = T(1);
        return ue + up;
    } else {  // |v cos th|, |v sin th|, wbar, abar
        if (d == 0) return vabs(tb.v * tb.c);
        if (d == 1) return vabs(tb.v * tb.s);
        dbnd[d - 2] = T(1);
        return a.hp[d - 2];
    }
}

// Reverse of interval(): v[0..5] = phi at I-2 .. I+3; gm, gp = adjoints of
// pm (node I+1) and pp (node I).  ub[r] receives the adjoint of the r-th
// one-sided difference D+ phi_{I-2+r} (r = 0..4); the stencil choices of
// ENO are those of the forward evaluation (same arithmetic).
template <typename T, int SCHEME>
__device__ __forceinline__ void interval_vjp(const T *v, T inv_dx, T dx, T gm, T gp, T (&ub)[5])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < 5; ++r) ub[r] = T(0);
    if constexpr (SCHEME == kSchemeFirst) {
        ub[2] = gm + gp;
    } else if constexpr (SCHEME == kSchemeWeno5) {
        T u[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) u[k] = (v[k + 1] - v[k]) * inv_dx;
        // forward, keeping what the reverse needs
        const T k1312 = T(13.0 / 12.0), k14 = T(0.25);
        const T A0 = fmaT(T(-2), u[1], u[0] + u[2]), B0 = fmaT(T(-4), u[1], fmaT(T(3), u[2], u[0]));
        const T A1 = fmaT(T(-2), u[2], u[1] + u[3]), B1 = u[1] - u[3];
        const T A2 = fmaT(T(-2), u[3], u[2] + u[4]), B2 = fmaT(T(-4), u[3], fmaT(T(3), u[2], u[4]));
        // S_k = cA_k A_k + cB_k B_k with cA_k = 13/12 A_k, cB_k = B_k / 4
        const T cA0 = k1312 * A0, cA1 = k1312 * A1, cA2 = k1312 * A2;
        const T cB0 = k14 * B0, cB1 = k14 * B1, cB2 = k14 * B2;
        const T s0 = fmaT(cA0, A0, cB0 * B0);
        const T s1 = fmaT(cA1, A1, cB1 * B1);
        const T s2 = fmaT(cA2, A2, cB2 * B2);
        // eps = 1e-6 max_k u_k^2 + floor; the lane masks c_k say where u_k^2
        // exceeds every earlier square, so the first maximising k is the
        // last k whose mask is set
        T sq[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) sq[k] = u[k] * u[k];
        const bool c1 = sq[1] > sq[0];
        T m = c1 ? sq[1] : sq[0];
        const bool c2 = sq[2] > m;
        m = c2 ? sq[2] : m;
        const bool c3 = sq[3] > m;
        m = c3 ? sq[3] : m;
        const bool c4 = sq[4] > m;
        m = c4 ? sq[4] : m;
        const bool is[5] = {!(c1 || c2 || c3 || c4), c1 && !(c2 || c3 || c4), c2 && !(c3 || c4), c3 && !c4, c4};
        const T eps = fmaT(T(1e-6), m, Arith<T>::kEpsFloor);
        const T r0 = Arith<T>::rcp(s0 + eps), r1 = Arith<T>::rcp(s1 + eps), r2 = Arith<T>::rcp(s2 + eps);
        const T q0 = r0 * r0, q1 = r1 * r1, q2 = r2 * r2;
        const T c13 = T(1.0 / 3.0), c16 = T(1.0 / 6.0), c56 = T(5.0 / 6.0), c76 = T(7.0 / 6.0),
                c116 = T(11.0 / 6.0);
        const T f0 = fmaT(c13, u[0], fmaT(-c76, u[1], c116 * u[2]));
        const T f1 = fmaT(-c16, u[1], fmaT(c56, u[2], c13 * u[3]));
        const T f2 = fmaT(c13, u[2], fmaT(c56, u[3], -c16 * u[4]));
        const T a0 = T(0.1) * q0, a1 = T(0.6) * q1, a2 = T(0.3) * q2;
        const T iDf = Arith<T>::rcp(a0 + a1 + a2);
        const T fwd = fmaT(a0, f0, fmaT(a1, f1, a2 * f2)) * iDf;
        // the mirrored substencils differ from the forward ones by half a
        // B: g2 = f0 - B0/2, g1 = f1 + B1/2, g0 = f2 + B2/2
        const T g0 = fmaT(T(0.5), B2, f2), g1 = fmaT(T(0.5), B1, f1), g2 = fmaT(T(-0.5), B0, f0);
        const T b0 = T(0.1) * q2, b2 = T(0.3) * q0;   // and b1 = a1
        const T iDr = Arith<T>::rcp(b0 + a1 + b2);
        const T rev = fmaT(b0, g0, fmaT(a1, g1, b2 * g2)) * iDr;
        // reverse: weighted means -> substencils and weights.  With the
        // normalised weights W_k = a_k / sum a (each in [0, 1]) the
        // sensitivity of the mean to S_k is -2 W_k (f_k - mean) / (S_k + eps);
        // written this way no intermediate overflows, even at the eps floor
        // (flat data) where q_k = 1/(S_k + eps)^2 alone is near the top of
        // the binary32 range.  The seeds enter scaled by -4 (exact), so that
        // t_k below is twice the adjoint of S_k and the factors 2 of the
        // squares in S_k cancel.
        const T wf0 = a0 * iDf, wf1 = a1 * iDf, wf2 = a2 * iDf;
        const T wr0 = b0 * iDr, wr1 = a1 * iDr, wr2 = b2 * iDr;
        const T gmq = T(-4) * gm, gpq = T(-4) * gp;
        const T F0 = gmq * wf0, F1 = gmq * wf1, F2 = gmq * wf2;   // -4 x the adjoints of f_k
        const T G0 = gpq * wr0, G1 = gpq * wr1, G2 = gpq * wr2;   // -4 x the adjoints of g_k
        // b_k weights q_{2-k}: S_0 enters rev through wr2, S_2 through wr0
        const T t0 = r0 * fmaT(F0, f0 - fwd, G2 * (g2 - rev));
        const T t1 = r1 * fmaT(F1, f1 - fwd, G1 * (g1 - rev));
        const T t2 = r2 * fmaT(F2, f2 - fwd, G0 * (g0 - rev));
        // adjoints of A_k and B_k; B_k also reaches the mirrored substencils
        const T Ab0 = cA0 * t0, Ab1 = cA1 * t1, Ab2 = cA2 * t2;
        const T Bb0 = fmaT(T(0.125), G2, cB0 * t0);
        const T Bb1 = fmaT(T(-0.125), G1, cB1 * t1);
        const T Bb2 = fmaT(T(-0.125), G0, cB2 * t2);
        // eps = 1e-6 u_km^2 + floor: d/du_km = 2e-6 u_km times the sum of the
        // adjoints of S_k, which is (t0 + t1 + t2) / 2
        const T e = T(1e-6) * ((t0 + t1) + t2);
        // the substencils, through f_k and the f_k inside g_{2-k}; their
        // constants carry the -1/4 that undoes the scale of F and G
        const T Ft0 = F0 + G2, Ft1 = F1 + G1, Ft2 = F2 + G0;
        const T q4 = T(-0.25);
        ub[0] = Ab0 + Bb0;
        ub[1] = fmaT(T(-2), Ab0, fmaT(T(-4), Bb0, Ab1 + Bb1));
        ub[2] = Ab0 + fmaT(T(3), Bb0, fmaT(T(-2), Ab1, Ab2 + T(3) * Bb2));
        ub[3] = (Ab1 - Bb1) + fmaT(T(-2), Ab2, T(-4) * Bb2);
        ub[4] = Ab2 + Bb2;
        ub[0] = fmaT(q4 * c13, Ft0, ub[0]);
        ub[1] = fmaT(q4 * -c76, Ft0, fmaT(q4 * -c16, Ft1, ub[1]));
        ub[2] = fmaT(q4 * c116, Ft0, fmaT(q4 * c56, Ft1, fmaT(q4 * c13, Ft2, ub[2])));
        ub[3] = fmaT(q4 * c13, Ft1, fmaT(q4 * c56, Ft2, ub[3]));
        ub[4] = fmaT(q4 * -c16, Ft2, ub[4]);
#pragma unroll
        for (int k = 0; k < 5; ++k) ub[k] = fmaT(is[k] ? e : T(0), u[k], ub[k]);
        // u_k = (v[k+1] - v[k]) inv_dx is applied by the caller per half-node
    } else {
        T d1[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) d1[k] = (v[k + 1] - v[k]) * inv_dx;
        const T h2 = T(0.5) * inv_dx;
        T d2[5];
#pragma unroll
        for (int k = 1; k < 5; ++k) d2[k] = (d1[k] - d1[k - 1]) * h2;
        const bool left = vabs(d2[2]) <= vabs(d2[3]);
        T d2b[5] = {T(0), T(0), T(0), T(0), T(0)};
        ub[2] = gm + gp;                     // D^1_{I+1/2}
        const T cb_ = (gm - gp) * dx;        // c
        d2b[left ? 2 : 3] += cb_;
        if constexpr (SCHEME == kSchemeEno3) {
            const T h3 = inv_dx * T(1.0 / 3.0);
            const int ia = left ? 1 : 2;     // lo = (d2[ia+1] - d2[ia]) h3, hi = (d2[ia+2] - d2[ia+1]) h3
            const T lo = (d2[ia + 1] - d2[ia]) * h3, hi = (d2[ia + 2] - d2[ia + 1]) * h3;
            const bool take_lo = vabs(lo) <= vabs(hi);
            const T dx2 = dx * dx;
            const T csb = (gm * (left ? T(2) : T(-1)) + gp * (left ? T(-1) : T(2))) * dx2;
            const int ib = take_lo ? ia : ia + 1;
            d2b[ib + 1] += csb * h3;
            d2b[ib] -= csb * h3;
        }
#pragma unroll
        for (int k = 1; k < 5; ++k) {
            ub[k] += d2b[k] * h2;
            ub[k - 1] -= d2b[k] * h2;
        }
    }
}

}  // namespace dev
}  // namespace hjx
