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
        const T s0 = fmaT(k1312 * A0, A0, k14 * B0 * B0);
        const T s1 = fmaT(k1312 * A1, A1, k14 * B1 * B1);
        const T s2 = fmaT(k1312 * A2, A2, k14 * B2 * B2);
        int km = 0;
        T m = u[0] * u[0];
#pragma unroll
        for (int k = 1; k < 5; ++k)
            if (u[k] * u[k] > m) {
                m = u[k] * u[k];
                km = k;
            }
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
        const T g0 = fmaT(c13, u[4], fmaT(-c76, u[3], c116 * u[2]));
        const T g1 = fmaT(-c16, u[3], fmaT(c56, u[2], c13 * u[1]));
        const T g2 = fmaT(c13, u[2], fmaT(c56, u[1], -c16 * u[0]));
        const T b0 = T(0.1) * q2, b1 = T(0.6) * q1, b2 = T(0.3) * q0;
        const T iDr = Arith<T>::rcp(b0 + b1 + b2);
        const T rev = fmaT(b0, g0, fmaT(b1, g1, b2 * g2)) * iDr;
        // reverse: weighted means -> substencils and weights.  With the
        // normalised weights W_k = a_k / sum a (each in [0, 1]) the
        // sensitivity of the mean to S_k is -2 W_k (f_k - mean) / (S_k + eps);
        // written this way no intermediate overflows, even at the eps floor
        // (flat data) where q_k = 1/(S_k + eps)^2 alone is near the top of
        // the binary32 range.
        const T wf0 = a0 * iDf, wf1 = a1 * iDf, wf2 = a2 * iDf;
        const T wr0 = b0 * iDr, wr1 = b1 * iDr, wr2 = b2 * iDr;
        const T fb0 = gm * wf0, fb1 = gm * wf1, fb2 = gm * wf2;   // adjoints of f_k
        const T gb0 = gp * wr0, gb1 = gp * wr1, gb2 = gp * wr2;   // adjoints of g_k
        // b_k weights q_{2-k}: S_0 enters rev through wr2, S_2 through wr0
        const T sb0 = T(-2) * r0 * fmaT(fb0, f0 - fwd, gb2 * (g2 - rev));
        const T sb1 = T(-2) * r1 * fmaT(fb1, f1 - fwd, gb1 * (g1 - rev));
        const T sb2 = T(-2) * r2 * fmaT(fb2, f2 - fwd, gb0 * (g0 - rev));
        const T epsb = sb0 + sb1 + sb2;
        // S_k = 13/12 A_k^2 + 1/4 B_k^2
        const T Ab0 = T(2) * k1312 * A0 * sb0, Bb0 = T(2) * k14 * B0 * sb0;
        const T Ab1 = T(2) * k1312 * A1 * sb1, Bb1 = T(2) * k14 * B1 * sb1;
        const T Ab2 = T(2) * k1312 * A2 * sb2, Bb2 = T(2) * k14 * B2 * sb2;
        ub[0] = Ab0 + Bb0;
        ub[1] = fmaT(T(-2), Ab0, fmaT(T(-4), Bb0, Ab1 + Bb1));
        ub[2] = Ab0 + fmaT(T(3), Bb0, fmaT(T(-2), Ab1, Ab2 + T(3) * Bb2));
        ub[3] = (Ab1 - Bb1) + fmaT(T(-2), Ab2, T(-4) * Bb2);
        ub[4] = Ab2 + Bb2;
        // eps = 1e-6 max_k u_k^2 + floor
        ub[km] = fmaT(T(2e-6) * epsb, u[km], ub[km]);
        // substencils
        ub[0] = fmaT(c13, fb0, fmaT(-c16, gb2, ub[0]));
        ub[1] = fmaT(-c76, fb0, fmaT(-c16, fb1, fmaT(c13, gb1, fmaT(c56, gb2, ub[1]))));
        ub[2] = fmaT(c116, fb0, fmaT(c56, fb1, fmaT(c13, fb2, fmaT(c116, gb0, fmaT(c56, gb1, fmaT(c13, gb2, ub[2]))))));
        ub[3] = fmaT(c13, fb1, fmaT(c56, fb2, fmaT(-c76, gb0, fmaT(-c16, gb1, ub[3]))));
        ub[4] = fmaT(-c16, fb2, fmaT(c13, gb0, ub[4]));
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
