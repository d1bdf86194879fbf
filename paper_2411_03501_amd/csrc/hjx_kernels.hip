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
// Layout: row-major, last axis fastest.  One thread per node; the thread
// grid covers the plane of the last two axes (x) times the remaining slow
// axes (y), so the fastest axis runs along the wave's lanes and every load
// of a row is coalesced.
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
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static constexpr double kEpsFloor = 1e-99;
};

template <typename T>
__device__ __forceinline__ T sq(T x) { return x * x; }

template <typename T>
__device__ __forceinline__ T vmax(T a, T b) { return a > b ? a : b; }

template <typename T>
__device__ __forceinline__ T vabs(T a) { return a < T(0) ? -a : a; }

// ---------------------------------------------------------------- derivatives

template <int SCHEME>
struct Radius;
template <> struct Radius<kSchemeFirst> { static constexpr int r = 1; };
template <> struct Radius<kSchemeEno2> { static constexpr int r = 2; };
template <> struct Radius<kSchemeEno3> { static constexpr int r = 3; };
template <> struct Radius<kSchemeWeno5> { static constexpr int r = 3; };

// WENO5 (Sec. IV-C) from five one-sided differences ordered towards the
// node: the three third-order substencils, their smoothness indicators,
// eps = 1e-6 max v^2 + floor, weights d_k / (S_k + eps)^2 with
// d = (0.1, 0.6, 0.3).
template <typename T>
__device__ __forceinline__ T weno5(T v1, T v2, T v3, T v4, T v5)
{
    const T c13 = T(1.0 / 3.0), c16 = T(1.0 / 6.0), c56 = T(5.0 / 6.0);
    const T f0 = c13 * v1 - T(7.0 / 6.0) * v2 + T(11.0 / 6.0) * v3;
    const T f1 = -c16 * v2 + c56 * v3 + c13 * v4;
    const T f2 = c13 * v3 + c56 * v4 - c16 * v5;

    const T k1312 = T(13.0 / 12.0), k14 = T(0.25);
    const T s0 = k1312 * sq(v1 - T(2) * v2 + v3) + k14 * sq(v1 - T(4) * v2 + T(3) * v3);
    const T s1 = k1312 * sq(v2 - T(2) * v3 + v4) + k14 * sq(v2 - v4);
    const T s2 = k1312 * sq(v3 - T(2) * v4 + v5) + k14 * sq(T(3) * v3 - T(4) * v4 + v5);

    const T m = vmax(vmax(vmax(sq(v1), sq(v2)), vmax(sq(v3), sq(v4))), sq(v5));
    const T eps = T(1e-6) * m + Arith<T>::kEpsFloor;

    const T a0 = T(0.1) * Arith<T>::rcp(sq(s0 + eps));
    const T a1 = T(0.6) * Arith<T>::rcp(sq(s1 + eps));
    const T a2 = T(0.3) * Arith<T>::rcp(sq(s2 + eps));
    return Arith<T>::div(a0 * f0 + a1 * f1 + a2 * f2, a0 + a1 + a2);
}

// v[0..2R] = phi at offsets -R..R along one axis (ghosts filled).
// The divided differences of the ENO table are evaluated without
// contraction so that a smaller-|D| choice on exactly representable data
// sees the same numbers as a plain IEEE evaluation.
template <typename T, int SCHEME>
__device__ __forceinline__ void derivatives(const T *v, T inv_dx, T dx, T &pm, T &pp)
{
    constexpr int R = Radius<SCHEME>::r;
    if constexpr (SCHEME == kSchemeFirst) {
        pm = (v[R] - v[R - 1]) * inv_dx;
        pp = (v[R + 1] - v[R]) * inv_dx;
    } else if constexpr (SCHEME == kSchemeWeno5) {
        T d1[6];  // d1[k] = D+ phi at node i-3+k
#pragma unroll
        for (int k = 0; k < 6; ++k) d1[k] = (v[k + 1] - v[k]) * inv_dx;
        pm = weno5(d1[0], d1[1], d1[2], d1[3], d1[4]);
        pp = weno5(d1[5], d1[4], d1[3], d1[2], d1[1]);
    } else {
#pragma clang fp contract(off)
        // ENO2 / ENO3 (Sec. IV-B).  With o = R - 2 the table is indexed so that
        // d1[k] = D^1 at node (i-2+k)+1/2, d2[k] = D^2 at node i-2+k,
        // d3[k] = D^3 at node (i-2+k)+1/2 for R = 2; ENO3 shifts by one.
        constexpr int W = 2 * R;  // differences available
        T d1[W];
#pragma unroll
        for (int k = 0; k < W; ++k) d1[k] = (v[k + 1] - v[k]) * inv_dx;
        const T h2 = T(0.5) * inv_dx;
        T d2[W];  // d2[k] = D^2 at node i-R+k, valid for k = 1..W-1
#pragma unroll
        for (int k = 1; k < W; ++k) d2[k] = (d1[k] - d1[k - 1]) * h2;
        // left-biased: k = i-1 (interval index R-1 in d1), right: k = i (index R)
        const int km = R - 1, kp = R;
        // ENO2 choice for the left-biased value
        T cm, cp;
        bool left_m, left_p;
        left_m = vabs(d2[km]) <= vabs(d2[km + 1]);
        cm = left_m ? d2[km] : d2[km + 1];
        left_p = vabs(d2[kp]) <= vabs(d2[kp + 1]);
        cp = left_p ? d2[kp] : d2[kp + 1];
        // Q2'(x_i) = c (2(i-k) - 1) dx: +c dx on the left, -c dx on the right
        pm = d1[km] + cm * dx;
        pp = d1[kp] - cp * dx;
        if constexpr (SCHEME == kSchemeEno3) {
            const T h3 = inv_dx * T(1.0 / 3.0);
            T d3[W];  // d3[k] = D^3 at (i-R+k)+1/2, valid for k = 1..W-2
#pragma unroll
            for (int k = 1; k < W - 1; ++k) d3[k] = (d2[k + 1] - d2[k]) * h3;
            // k* = k-1 when the left point was taken, else k; the candidates
            // are D^3 at k*+1/2 and k*+3/2; multiplier 3m^2 - 6m + 2, m = i-k*
            const int ksm = left_m ? km - 1 : km;
            const int ksp = left_p ? kp - 1 : kp;
            const T am = vabs(d3[ksm]) <= vabs(d3[ksm + 1]) ? d3[ksm] : d3[ksm + 1];
            const T ap = vabs(d3[ksp]) <= vabs(d3[ksp + 1]) ? d3[ksp] : d3[ksp + 1];
            const int mm = R - ksm, mp = R - ksp;
            const T dx2 = dx * dx;
            pm = pm + am * T(3 * mm * mm - 6 * mm + 2) * dx2;
            pp = pp + ap * T(3 * mp * mp - 6 * mp + 2) * dx2;
        }
    }
}

// Gather phi at offsets -R..R along one axis of node idx (coordinate j of n,
// stride s), filling ghosts: periodic wrap, else linear extrapolation from
// the two end nodes.
template <typename T, int R>
__device__ __forceinline__ void gather(const T *__restrict__ phi, int idx, int j, int n, int s, bool per,
                                       T (&v)[2 * R + 1])
{
    if (j >= R && j < n - R) {
#pragma unroll
        for (int k = 0; k < 2 * R + 1; ++k) v[k] = phi[idx + (k - R) * s];
        return;
    }
#pragma unroll
    for (int k = 0; k < 2 * R + 1; ++k) {
        int jj = j + k - R;
        if (per) {
            jj = jj < 0 ? jj + n : (jj >= n ? jj - n : jj);
            v[k] = phi[idx + (jj - j) * s];
        } else if (jj < 0) {
            const T a = phi[idx - j * s], b = phi[idx + (1 - j) * s];
            v[k] = a + T(-jj) * (a - b);
        } else if (jj >= n) {
            const T a = phi[idx + (n - 1 - j) * s], b = phi[idx + (n - 2 - j) * s];
            v[k] = a + T(jj - n + 1) * (a - b);
        } else {
            v[k] = phi[idx + (k - R) * s];
        }
    }
}

// ---------------------------------------------------------------- Hamiltonians

template <typename T, int D, int HAM>
__device__ __forceinline__ T ham_value(const StageArgs<T> &a, const int *j, const T *p)
{
    if constexpr (HAM == kHamNormal) {
        T s = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) s += p[d] * p[d];
        return a.hp[0] * sqrt(s);
    } else if constexpr (HAM == kHamDubins3) {
        const T x = a.tab.coord[0][j[0]], y = a.tab.coord[1][j[1]];
        const T c = a.tab.cosv[2][j[2]], sn = a.tab.sinv[2][j[2]];
        const T ve = a.hp[0], vp = a.hp[1], we = a.hp[2], wp = a.hp[3];
        const T drift = p[0] * (-ve + vp * c) + p[1] * (vp * sn);
        return -(drift + we * vabs(p[0] * y - p[1] * x - p[2]) - wp * vabs(p[2]));
    } else {
        const T c = a.tab.cosv[2][j[2]], sn = a.tab.sinv[2][j[2]];
        const T v = a.tab.coord[3][j[3]];
        return -v * (p[0] * c + p[1] * sn) + a.hp[0] * vabs(p[2]) + a.hp[1] * vabs(p[3]);
    }
}

// ---------------------------------------------------------------- stage kernel

template <typename T, int D, int SCHEME, int HAM>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs<T> a)
{
    constexpr int R = Radius<SCHEME>::r;
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= a.g.plane) return;

    int j[kMaxDim];
    if constexpr (D == 1) {
        j[0] = q;
    } else {
        const int nl = a.g.n[D - 1];
        int jm = (int)((double)q / (double)nl);
        int jl = q - jm * nl;
        if (jl < 0) { --jm; jl += nl; } else if (jl >= nl) { ++jm; jl -= nl; }
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

        T pm[D], pp[D];
        T center = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T v[2 * R + 1];
            gather<T, R>(a.phi_in, idx, j[d], a.g.n[d], a.g.stride[d], (a.g.periodic >> d) & 1u, v);
            center = v[R];
            derivatives<T, SCHEME>(v, a.inv_dx[d], a.dx[d], pm[d], pp[d]);
        }

        T pbar[D];
#pragma unroll
        for (int d = 0; d < D; ++d) pbar[d] = T(0.5) * (pm[d] + pp[d]);
        T hhat = ham_value<T, D, HAM>(a, j, pbar);
#pragma unroll
        for (int d = 0; d < D; ++d) hhat -= a.alpha[d] * T(0.5) * (pp[d] - pm[d]);
        const T L = -hhat;

        T res;
        if (a.rhs_only) {
            res = L;
        } else {
            res = a.cb * (center + a.dt * L);
            if (a.ca != T(0)) res += a.ca * a.phi_n[idx];
            if (a.target) {
                const T tg = a.target[idx];
                res = tg < res ? tg : res;
            }
        }
        a.out[idx] = res;
    }
}

template <typename T, int D, int SCHEME, int HAM>
hipError_t launch_one(const StageArgs<T> &a, hipStream_t s)
{
    dim3 grid((a.g.plane + 255) / 256, a.g.slow < 65535 ? a.g.slow : 65535);
    hipLaunchKernelGGL((stage_kernel<T, D, SCHEME, HAM>), grid, dim3(256), 0, s, a);
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
