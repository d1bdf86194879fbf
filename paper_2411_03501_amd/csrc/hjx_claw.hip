// Scalar conservation laws v_t + sum_d f_d(v)_{x_d} = 0 by the Lax-Friedrichs
// scheme (LevelSetPy, arXiv 2411.03501, Sec. IV-D), on gfx950.
//
// One thread per node, the fastest axis along the lanes.  The new value is
// the mean of the 2N axis neighbours minus the central flux differences,
//   v' = (1/2N) sum_d (v_{+d} + v_{-d}) - sum_d (dt/dx_d)/2 (f_d(v_{+d}) - f_d(v_{-d})),
// the printed one-dimensional scheme for N = 1.  The node's own value is not
// an input, so a stage reads 2N neighbours (through L1/L2; HBM sees each value
// about once) and writes one value: the kernel streams, and is bound by HBM.
// Periodic axes wrap; elsewhere the value beyond the edge is the edge value.
#include <algorithm>

#include "hjx_internal.h"

namespace hjx {
namespace {

template <typename T, int FLUX>
__device__ __forceinline__ T claw_flux(T c, T v)
{
    if constexpr (FLUX == kFluxLinear) return c * v;
    else return (T(0.5) * c) * (v * v);
}

template <typename T, int D, int FLUX>
__global__ __launch_bounds__(256) void claw_kernel(ClawArgs<T> a)
{
#pragma clang fp contract(off)
    // XCD-aware order, as in the stage kernel: each XCD takes a contiguous
    // run of blocks, so the rows a block's neighbours reach share its L2
    const int G = (int)(gridDim.x * gridDim.y);
    int lb = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if ((G & 7) == 0) lb = (lb & 7) * (G >> 3) + (lb >> 3);
    const int bx = lb % (int)gridDim.x, by = lb / (int)gridDim.x;
    const int nl = a.n[D - 1];
    const int jl = bx * 256 + (int)threadIdx.x;
    if (jl >= nl) return;
    for (int r = by; r < a.rows; r += (int)gridDim.y) {
        int j[kMaxDim] = {0, 0, 0, 0};
        j[D - 1] = jl;
        int rem = r;
#pragma unroll
        for (int d = D - 2; d >= 0; --d) {
            j[d] = rem % a.n[d];
            rem /= a.n[d];
        }
        const int idx = r * nl + jl;
        T mean = T(0), fl = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int st = a.stride[d];
            const bool per = (a.periodic >> d) & 1u;
            int op = st, om = st;  // offsets to the + and - neighbours
            if (j[d] + 1 >= a.n[d]) op = per ? -(a.n[d] - 1) * st : 0;
            if (j[d] == 0) om = per ? -(a.n[d] - 1) * st : 0;
            const T vp = a.v[idx + op], vm = a.v[idx - om];
            mean = mean + (vp + vm);
            fl = fl + a.half_lam[d] * (claw_flux<T, FLUX>(a.c[d], vp) - claw_flux<T, FLUX>(a.c[d], vm));
        }
        a.out[idx] = mean * a.inv_2n - fl;
    }
}

// max |v| over n values into *out (the bits of a non-negative double, which
// order like the doubles; *out must start at 0)
template <typename T>
__global__ __launch_bounds__(256) void claw_maxabs_kernel(const T *v, int n, unsigned long long *out)
{
    double m = 0.0;
    for (int i = blockIdx.x * 256 + (int)threadIdx.x; i < n; i += gridDim.x * 256) {
        const double x = fabs((double)v[i]);
        m = x > m ? x : m;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// About 4096 blocks, each thread walking rows a.rows / gy apart: one node
// per thread (a grid of every row) left the step bound by starting short
// waves.  At 4096^2 periodic Burgers: 44.9 -> 27.3 us FP32 (3.0 -> 4.9 TB/s)
// and 56.9 -> 52.5 us FP64; 1024 and 16384 blocks were within 10 %.
template <typename T, int D>
hipError_t launch_claw_d(const ClawArgs<T> &a, int flux, hipStream_t s)
{
    const int gx = (a.n[D - 1] + 255) / 256;
    const int gy = std::min(a.rows, std::max(1, 4096 / gx));
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (flux == kFluxLinear) hipLaunchKernelGGL((claw_kernel<T, D, kFluxLinear>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((claw_kernel<T, D, kFluxBurgers>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_claw(const ClawArgs<T> &a, int flux, hipStream_t s)
{
    if (flux != kFluxLinear && flux != kFluxBurgers) return hipErrorInvalidValue;
    switch (a.dim) {
    case 1: return launch_claw_d<T, 1>(a, flux, s);
    case 2: return launch_claw_d<T, 2>(a, flux, s);
    case 3: return launch_claw_d<T, 3>(a, flux, s);
    case 4: return launch_claw_d<T, 4>(a, flux, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_maxabs(const T *v, int n, unsigned long long *out, hipStream_t s)
{
    hipError_t e = launch_zero_f64acc(reinterpret_cast<double *>(out), 1, s);
    if (e != hipSuccess) return e;
    const int blocks = std::min((n + 255) / 256, 1024);
    hipLaunchKernelGGL((claw_maxabs_kernel<T>), dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_claw_f32(const ClawArgs<float> &a, int flux, hipStream_t s) { return launch_claw<float>(a, flux, s); }
hipError_t launch_claw_f64(const ClawArgs<double> &a, int flux, hipStream_t s)
{
    return launch_claw<double>(a, flux, s);
}
hipError_t launch_maxabs_f32(const float *v, int n, unsigned long long *out, hipStream_t s)
{
    return launch_maxabs<float>(v, n, out, s);
}
hipError_t launch_maxabs_f64(const double *v, int n, unsigned long long *out, hipStream_t s)
{
    return launch_maxabs<double>(v, n, out, s);
}

}  // namespace hjx
