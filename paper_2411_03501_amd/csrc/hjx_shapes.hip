// Implicit surfaces and shape operations on the device (LevelSetPy, arXiv
// 2411.03501, Sec. III: implicit surface representations, Listing 2, and the
// calculus on implicit functions), so that initial data is built where it is
// used instead of on the host.
//
// Shapes at every grid node x (node coordinates gmin_d + j_d dx_d, as the
// library's own tables):
//   ball       sqrt(sum_{d in mask} (x_d - c_d)^2) - r  (a sphere over every
//              axis, a cylinder over some);
//   ellipsoid  sum_{d in mask} w_d (x_d - c_d)^2 - r    (Listing 2's form).
// Both are evaluated in double and rounded once to the output type.
// Operations, elementwise: union min(a, b), intersection max(a, b),
// complement -a, subtraction max(a, -b).  All kernels stream one value per
// node: bound by HBM.
#include <algorithm>
#include <mutex>

#include "hjx_internal.h"

namespace hjx {
namespace {

// One thread per node of the fastest axis, walking rows; a row's index is the
// same for the whole block, so its decomposition into the slower axes is
// scalar work.  The sum runs from the fastest axis to the slowest.
template <typename T>
__global__ __launch_bounds__(256) void shape_kernel(ShapeArgs a, T *out)
{
    const int dl = a.dim - 1, nl = a.n[dl];
    const int jl = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (jl >= nl) return;
    double last = 0.0;
    if ((a.mask >> dl) & 1u) {
        const double q = (a.gmin[dl] + (double)jl * a.dx[dl]) - a.center[dl];
        last = a.kind == kShapeBall ? q * q : (a.weights[dl] * q) * q;
    }
    for (int r = (int)blockIdx.y; r < a.rows; r += (int)gridDim.y) {
        int rem = r;
        double acc = last;
        for (int d = dl - 1; d >= 0; --d) {
            const int j = rem % a.n[d];
            rem /= a.n[d];
            if ((a.mask >> d) & 1u) {
                const double q = (a.gmin[d] + (double)j * a.dx[d]) - a.center[d];
                acc = a.kind == kShapeBall ? fma(q, q, acc) : fma(a.weights[d] * q, q, acc);
            }
        }
        out[(long)r * nl + jl] = T((a.kind == kShapeBall ? sqrt(acc) : acc) - a.radius);
    }
}

// Many members in one launch: grid row blockIdx.y is member blockIdx.y, so a
// block's member and its arguments are uniform (scalar loads, no search); the
// blocks of a row stride over the member's nodes, and a node's grid index
// comes from multiplying with a rounded reciprocal of each n and correcting
// by one either way.
template <typename T>
__global__ __launch_bounds__(256) void shape_batch_kernel(const ShapeMember *__restrict__ m, int nm)
{
    const ShapeMember &mb = m[blockIdx.y];
    const ShapeArgs &a = mb.a;
    T *out = static_cast<T *>(mb.out);
    for (long f = (long)blockIdx.x * 256 + threadIdx.x; f < a.total; f += (long)gridDim.x * 256) {
        int rem = (int)f;
        double acc = 0.0;
        for (int d = a.dim - 1; d >= 0; --d) {
            int j = rem;
            if (d > 0) {
                const int n = a.n[d];
                int q = (int)((double)rem * (1.0 / (double)n));
                int r = rem - q * n;
                if (r < 0) {
                    --q;
                    r += n;
                } else if (r >= n) {
                    ++q;
                    r -= n;
                }
                j = r;
                rem = q;
            }
            if ((a.mask >> d) & 1u) {
                const double qd = (a.gmin[d] + (double)j * a.dx[d]) - a.center[d];
                acc = a.kind == kShapeBall ? fma(qd, qd, acc) : fma(a.weights[d] * qd, qd, acc);
            }
        }
        out[f] = T((a.kind == kShapeBall ? sqrt(acc) : acc) - a.radius);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void shape_op_kernel(int op, const T *a, const T *b, T *out, long n)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const T x = a[i];
        T r;
        if (op == kOpUnion) r = b[i] < x ? b[i] : x;
        else if (op == kOpIntersection) r = b[i] > x ? b[i] : x;
        else if (op == kOpComplement) r = -x;
        else r = -b[i] > x ? -b[i] : x;
        out[i] = r;
    }
}

unsigned blocks_for(long n)
{
    const long b = (n + 255) / 256;
    return (unsigned)std::max(1L, std::min(b, 8192L));
}

// about 4096 blocks, as for the conservation-law step
dim3 shape_grid(const ShapeArgs &a)
{
    const int gx = (a.n[a.dim - 1] + 255) / 256;
    return dim3((unsigned)gx, (unsigned)std::min(a.rows, std::max(1, 4096 / gx)));
}

}  // namespace

hipError_t launch_shape_f32(const ShapeArgs &a, float *out, hipStream_t s)
{
    hipLaunchKernelGGL((shape_kernel<float>), shape_grid(a), dim3(256), 0, s, a, out);
    return hipGetLastError();
}
hipError_t launch_shape_f64(const ShapeArgs &a, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((shape_kernel<double>), shape_grid(a), dim3(256), 0, s, a, out);
    return hipGetLastError();
}
// blocks per member row: enough for the largest member, about 16 K blocks in all
dim3 batch_grid(int nm, long largest)
{
    const long per = std::max(1L, std::min((largest + 255) / 256, std::max(8L, 16384L / nm)));
    return dim3((unsigned)per, (unsigned)nm);
}

hipError_t launch_shape_batch_f32(const ShapeMember *members, int nm, long largest, hipStream_t s)
{
    hipLaunchKernelGGL((shape_batch_kernel<float>), batch_grid(nm, largest), dim3(256), 0, s, members, nm);
    return hipGetLastError();
}
hipError_t launch_shape_batch_f64(const ShapeMember *members, int nm, long largest, hipStream_t s)
{
    hipLaunchKernelGGL((shape_batch_kernel<double>), batch_grid(nm, largest), dim3(256), 0, s, members, nm);
    return hipGetLastError();
}
// The descriptor staging of hjx_shape_batch_noalloc: a file-scope device
// array of kShapeNoAllocMax members, one copy on every GPU the library runs
// on, held until the process ends.  On the host its name is only a stand-in:
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) ShapeMember scratch[kShapeNoAllocMax];

hipError_t shape_noalloc_scratch(ShapeMember **out)
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static ShapeMember *addr[kDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<ShapeMember *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_shape_op_f32(int op, const float *a, const float *b, float *out, long n, hipStream_t s)
{
    hipLaunchKernelGGL((shape_op_kernel<float>), dim3(blocks_for(n)), dim3(256), 0, s, op, a, b, out, n);
    return hipGetLastError();
}
hipError_t launch_shape_op_f64(int op, const double *a, const double *b, double *out, long n, hipStream_t s)
{
    hipLaunchKernelGGL((shape_op_kernel<double>), dim3(blocks_for(n)), dim3(256), 0, s, op, a, b, out, n);
    return hipGetLastError();
}

}  // namespace hjx
