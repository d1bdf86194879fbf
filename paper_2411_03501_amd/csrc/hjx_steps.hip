// The steps variant of 1-D and 2-D grids: several whole RK steps (Sec. V,
// Sec. VI) of one output tile per launch, each stage with the node
// arithmetic of the other stage kernels (Sec. IV-A..IV-D: node_derivs,
// stage_rate), so the same bits.  The tile and a halo of k * rk * radius
// nodes sit in LDS; each stage runs on the part of that region whose inputs
// are still exact, which shrinks by the radius per stage on every side that
// is not a non-periodic end of the grid (there the ghost rule needs only the
// two end nodes, which stay exact).  After k steps the tile is exact and is
// stored.  Small grids are bound by the gaps between dependent launches, not
// by arithmetic, and this trades redundant halo work for k - 1 fewer gaps.
#include "hjx_device.h"

namespace hjx {
namespace {

using namespace dev;

constexpr int kStepsThreads = 256;

// q mod n for -n <= q < 2n (a periodic halo is at most one period deep)
__device__ __forceinline__ int wrap1(int q, int n) { return q < 0 ? q + n : (q >= n ? q - n : q); }

// floor((q + 0.5) / w) for 0 <= q < 2^20 from the float reciprocal rw of w:
// the product lies within 2^-3 / w of (q + 0.5) / w, which is at least
// 0.5 / w away from every integer, so the floor is exact.
__device__ __forceinline__ int row_of(int q, float rw) { return (int)(((float)q + 0.5f) * rw); }

// phi at offsets -3..3 along one axis from LDS index p, the node being at
// position q of a region w long along that axis with LDS stride s.  Offsets
// beyond the scheme's radius R are never read by the scheme and hold the
// node's own value.  Where the region starts (lo) or ends (hi) at a
// non-periodic end of the grid, region positions are grid coordinates from
// that end and the ghosts are gather7's linear extrapolation from the two end
// nodes, with its arithmetic; everywhere else the region holds the
// neighbours themselves (a periodic axis is unrolled into the halo).
template <typename T, int R>
__device__ __forceinline__ void gather_lds(const T *buf, int p, int q, int w, int s, bool lo, bool hi, T (&v)[7])
{
    v[3] = buf[p];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const int o = k - 3;
        if (o == 0) continue;
        if (o < -R || o > R) {
            v[k] = v[3];
            continue;
        }
        const int qq = q + o;
        if (lo && qq < 0) {
            const T p0 = buf[p - q * s], p1 = buf[p + (1 - q) * s];
            v[k] = fmaT(T(-qq), p0 - p1, p0);
        } else if (hi && qq >= w) {
            const T p0 = buf[p + (w - 1 - q) * s], p1 = buf[p + (w - 2 - q) * s];
            v[k] = fmaT(T(qq - w + 1), p0 - p1, p0);
        } else {
            v[k] = buf[p + o * s];
        }
    }
}

// l.k RK steps of one tile.  Block b owns tile (b mod tiles_x, b / tiles_x)
// of the output: x (the fastest axis) by y (axis 0 of a 2-D grid).  LDS holds
// two or three buffers of l.area_max values: P, phi^n of the current step
// (and, for forward Euler, the stage input), and the stage results X (and Y
// for the middle stage of RK3).  A stage writes only nodes that no thread
// reads in the same stage: X and Y are read in the stage after the one that
// writes them, and the last stage of RK2 and RK3 rewrites P at its own node,
// where it is the only reader of P.
template <typename T, int D, int SCHEME, int HAM, int MODE>
__global__ __launch_bounds__(kStepsThreads) void steps_kernel(StageArgs<T> a, StepsLaunch l)
{
    extern __shared__ __align__(16) unsigned char steps_lds[];
    constexpr int R = scheme_radius(SCHEME);
    constexpr int X = D - 1;  // the fastest axis
    const int nx = a.g.n[X], ny = D == 2 ? a.g.n[0] : 1;
    const bool perx = (a.g.periodic >> X) & 1u, pery = D == 2 && (a.g.periodic & 1u);
    const int by = (int)blockIdx.x / l.tiles_x, bx = (int)blockIdx.x - by * l.tiles_x;
    const int x0 = bx * l.tx, x1 = min(x0 + l.tx, nx);
    const int y0 = by * l.ty, y1 = min(y0 + l.ty, ny);
    const int H = l.k * l.rk * R;
    const int rx0 = perx ? x0 - H : max(x0 - H, 0), rx1 = perx ? x1 + H : min(x1 + H, nx);
    int ry0 = 0, ry1 = 1;
    if (D == 2) {
        ry0 = pery ? y0 - H : max(y0 - H, 0);
        ry1 = pery ? y1 + H : min(y1 + H, ny);
    }
    const int w = rx1 - rx0, h = ry1 - ry0;
    const bool xlo = !perx && rx0 == 0, xhi = !perx && rx1 == nx;
    const bool ylo = D == 2 && !pery && ry0 == 0, yhi = D == 2 && !pery && ry1 == ny;
    T *P = reinterpret_cast<T *>(steps_lds);
    T *Xb = P + l.area_max;
    T *const Yb = Xb + l.area_max;  // RK3 only

    // the region from the stage input, periodic axes wrapped (every node of
    // the input lies in some block's region, so with flag_in the launch also
    // checks the whole input for NaN and Inf)
    const float rw = 1.0f / (float)w;
    bool bad = false;
    for (int q = threadIdx.x; q < w * h; q += kStepsThreads) {
        const int py = D == 2 ? row_of(q, rw) : 0, px = q - py * w;
        const int gx = wrap1(rx0 + px, nx), gy = D == 2 ? wrap1(ry0 + py, ny) : 0;
        const T v = ld32(a.phi_in, gy * nx + gx);
        bad |= !__builtin_isfinite(v);
        P[q] = v;
    }
    if (l.flag_in && bad) atomicOr(l.flag_in, 1);
    __syncthreads();

    int m = 0;  // stages done
    for (int step = 0; step < l.k; ++step) {
        const T dt = T(step + 1 == l.k ? l.dt_last : l.dt);
        for (int st = 0; st < l.rk; ++st) {
            ++m;
            // the stage: out = ca phi^n + cb (in + dt L(in)), the averages of
            // odeCFL2 / odeCFL3 in the host's rounding of each coefficient
            const T *in = P;
            T *out = Xb;
            T ca = T(0), cb = T(1);
            if (st == 1 && l.rk == 2) {
                in = Xb;
                out = P;
                ca = T(0.5);
                cb = T(0.5);
            } else if (st == 1) {
                in = Xb;
                out = Yb;
                ca = T(0.75);
                cb = T(0.25);
            } else if (st == 2) {
                in = Yb;
                out = P;
                ca = T(1.0 / 3.0);
                cb = T(2.0 / 3.0);
            }
            const bool with_target = st + 1 == l.rk && a.target != nullptr;
            // nodes still exact after m stages
            const int vx0 = xlo ? 0 : m * R, vx1 = xhi ? w : w - m * R;
            int vy0 = 0, vy1 = 1;
            if (D == 2) {
                vy0 = ylo ? 0 : m * R;
                vy1 = yhi ? h : h - m * R;
            }
            const int cw = vx1 - vx0, cnt = cw * (vy1 - vy0);
            const float rcw = 1.0f / (float)cw;
            for (int q = threadIdx.x; q < cnt; q += kStepsThreads) {
                const int qy = D == 2 ? row_of(q, rcw) : 0;
                const int px = vx0 + (q - qy * cw), py = vy0 + qy;
                const int p = py * w + px;
                T pm[D], pp[D], v[7];
                gather_lds<T, R>(in, p, px, w, 1, xlo, xhi, v);
                node_derivs<T, SCHEME>(v, a.inv_dx[X], a.dx[X], pm[X], pp[X]);
                const T center = v[3];
                if constexpr (D == 2) {
                    gather_lds<T, R>(in, p, py, h, w, ylo, yhi, v);
                    node_derivs<T, SCHEME>(v, a.inv_dx[0], a.dx[0], pm[0], pp[0]);
                }
                const int gx = wrap1(rx0 + px, nx), gy = D == 2 ? wrap1(ry0 + py, ny) : 0;
                const int j[kMaxDim] = {D == 2 ? gy : gx, gx, 0, 0};
                const T L = stage_rate<T, D, HAM, MODE>(a, j, pm, pp);
                T res = cb * fmaT(dt, L, center);
                if (ca != T(0)) res = fmaT(ca, P[p], res);
                if (with_target) {
                    const T tg = ld32(a.target, gy * nx + gx);
                    res = tg < res ? tg : res;
                }
                out[p] = res;
            }
            __syncthreads();
            if (l.rk == 1) {  // forward Euler: the result is the next step's input
                T *t = P;
                P = Xb;
                Xb = t;
            }
        }
    }

    // the tile itself
    const int tw = x1 - x0, tcnt = tw * (y1 - y0);
    const float rtw = 1.0f / (float)tw;
    bad = false;
    for (int q = threadIdx.x; q < tcnt; q += kStepsThreads) {
        const int qy = D == 2 ? row_of(q, rtw) : 0;
        const int x = x0 + (q - qy * tw), y = y0 + qy;
        const T v = P[(y - ry0) * w + (x - rx0)];
        bad |= !__builtin_isfinite(v);
        at32(a.out, y * nx + x) = v;
    }
    if (l.flag_out && bad) atomicOr(l.flag_out, 1);
}

template <typename T, int D, int SCHEME, int HAM, int M>
hipError_t launch_steps_mode(const StageArgs<T> &a, const StepsLaunch &l, hipStream_t s)
{
    const int nx = a.g.n[D - 1], ny = D == 2 ? a.g.n[0] : 1;
    const int H = l.k * l.rk * scheme_radius(SCHEME);
    const size_t lds = (size_t)steps_buffers(l.rk) * (size_t)l.area_max * sizeof(T);
    const bool perx = (a.g.periodic >> (D - 1)) & 1u, pery = D == 2 && (a.g.periodic & 1u);
    if (l.k < 1 || l.rk < 1 || l.rk > 3 || l.tx < 1 || l.ty < 1 || (D == 1 && l.ty != 1) ||
        l.tiles_x != (nx + l.tx - 1) / l.tx || lds > kStepsLdsMax || l.area_max >= (1 << 20) ||
        l.area_max < steps_area(l.tx, l.ty, H, nx, ny, perx, pery, D == 2) || (perx && H > nx) || (pery && H > ny))
        return hipErrorInvalidConfiguration;
    const long blocks = (long)l.tiles_x * ((ny + l.ty - 1) / l.ty);
    hipLaunchKernelGGL((steps_kernel<T, D, SCHEME, HAM, M>), dim3((unsigned)blocks), dim3(kStepsThreads), lds, s, a,
                       l);
    return hipGetLastError();
}

// node modes as launch_one picks them (no kept p-, p+: the tape steps stage
// by stage)
template <typename T, int D, int SCHEME, int HAM>
hipError_t steps_one(const StageArgs<T> &a, const StepsLaunch &l, hipStream_t s)
{
    const int mode = (a.clip != 0 ? kNodeClip : 0) | (a.diss == 1 ? kNodeLocal : 0);
    if constexpr (HAM == kHamNormalGodunov) {
        if (mode == kNodePlain) return launch_steps_mode<T, D, SCHEME, HAM, kNodePlain>(a, l, s);
        if (mode == kNodeClip) return launch_steps_mode<T, D, SCHEME, HAM, kNodeClip>(a, l, s);
        return hipErrorInvalidValue;
    }
    switch (mode) {
    case kNodePlain: return launch_steps_mode<T, D, SCHEME, HAM, kNodePlain>(a, l, s);
    case kNodeClip: return launch_steps_mode<T, D, SCHEME, HAM, kNodeClip>(a, l, s);
    case kNodeLocal: return launch_steps_mode<T, D, SCHEME, HAM, kNodeLocal>(a, l, s);
    case kNodeLocal | kNodeClip: return launch_steps_mode<T, D, SCHEME, HAM, kNodeLocal | kNodeClip>(a, l, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int D, int HAM>
hipError_t steps_scheme(const StageArgs<T> &a, const StepsLaunch &l, int scheme, hipStream_t s)
{
    switch (scheme) {
    case kSchemeFirst: return steps_one<T, D, kSchemeFirst, HAM>(a, l, s);
    case kSchemeEno2: return steps_one<T, D, kSchemeEno2, HAM>(a, l, s);
    case kSchemeEno3: return steps_one<T, D, kSchemeEno3, HAM>(a, l, s);
    case kSchemeWeno5: return steps_one<T, D, kSchemeWeno5, HAM>(a, l, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_steps(const StageArgs<T> &a, const StepsLaunch &l, int scheme, int ham, hipStream_t s)
{
    if (ham != kHamNormal || a.rhs_only || a.dp_out || a.mask || a.phi_in == a.out) return hipErrorInvalidValue;
    const bool god = a.diss == 2;
    switch (a.g.dim) {
    case 1: return god ? steps_scheme<T, 1, kHamNormalGodunov>(a, l, scheme, s) : steps_scheme<T, 1, kHamNormal>(a, l, scheme, s);
    case 2: return god ? steps_scheme<T, 2, kHamNormalGodunov>(a, l, scheme, s) : steps_scheme<T, 2, kHamNormal>(a, l, scheme, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_steps_f32(const StageArgs<float> &a, const StepsLaunch &l, int scheme, int ham, hipStream_t s)
{
    return launch_steps<float>(a, l, scheme, ham, s);
}

hipError_t launch_steps_f64(const StageArgs<double> &a, const StepsLaunch &l, int scheme, int ham, hipStream_t s)
{
    return launch_steps<double>(a, l, scheme, ham, s);
}

}  // namespace hjx
