// Adjoint (reverse mode) of the fused level-set stage on gfx950.
//
// The forward stage is out = ca phi_n + cb (phi_in + h L(phi_in)), then
// min with the target, where L = -(H(x, pbar) - sum_d alpha_d (p+_d - p-_d)/2)
// and p-_d, p+_d are the upwind derivative approximations (LevelSetPy,
// arXiv 2411.03501: Sec. IV-A..IV-D, Sec. V, Sec. VI).  Its reverse takes
// two kinds of kernel:
//   adj_seed_kernel  one or two nodes per thread: reads p-, p+ kept by the
//                    replay (or evaluates them again) and H at phi_in, turns
//                    lam_out (plus the per-axis sums still pending from the
//                    stage reversed before) into the seeds w dL/dp-_d,
//                    w dL/dp+_d (w = cb h lam_out), writes the pass-through
//                    parts of the adjoint and accumulates dL/dh, dL/dalpha
//                    and dL/dtheta per block; adj_seed_replay_kernel runs the
//                    same blocks beside those of one forward stage of the
//                    replay of the preceding segment;
//   adj_axes_kernel  one launch for all axes, line tiles of each axis in LDS:
//                    every derivative interval is recomputed once, its
//                    transpose applied to the seeds of its two nodes, and
//                    each node gathers the contributions of the six
//                    intervals whose stencils contain it; contributions to
//                    extrapolated ghost cells are folded back onto the two
//                    end nodes they were extrapolated from.  Each axis writes
//                    its own sum (added by the next seed kernel, or by
//                    combine_kernel at the end).
#include "hjx_adjoint_device.h"

#include <algorithm>

namespace hjx {
namespace {

using namespace dev;

constexpr int kSeedThreads = 256;
constexpr int kAxisThreads = 256;  // block of the per-axis transpose

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Reduce-scatter over the 64 lanes of a wave: each lane brings V values
// (V a power of two, at most 64); at every butterfly step a lane keeps half
// of its values and adds its partner's copy of that half, so value i ends
// summed over all lanes in the lanes whose bits 5, 4, ... spell i (lane
// i << (6 - log2 V) among them).  About V + log2(64/V) exchanges instead of
// 6 V for V separate sums.  Returns the value this lane holds.
template <int V>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[V], int lane)
{
    static_assert(V >= 1 && V <= 64 && (V & (V - 1)) == 0, "V must be a power of two");
    int off = 32;
#pragma unroll
    for (int half = V / 2; half >= 1; half >>= 1, off >>= 1) {
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            // the empty asm pins both values in registers: without it the
            // two selects fold into one array access at a lane-dependent
            // index, a chain of selects over all V values
            double lo = v[i], hi = v[i + half];
            asm volatile("" : "+v"(lo), "+v"(hi));
            const double send = upper ? lo : hi;
            const double keep = upper ? hi : lo;
            v[i] = keep + __shfl_xor(send, off, 64);
        }
    }
    double x = v[0];
    for (; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <int HAM>
constexpr int ham_params()
{
    return HAM == kHamDubins3 || HAM == kHamRockets ? 4 : (HAM == kHamDubins4 ? 2 : 1);
}

constexpr int pow2_at_least(int n) { return n <= 1 ? 1 : 2 * pow2_at_least((n + 1) / 2); }

// ---------------------------------------------------------------- seeds

// Planes of the slow axes per seed block: with two, each thread has the
// loads of two nodes in flight at once and the block reduction serves twice
// the nodes.  Only FP32 with stored derivatives stays within 64 vector
// registers (8 waves per SIMD) that way.
template <typename T, int D, bool STORED>
constexpr int seed_planes()
{
    return sizeof(T) == 4 && STORED && D >= 3 ? 2 : 1;
}

// The operands of one node of the seed pass, all loaded before any is used.
template <typename T, int D>
struct SeedNode {
    int idx, j[kMaxDim];
    T lo, add[kMaxDim], in_old, n_old, tg_old;
    unsigned char mk;
    T pm[D], pp[D];
    HamTab<T> tb;
};

// Every load of a node, issued before any arithmetic needs one, so that a
// wave waits for memory once (an operand that a uniform flag leaves out is
// the constant 0, never a copy of another load).  The sweep never aliases
// lam_out, lam_in, lam_n and lam_target.
template <typename T, int D, int SCHEME, int HAM, bool STORED>
__device__ __forceinline__ void seed_load(const AdjSeedArgs<T> &a, SeedNode<T, D> &s)
{
    const StageArgs<T> &st = a.st;
    const int idx = s.idx;
    s.lo = ld32(a.lam_out, idx);
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k) s.add[k] = k < a.n_add ? ld32(a.lam_add[k], idx) : T(0);
    // (the mask byte is read unconditionally, from lam_out's first bytes
    // when there is no mask, so that its test is not a branch on a load)
    s.mk = ld32(a.mask ? a.mask : reinterpret_cast<const unsigned char *>(a.lam_out), idx);
    s.in_old = a.in_mode ? ld32(a.lam_in, idx) : T(0);
    s.n_old = a.n_mode == 2 ? ld32(a.lam_n, idx) : T(0);
    s.tg_old = a.lam_target ? ld32(a.lam_target, idx) : T(0);
    if constexpr (STORED) {  // the replay kept them
#pragma unroll
        for (int d = 0; d < D; ++d) {
            s.pm[d] = ld32(a.dp_in + (size_t)(2 * d) * (size_t)a.dp_stride, idx);
            s.pp[d] = ld32(a.dp_in + (size_t)(2 * d + 1) * (size_t)a.dp_stride, idx);
        }
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T v[7];
            if (d == D - 1) gather7_row(st.phi_in, idx, s.j[d], st.g.n[d], (st.g.periodic >> d) & 1u, v);
            else gather7(st.phi_in, idx, s.j[d], st.g.n[d], st.g.stride[d], (st.g.periodic >> d) & 1u, v);
            node_derivs<T, SCHEME>(v, st.inv_dx[d], st.dx[d], s.pm[d], s.pp[d]);
        }
    }
    s.tb = ham_tab<T, D, HAM>(st, s.j);
}

// The arithmetic and stores of one node; its block-sum terms are added to
// part: [0] dL/dh, [1..D] dL/dalpha_d, [D+1..D+NP] dL/dtheta.
template <typename T, int D, int HAM, int V, bool LOCAL>
__device__ __forceinline__ void seed_finish(const AdjSeedArgs<T> &a, const SeedNode<T, D> &s, double (&part)[V])
{
    const StageArgs<T> &st = a.st;
    constexpr int NP = ham_params<HAM>();
    const int idx = s.idx;
    T lo = s.lo;
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k)
        if (k < a.n_add) lo += s.add[k];
    // where the target was kept (bit 0 of the mask), its adjoint takes
    // lam_out; where the replay clipped the rate (bit 1), the rate is the
    // constant 0 and takes no adjoint
    const bool kept = a.mask != nullptr && (s.mk & 1) != 0;
    const bool clipped = a.mask != nullptr && (s.mk & 2) != 0;
    const T tg_new = s.tg_old + lo;
    if (kept) lo = T(0);
    T dmH[8] = {};
    T hhat;
    const T w = clipped ? T(0) : a.cb * a.h * lo;
    if constexpr (HAM == kHamNormalGodunov) {
        // Godunov's Hamiltonian for a|p|: Hhat = a |q| with q_d the one-sided
        // value each axis selects (as stage_rate selects it, ties alike), so
        // dHhat/dp-_d, dHhat/dp+_d = (a q_d / |q|) dq_d/dp-_d, dq_d/dp+_d
        // (0 where q = 0), and d(-Hhat)/da = -|q|.  No alpha.
        const T av = st.hp[0];
        T q[D], gm[D], gp[D];
        T ss = T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const T pm = s.pm[d], pp = s.pp[d];
            if (av >= T(0)) {
                const T up = pm > T(0) ? pm : T(0), dn = pp < T(0) ? -pp : T(0);
                const bool takedn = dn > up;
                q[d] = takedn ? dn : up;
                gm[d] = !takedn && pm > T(0) ? T(1) : T(0);
                gp[d] = takedn && pp < T(0) ? T(-1) : T(0);
            } else {
                const T dn = pm < T(0) ? -pm : T(0), up = pp > T(0) ? pp : T(0);
                const bool takeup = up > dn;
                q[d] = takeup ? up : dn;
                gm[d] = !takeup && pm < T(0) ? T(-1) : T(0);
                gp[d] = takeup && pp > T(0) ? T(1) : T(0);
            }
            ss = fmaT(q[d], q[d], ss);
        }
        const T nq = sqrt(ss);
        hhat = av * nq;
        const T inv = nq > T(0) ? av / nq : T(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const T dq = inv * q[d];  // dHhat/dq_d; L = -Hhat
            at32(a.seed_m[d], idx) = w * (-dq * gm[d]);
            at32(a.seed_p[d], idx) = w * (-dq * gp[d]);
        }
        dmH[0] = -nq;
    } else {
        T pbar[D], dHdp[kMaxDim] = {};
#pragma unroll
        for (int d = 0; d < D; ++d) pbar[d] = T(0.5) * (s.pm[d] + s.pp[d]);
        hhat = ham_grad<T, D, HAM>(st, s.tb, pbar, dHdp, dmH);
        // alpha_d: the grid maximum, or (LOCAL) the bound at the node, whose
        // parameter gradient then joins dL/dtheta here (the grid maxima only
        // reach the parameters through the CFL step)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T al = st.alpha[d];
            const T half = T(0.5) * (s.pp[d] - s.pm[d]);
            if constexpr (LOCAL) {
                T dbnd[8];
                al = bound_grad<T, D, HAM>(st, s.tb, d, dbnd);
#pragma unroll
                for (int m = 0; m < NP; ++m) dmH[m] = fmaT(half, dbnd[m], dmH[m]);
            } else {
                part[1 + d] += (double)(w * half);
            }
            hhat = fmaT(-al, half, hhat);
            // L = -H(pbar) + sum alpha (p+ - p-)/2, pbar = (p- + p+)/2
            at32(a.seed_m[d], idx) = w * (T(-0.5) * dHdp[d] - T(0.5) * al);
            at32(a.seed_p[d], idx) = w * (T(-0.5) * dHdp[d] + T(0.5) * al);
        }
    }
    const T L = -hhat;
#pragma unroll
    for (int m = 0; m < NP; ++m) part[1 + D + m] += (double)(w * dmH[m]);
    if (!clipped) part[0] += (double)(a.cb * lo) * (double)L;

    if (kept && a.lam_target) at32(a.lam_target, idx) = tg_new;
    const T cin = a.cb * lo;
    at32(a.lam_in, idx) = a.in_mode ? s.in_old + cin : cin;
    if (a.n_mode) {
        const T cn = a.ca * lo;
        at32(a.lam_n, idx) = a.n_mode == 2 ? s.n_old + cn : cn;
    }
}

// Block (bx, by) of the seed pass: nodes bx*256 .. of the planes
// by*P .. by*P+P-1 of the slow axes (P = seed_planes), gx blocks per plane.
// Every thread of the block must call it (block reduction).
template <typename T, int D, int SCHEME, int HAM, bool STORED, bool LOCAL>
__device__ __forceinline__ void seed_block(const AdjSeedArgs<T> &a, int bx, int by, int gx)
{
    const StageArgs<T> &st = a.st;
    constexpr int P = seed_planes<T, D, STORED>();
    const int q = bx * kSeedThreads + threadIdx.x;
    const bool live = q < st.g.plane;
    constexpr int NP = ham_params<HAM>();
    constexpr int V = pow2_at_least(1 + D + NP);
    double part[V] = {};

    int jm = 0, jl = 0;
    if (live && D >= 2) {
        const int nl = st.g.n[D - 1];
        jm = (int)((double)q / (double)nl);
        jl = q - jm * nl;
        if (jl < 0) {
            --jm;
            jl += nl;
        } else if (jl >= nl) {
            ++jm;
            jl -= nl;
        }
    }
    SeedNode<T, D> nd[P];
    bool ok[P];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const int sy = by * P + r;
        ok[r] = live && sy < st.g.slow;
        if (ok[r]) {
            int *j = nd[r].j;
            j[0] = j[1] = j[2] = j[3] = 0;
            if constexpr (D == 1) {
                j[0] = q;
            } else {
                j[D - 2] = jm;
                j[D - 1] = jl;
            }
            if constexpr (D == 3) j[0] = sy;
            if constexpr (D == 4) {
                j[0] = sy / st.g.n[1];
                j[1] = sy - j[0] * st.g.n[1];
            }
            int idx = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) idx += j[d] * st.g.stride[d];
            nd[r].idx = idx;
            seed_load<T, D, SCHEME, HAM, STORED>(a, nd[r]);
        }
    }
    // Block sums of each plane apart, into the slot of that plane's blocks,
    // (plane) gx + bx, in a fixed order: the same sums, to the bit, for any
    // number of planes per block.  Whether a plane exists is uniform over
    // the block, so every thread reaches the same barriers.
    __shared__ double red[kSeedThreads / 64][V];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kShift = 6 - (V == 1 ? 0 : V == 2 ? 1 : V == 4 ? 2 : V == 8 ? 3 : V == 16 ? 4 : 5);
#pragma unroll
    for (int r = 0; r < P; ++r) {
        const int sy = by * P + r;
        if (sy >= st.g.slow) break;
#pragma unroll
        for (int k = 0; k < V; ++k) part[k] = 0.0;
        if (ok[r]) seed_finish<T, D, HAM, V, LOCAL>(a, nd[r], part);
        if (r > 0) __syncthreads();  // red of the plane before has been read
        const double mine = wave_reduce_scatter<V>(part, lane);
        if ((lane & ((1 << kShift) - 1)) == 0) red[wave][lane >> kShift] = mine;
        __syncthreads();
        if (threadIdx.x < 1 + D + NP) {
            const int k = threadIdx.x;
            double s = 0.0;
            for (int w = 0; w < kSeedThreads / 64; ++w) s += red[w][k];
            const int acc_slot = k == 0 ? a.h_slot : (k <= D ? kAccAlpha + (k - 1) : kAccTheta + (k - 1 - D));
            a.acc[(sy * gx + bx) * kAccCount + acc_slot] += s;
        }
    }
}

template <typename T, int D, int SCHEME, int HAM, bool STORED, bool LOCAL>
__global__ __launch_bounds__(kSeedThreads) __attribute__((amdgpu_num_sgpr(96))) void adj_seed_kernel(AdjSeedArgs<T> a)
{
    seed_block<T, D, SCHEME, HAM, STORED, LOCAL>(a, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// The seed pass of one reversed stage and one forward stage of the replay of
// the preceding segment, in one launch.  The two are independent: the seed
// pass waits on memory, the forward stage on arithmetic, so blocks of both
// kinds sharing the CUs overlap well.  Both cover the grid in blocks of 256
// nodes of a plane (gx per plane): ns seed blocks of P planes each, nr stage
// blocks of one plane.  They are dealt in groups of one run of eight seed
// blocks and P runs of eight stage blocks, so that each XCD (blocks go to the
// eight XCDs in turn) takes both kinds; the leftovers of each kind follow.  A
// block keeps its XCD's residue mod 8 in its own numbering, and the stage
// blocks are renumbered, as in the direct stage kernel, so that each XCD
// walks a contiguous run of them.  The stage keeps p-, p+ (dp_out) exactly
// when the seed pass reads them.
template <typename T, int D, int SCHEME, int HAM, bool STORED, bool LOCAL>
__global__ __launch_bounds__(kSeedThreads) __attribute__((amdgpu_num_sgpr(96))) void adj_seed_replay_kernel(
    AdjSeedArgs<T> a, StageArgs<T> r, int gx, int ns, int nr)
{
    constexpr int P = seed_planes<T, D, STORED>();
    constexpr int G = 8 * (1 + P);
    const int lb = (int)blockIdx.x;
    const int groups = min(ns / 8, nr / (8 * P));
    bool seed;
    int idx;
    if (lb < groups * G) {
        const int g = lb / G, o = lb - g * G;
        seed = o < 8;
        idx = seed ? g * 8 + o : (g * P + ((o - 8) >> 3)) * 8 + (o & 7);
    } else {
        const int t = lb - groups * G, left = ns - groups * 8;
        seed = t < left;
        idx = seed ? groups * 8 + t : groups * 8 * P + (t - left);
    }
    if (seed) {
        seed_block<T, D, SCHEME, HAM, STORED, LOCAL>(a, idx % gx, idx / gx, gx);
        return;
    }
    if ((nr & 7) == 0) idx = (idx & 7) * (nr >> 3) + (idx >> 3);
    const int bx = idx % gx, by = idx / gx;
    const int q = bx * kSeedThreads + threadIdx.x;
    if (q >= r.g.plane) return;
    int j[kMaxDim] = {0, 0, 0, 0};
    if constexpr (D == 1) {
        j[0] = q;
    } else {
        const int nl = r.g.n[D - 1];
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
    if constexpr (D == 3) j[0] = by;
    if constexpr (D == 4) {
        j[0] = by / r.g.n[1];
        j[1] = by - j[0] * r.g.n[1];
    }
    // clip and mark take effect only for a restricted update (r.clip != 0):
    // otherwise the values, and the target mask of a last stage, are those
    // of the plain replay
    direct_node<T, D, SCHEME, HAM,
                (STORED ? kNodeKeep : kNodePlain) | kNodeClip | kNodeMark | (LOCAL ? kNodeLocal : kNodePlain)>(r, j);
}

template <typename T, int D, int SCHEME, int HAM, bool LOCAL>
hipError_t launch_seed_one(const AdjSeedArgs<T> &a, const StageArgs<T> *rep, hipStream_t s)
{
    const int gx = (a.st.g.plane + kSeedThreads - 1) / kSeedThreads;
    if (rep) {
        // same geometry for both jobs; p-, p+ kept exactly when read
        if ((rep->dp_out != nullptr) != (a.dp_in != nullptr) || rep->g.plane != a.st.g.plane ||
            rep->g.slow != a.st.g.slow)
            return hipErrorInvalidValue;
        const long nr = (long)gx * a.st.g.slow;
        const int P = a.dp_in ? seed_planes<T, D, true>() : seed_planes<T, D, false>();
        const long ns = (long)gx * ((a.st.g.slow + P - 1) / P);
        if (ns + nr > 0x7fffffffL) return hipErrorInvalidConfiguration;
        const dim3 grid((unsigned)(ns + nr));
        if (a.dp_in)
            hipLaunchKernelGGL((adj_seed_replay_kernel<T, D, SCHEME, HAM, true, LOCAL>), grid, dim3(kSeedThreads), 0, s, a,
                               *rep, gx, (int)ns, (int)nr);
        else
            hipLaunchKernelGGL((adj_seed_replay_kernel<T, D, SCHEME, HAM, false, LOCAL>), grid, dim3(kSeedThreads), 0, s, a,
                               *rep, gx, (int)ns, (int)nr);
        return hipGetLastError();
    }
    const int P = a.dp_in ? seed_planes<T, D, true>() : seed_planes<T, D, false>();
    dim3 grid(gx, (a.st.g.slow + P - 1) / P);
    if (a.dp_in)
        hipLaunchKernelGGL((adj_seed_kernel<T, D, SCHEME, HAM, true, LOCAL>), grid, dim3(kSeedThreads), 0, s, a);
    else
        hipLaunchKernelGGL((adj_seed_kernel<T, D, SCHEME, HAM, false, LOCAL>), grid, dim3(kSeedThreads), 0, s, a);
    return hipGetLastError();
}

template <typename T, int D, int HAM, bool LOCAL>
hipError_t launch_seed_local(const AdjSeedArgs<T> &a, const StageArgs<T> *rep, int scheme, hipStream_t s)
{
    switch (scheme) {
    case kSchemeFirst: return launch_seed_one<T, D, kSchemeFirst, HAM, LOCAL>(a, rep, s);
    case kSchemeEno2: return launch_seed_one<T, D, kSchemeEno2, HAM, LOCAL>(a, rep, s);
    case kSchemeEno3: return launch_seed_one<T, D, kSchemeEno3, HAM, LOCAL>(a, rep, s);
    case kSchemeWeno5: return launch_seed_one<T, D, kSchemeWeno5, HAM, LOCAL>(a, rep, s);
    }
    return hipErrorInvalidValue;
}

// the global dissipation, or alpha_d at the node (a.st.diss == 1)
template <typename T, int D, int HAM>
hipError_t launch_seed_scheme(const AdjSeedArgs<T> &a, const StageArgs<T> *rep, int scheme, hipStream_t s)
{
    if constexpr (HAM == kHamNormalGodunov) return launch_seed_local<T, D, HAM, false>(a, rep, scheme, s);
    if (a.st.diss == 1) return launch_seed_local<T, D, HAM, true>(a, rep, scheme, s);
    if (a.st.diss == 0) return launch_seed_local<T, D, HAM, false>(a, rep, scheme, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_seed(const AdjSeedArgs<T> &a, const StageArgs<T> *rep, int scheme, int ham, hipStream_t s)
{
    if (a.st.g.slow > 65535) return hipErrorInvalidConfiguration;
    if (ham == kHamDubins3) return a.st.g.dim == 3 ? launch_seed_scheme<T, 3, kHamDubins3>(a, rep, scheme, s)
                                                   : hipErrorInvalidValue;
    if (ham == kHamDubins4) return a.st.g.dim == 4 ? launch_seed_scheme<T, 4, kHamDubins4>(a, rep, scheme, s)
                                                   : hipErrorInvalidValue;
    if (ham == kHamRockets) return a.st.g.dim == 3 ? launch_seed_scheme<T, 3, kHamRockets>(a, rep, scheme, s)
                                                   : hipErrorInvalidValue;
    if (a.st.diss == 2) {  // Godunov's numerical Hamiltonian for normal motion
        switch (a.st.g.dim) {
        case 1: return launch_seed_scheme<T, 1, kHamNormalGodunov>(a, rep, scheme, s);
        case 2: return launch_seed_scheme<T, 2, kHamNormalGodunov>(a, rep, scheme, s);
        case 3: return launch_seed_scheme<T, 3, kHamNormalGodunov>(a, rep, scheme, s);
        case 4: return launch_seed_scheme<T, 4, kHamNormalGodunov>(a, rep, scheme, s);
        }
        return hipErrorInvalidValue;
    }
    switch (a.st.g.dim) {
    case 1: return launch_seed_scheme<T, 1, kHamNormal>(a, rep, scheme, s);
    case 2: return launch_seed_scheme<T, 2, kHamNormal>(a, rep, scheme, s);
    case 3: return launch_seed_scheme<T, 3, kHamNormal>(a, rep, scheme, s);
    case 4: return launch_seed_scheme<T, 4, kHamNormal>(a, rep, scheme, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- per-axis transpose

// LDS of one block: phi at l0-5 .. l0+tl+4, the two seeds at l0-3 .. l0+tl+2
// and the five difference adjoints of each interval l0-3 .. l0+tl+1.
// j modulo n for |j| < 2n (ghost positions at most 5 beyond an axis of
// n >= 3 nodes): two corrections each way, with selects
__device__ __forceinline__ int wrap_near(int j, int n)
{
    j += j < 0 ? n : 0;
    j += j < 0 ? n : 0;
    j -= j >= n ? n : 0;
    j -= j >= n ? n : 0;
    return j;
}

// (position, column) -> LDS index: columns of npos positions when the line
// runs along the lanes (LX), else positions of tw = 2^lw columns
template <bool LX>
__device__ __forceinline__ int lds_at(int pos, int col, int npos, int lw)
{
    return LX ? col * npos + pos : (pos << lw) + col;
}

// One line tile of one axis.  LX: the line axis is the fastest axis and
// runs along the lanes (thread t: position t % tl, column t / tl);
// otherwise the columns run along the lanes (column t % tw, position t / tw).
// Threads t >= tl * tw only take part in the barriers.
// TWC > 0 (off the line axis only): the tile width is that constant, so every
// LDS offset between the accesses of one thread is an immediate.
template <typename T, int SCHEME, bool LX, int TWC>
__device__ __forceinline__ void axis_tile(const AdjAxisArgs<T> &a, int bx, int by, int tid, unsigned char *smem_raw)
{
    static_assert(TWC == 0 || (!LX && (TWC & (TWC - 1)) == 0), "constant tile widths are powers of two off the line axis");
    const int tl = a.tl, tw = TWC > 0 ? TWC : a.tw;
    constexpr bool lx = LX;
    // off the line axis tw is a power of two (the launcher checks): shifts
    // and masks instead of integer division and multiplication
    const int lw = lx ? 0 : __builtin_ctz((unsigned)tw);
    const bool active = tid < tl * tw;
    // along the lanes, t / tl as (t + 1/2) times a one-ulp reciprocal: t < 256
    // and tl <= 64 keep the product within 1e-4 of the exact quotient, whose
    // fraction is at least 1/128 from an integer
    const int qt = lx ? (int)(((float)tid + 0.5f) * __builtin_amdgcn_rcpf((float)tl)) : 0;
    const int ip = active ? (lx ? tid - qt * tl : tid >> lw) : tl;
    const int ic = active ? (lx ? qt : tid & (tw - 1)) : 0;
    const int NP = tl + 10, NS = tl + 6, NI = tl + 5;
    T *PH = reinterpret_cast<T *>(smem_raw);   // NP x tw
    T *SM = PH + NP * tw;                      // NS x tw
    T *SP = SM + NS * tw;                      // NS x tw
    T *UB = SP + NS * tw;                      // NI x 5 x tw

    const int d = a.d, nd = a.g.n[d], sd = a.g.stride[d];
    const bool per = (a.g.periodic >> d) & 1u;
    const int nc = a.c >= 0 ? a.g.n[a.c] : 1, sc = a.c >= 0 ? a.g.stride[a.c] : 0;
    const int tiles_d = a.tiles_d;
    const int ct = udiv(bx, tiles_d, a.m_tiles);
    const int l0 = (bx - ct * tiles_d) * tl, c0 = ct * tw;
    const int col = c0 + ic;
    const bool col_ok = active && col < nc;
    int base = col_ok ? col * sc : 0;
    // the remaining axes: by = r0 n1 + r1 (one of them, or none, may be absent)
    if (a.rest[1] >= 0) {
        const int n1 = a.g.n[a.rest[1]];
        const int r0 = udiv(by, n1, a.m_rest1);
        base += (by - r0 * n1) * a.g.stride[a.rest[1]] + r0 * a.g.stride[a.rest[0]];
    } else if (a.rest[0] >= 0) {
        base += by * a.g.stride[a.rest[0]];
    }

    // stage phi and the seeds of this axis in one pass: thread (ip, ic) takes
    // positions ip, ip + tl, ... of column ic, stepping its offset by tl
    // strides (the line axis along the lanes is the fastest axis: stride 1).
    // Position p holds phi at node l0 - 5 + p and, for 2 <= p < NS + 2, the
    // seeds of that node at seed position p - 2.  A ghost along d wraps on a
    // periodic axis; otherwise phi is extrapolated linearly from the two end
    // nodes and the ghost carries no seed.
    const int sdl = lx ? 1 : sd;
    const int step = tl * sdl;
    if (active) {
        int gpos = l0 - 5 + ip, off = base + gpos * sdl;
        for (int p = ip; p < NP; p += tl, gpos += tl, off += step) {
            const bool seed = (unsigned)(p - 2) < (unsigned)NS;
            T v = T(0), m = T(0), pl = T(0);
            if (col_ok) {
                const bool in = (unsigned)gpos < (unsigned)nd;
                if (in || per) {
                    const int o = in ? off : base + wrap_near(gpos, nd) * sd;
                    v = ld32(a.phi, o);
                    if (seed) {
                        m = ld32(a.seed_m, o);
                        pl = ld32(a.seed_p, o);
                    }
                } else {
                    const int e = gpos < 0 ? 0 : nd - 1, e2 = gpos < 0 ? 1 : nd - 2;
                    const T c = T(gpos < 0 ? -gpos : gpos - (nd - 1));
                    const T p0 = ld32(a.phi, base + e * sd), p1 = ld32(a.phi, base + e2 * sd);
                    v = fmaT(c, p0 - p1, p0);
                }
            }
            PH[lds_at<LX>(p, ic, NP, lw)] = v;
            if (seed) {
                SM[lds_at<LX>(p - 2, ic, NS, lw)] = m;
                SP[lds_at<LX>(p - 2, ic, NS, lw)] = pl;
            }
        }
    }
    __syncthreads();

    // transpose every interval I = l0-3+iv once: the NI x tw (interval,
    // column) pairs are spread over all the block's threads (the host sizes
    // tiles so that there are at most as many pairs as threads), consecutive
    // lanes taking consecutive intervals of a line (lx) or consecutive
    // columns (otherwise), as the LDS layout is laid out
    const float inv_ni = __builtin_amdgcn_rcpf((float)NI);  // e < 256, NI <= 69: as above
    for (int e = tid; e < NI * tw; e += kAxisThreads) {  // every thread of the block takes part
        int iv, cc;
        if (lx) {
            cc = (int)(((float)e + 0.5f) * inv_ni);
            iv = e - cc * NI;
        } else {
            cc = e & (tw - 1);
            iv = e >> lw;
        }
        T ub[5] = {T(0), T(0), T(0), T(0), T(0)};
        if (c0 + cc < nc) {
            T v[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) v[k] = PH[lds_at<LX>(iv + k, cc, NP, lw)];
            const T gm = SM[lds_at<LX>(iv + 1, cc, NS, lw)];  // left-biased seed of node I+1
            const T gp = SP[lds_at<LX>(iv, cc, NS, lw)];      // right-biased seed of node I
            interval_vjp<T, SCHEME>(v, a.inv_dx, a.dx, gm, gp, ub);
        }
#pragma unroll
        for (int r = 0; r < 5; ++r) UB[lds_at<LX>(iv * 5 + r, cc, NI * 5, lw)] = ub[r];
    }
    __syncthreads();

    // the two half-nodes of a node of this tile, m = g - 1 and g, read the
    // intervals ip .. ip + 5, all inside the tile: no bounds checks.  Half-node
    // g - 1 + o (o = 0, 1) takes difference r of interval ip + 4 + o - r, at
    // position 5 ip + 20 + 5 o - 4 r: one base per thread, constant offsets.
    const T *ub_node = UB + lds_at<LX>(5 * ip, ic, NI * 5, lw);
    auto ubar_in = [&](int o) -> T {
        T s = T(0);
#pragma unroll
        for (int r = 0; r < 5; ++r) s += ub_node[lx ? 20 + 5 * o - 4 * r : (20 + 5 * o - 4 * r) << lw];
        return s;
    };
    const int g = l0 + ip;
    if (ip < tl && g < nd && col_ok) {
        T uL = ubar_in(0), uR = ubar_in(1);   // adjoints of the differences left and right of g
        if (!per && (g <= 1 || g >= nd - 2)) {
            // Linear extrapolation makes every ghost difference beyond an end
            // the end difference itself (half-node 0, or nd - 2), as a
            // function of the nodes: the adjoints of the ghost differences
            // fold onto that half-node.  They sit in six slots at each end:
            // differences r of intervals -1 (r = 0..2), 0 (r = 0, 1) and 1
            // (r = 0) on the left, nd - 3 (r = 4), nd - 2 (r = 3, 4) and nd - 1
            // (r = 2..4) on the right; intervals further out carry no seeds.
            // A node within two of an end lies in the first tile (l0 = 0) or
            // sees intervals nd - 3 .. nd - 1 in its own tile.
            const T *ub_col = UB + lds_at<LX>(0, ic, NI * 5, lw);
            auto slot = [&](int iv, int r) -> T { return ub_col[lx ? iv * 5 + r : (iv * 5 + r) << lw]; };
            T eL = T(0), eR = T(0);
            if (g <= 1) eL = ((slot(2, 0) + slot(2, 1)) + (slot(2, 2) + slot(3, 0))) + (slot(3, 1) + slot(4, 0));
            if (g >= nd - 2) {
                const int j = nd - l0;   // interval nd - 3 of the tile
                eR = ((slot(j, 4) + slot(j + 1, 3)) + (slot(j + 1, 4) + slot(j + 2, 2))) +
                     (slot(j + 2, 3) + slot(j + 2, 4));
            }
            uL = ((g == 0 ? T(0) : uL) + (g == 1 ? eL : T(0))) + (g == nd - 1 ? eR : T(0));
            uR = ((g == nd - 1 ? T(0) : uR) + (g == 0 ? eL : T(0))) + (g == nd - 2 ? eR : T(0));
        }
        const T acc = (uL - uR) * a.inv_dx;
        if (a.out) at32(a.out, base + g * sd) = acc;
        else at32(a.lam, base + g * sd) += acc;
    }
}

// The transposes of every axis in one launch: block b belongs to the axis k
// with start[k] <= b < start[k+1] and is tile (bx, by) of that axis.  With
// several axes each writes its own contribution array (out), so the blocks of
// different axes never touch the same memory and overlap freely.
template <typename T, int SCHEME>
__global__ __launch_bounds__(kAxisThreads) void adj_axes_kernel(AdjAxesArgs<T> a)
{
    extern __shared__ unsigned char smem_raw[];
    const int b = (int)blockIdx.x;
    int k = 0;
    while (k + 1 < a.nax && b >= a.start[k + 1]) ++k;
    const int lb = b - a.start[k];
    const int by = udiv(lb, a.gx[k], a.m_gx[k]), bx = lb - by * a.gx[k];
    const AdjAxisArgs<T> &A = a.ax[k];
    if (A.d == A.g.dim - 1) axis_tile<T, SCHEME, true, 0>(A, bx, by, (int)threadIdx.x, smem_raw);
    else if (A.tw == 8) axis_tile<T, SCHEME, false, 8>(A, bx, by, (int)threadIdx.x, smem_raw);
    else axis_tile<T, SCHEME, false, 0>(A, bx, by, (int)threadIdx.x, smem_raw);
}

// lam += c[0] (+ c[1]) (+ c[2]) (+ c[3]), added in that order
template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(T *lam, AdjCombineArgs<T> c, int n)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        T v = ld32(lam, i);
        for (int k = 0; k < c.n; ++k) v += ld32(c.c[k], i);
        at32(lam, i) = v;
    }
}

template <typename T>
hipError_t launch_axes(const AdjAxesArgs<T> &in, int scheme, hipStream_t s)
{
    AdjAxesArgs<T> a = in;
    if (a.nax < 1 || a.nax > kMaxDim) return hipErrorInvalidValue;
    size_t lds = 0;
    long total = 0;
    for (int k = 0; k < a.nax; ++k) {
        const AdjAxisArgs<T> &x = a.ax[k];
        const int nd = x.g.n[x.d], nc = x.c >= 0 ? x.g.n[x.c] : 1;
        if (x.tl < 2 || x.tw < 1 || (x.tl + 5) * x.tw > kAxisThreads) return hipErrorInvalidConfiguration;
        if (x.d != x.g.dim - 1 && (x.tw & (x.tw - 1))) return hipErrorInvalidConfiguration;
        int rest = 1;
        for (int r = 0; r < 2; ++r)
            if (x.rest[r] >= 0) rest *= x.g.n[x.rest[r]];
        a.ax[k].tiles_d = (nd + x.tl - 1) / x.tl;
        a.gx[k] = a.ax[k].tiles_d * ((nc + x.tw - 1) / x.tw);
        a.start[k] = (int)total;
        total += (long)a.gx[k] * rest;
        a.m_gx[k] = fast_div_multiplier(a.gx[k], (long)a.gx[k] * rest);
        a.ax[k].m_tiles = fast_div_multiplier(a.ax[k].tiles_d, a.gx[k]);
        a.ax[k].m_rest1 = x.rest[1] >= 0 ? fast_div_multiplier(x.g.n[x.rest[1]], rest) : 0;
        lds = std::max(lds, sizeof(T) * (size_t)x.tw * ((x.tl + 10) + 2 * (x.tl + 6) + 5 * (x.tl + 5)));
    }
    if (total > 0x7fffffffL) return hipErrorInvalidConfiguration;
    a.start[a.nax] = (int)total;
    const dim3 grid((unsigned)total);
    switch (scheme) {
    case kSchemeFirst: hipLaunchKernelGGL((adj_axes_kernel<T, kSchemeFirst>), grid, dim3(kAxisThreads), lds, s, a); break;
    case kSchemeEno2: hipLaunchKernelGGL((adj_axes_kernel<T, kSchemeEno2>), grid, dim3(kAxisThreads), lds, s, a); break;
    case kSchemeEno3: hipLaunchKernelGGL((adj_axes_kernel<T, kSchemeEno3>), grid, dim3(kAxisThreads), lds, s, a); break;
    case kSchemeWeno5: hipLaunchKernelGGL((adj_axes_kernel<T, kSchemeWeno5>), grid, dim3(kAxisThreads), lds, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- helpers

__global__ __launch_bounds__(256) void acc_reduce_kernel(const double *acc, int blocks, double *out)
{
    // one block: thread t sums slot t % kAccCount over a strided subset of blocks
    __shared__ double red[256];
    const int k = threadIdx.x % kAccCount, lane = threadIdx.x / kAccCount, lanes = 256 / kAccCount;
    double s = 0.0;
    for (int b = lane; b < blocks; b += lanes) s += acc[b * kAccCount + k];
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < kAccCount) {
        double t = 0.0;
        for (int l = 0; l < lanes; ++l) t += red[l * kAccCount + threadIdx.x];
        out[threadIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T *x, int n)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) x[i] = T(0);
}

int zero_blocks(int n)
{
    const int b = (n + 255) / 256;
    return b < 4096 ? (b > 0 ? b : 1) : 4096;
}

// smoothed volume: partial[b] = sum over this block's nodes of s(-phi/eps);
// grad = d(vol * sum)/dphi
template <typename T>
__global__ __launch_bounds__(256) void loss_kernel(const T *phi, int n, double inv_eps, double vol, T *grad,
                                                   double *partial)
{
    double acc = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double z = -(double)phi[i] * inv_eps;
        const double sg = 1.0 / (1.0 + exp(-z));
        acc += sg;
        if (grad) grad[i] = T(-vol * inv_eps * sg * (1.0 - sg));
    }
    __shared__ double red[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void sum_kernel(const double *partial, int n, double scale, double *out)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = scale * (red[0] + red[1] + red[2] + red[3]);
}

template <typename T>
hipError_t launch_loss(const T *phi, int n, double eps, double vol, T *grad, double *partial, int blocks,
                       double *out, hipStream_t s)
{
    hipLaunchKernelGGL(loss_kernel<T>, dim3(blocks), dim3(256), 0, s, phi, n, 1.0 / eps, vol, grad, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, partial, blocks, vol, out);
    return hipGetLastError();
}

}  // namespace

// accumulator slots: one per seed block of one plane, the most any variant
// uses (slots a variant leaves unwritten stay zero)
int adj_seed_blocks(const GridGeom &g) { return ((g.plane + kSeedThreads - 1) / kSeedThreads) * g.slow; }

hipError_t launch_adj_seed_f32(const AdjSeedArgs<float> &a, const StageArgs<float> *rep, int scheme, int ham,
                               hipStream_t s)
{
    return launch_seed<float>(a, rep, scheme, ham, s);
}
hipError_t launch_adj_seed_f64(const AdjSeedArgs<double> &a, const StageArgs<double> *rep, int scheme, int ham,
                               hipStream_t s)
{
    return launch_seed<double>(a, rep, scheme, ham, s);
}
hipError_t launch_adj_axes_f32(const AdjAxesArgs<float> &a, int scheme, hipStream_t s)
{
    return launch_axes<float>(a, scheme, s);
}
hipError_t launch_adj_axes_f64(const AdjAxesArgs<double> &a, int scheme, hipStream_t s)
{
    return launch_axes<double>(a, scheme, s);
}
hipError_t launch_combine_f32(float *lam, const AdjCombineArgs<float> &c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(combine_kernel<float>, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, lam, c, n);
    return hipGetLastError();
}
hipError_t launch_combine_f64(double *lam, const AdjCombineArgs<double> &c, int n, hipStream_t s)
{
    hipLaunchKernelGGL(combine_kernel<double>, dim3(std::min((n + 255) / 256, 4096)), dim3(256), 0, s, lam, c, n);
    return hipGetLastError();
}
hipError_t launch_acc_reduce(const double *acc, int blocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(acc_reduce_kernel, dim3(1), dim3(256), 0, s, acc, blocks, out);
    return hipGetLastError();
}
hipError_t launch_zero_f32(float *x, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel<float>, dim3(zero_blocks(n)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}
hipError_t launch_zero_f64(double *x, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel<double>, dim3(zero_blocks(n)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}
hipError_t launch_zero_f64acc(double *x, int n, hipStream_t s) { return launch_zero_f64(x, n, s); }
hipError_t launch_loss_f32(const float *phi, int n, double eps, double vol, float *grad, double *partial, int blocks,
                           double *out, hipStream_t s)
{
    return launch_loss<float>(phi, n, eps, vol, grad, partial, blocks, out, s);
}
hipError_t launch_loss_f64(const double *phi, int n, double eps, double vol, double *grad, double *partial,
                           int blocks, double *out, hipStream_t s)
{
    return launch_loss<double>(phi, n, eps, vol, grad, partial, blocks, out, s);
}

}  // namespace hjx
