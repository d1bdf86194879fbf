// C ABI of libhjx (include/hjx.h): argument validation, per-axis tables,
// workspace ownership and the explicit time loop (LevelSetPy, arXiv
// 2411.03501, Sec. V: odeCFL1/2/3 with the CFL step of Sec. IV-D).
#include "../../include/hjx.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "hjx_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

using namespace hjx;

namespace {

thread_local std::string g_last_error;

hjx_status fail(hjx_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

hjx_status ok()
{
    g_last_error.clear();
    return HJX_OK;
}

#define HIP_TRY(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? HJX_ERR_OOM : HJX_ERR_DEVICE, "%s: %s (%s)", \
                        #call, hipGetErrorString(e_), __func__);                              \
    } while (0)

// Optional cap on the device workspace one create call may allocate
// (environment variable HJX_MAX_WORKSPACE, bytes; read at every call), for
// exercising the out-of-memory paths without exhausting the device.
bool over_workspace_cap(size_t bytes, size_t *cap_out)
{
    const char *v = std::getenv("HJX_MAX_WORKSPACE");
    if (!v || !*v) return false;
    char *end = nullptr;
    const unsigned long long cap = std::strtoull(v, &end, 10);
    if (end == v) return false;
    *cap_out = (size_t)cap;
    return bytes > (size_t)cap;
}

// roctx ranges around the library's calls (and the segments of a reverse
// sweep) when the environment variable HJX_TRACE is set to anything but 0;
// rocprofv3 --marker-trace shows them beside the kernels.
bool trace_on()
{
    const char *v = std::getenv("HJX_TRACE");
    return v && *v && !(v[0] == '0' && v[1] == 0);
}

struct TraceRange {
    bool on;
    explicit TraceRange(const char *name) : on(trace_on())
    {
        if (on) roctxRangePushA(name);
    }
    TraceRange(const char *fmt, long a) : on(trace_on())
    {
        if (on) {
            char buf[96];
            std::snprintf(buf, sizeof buf, fmt, a);
            roctxRangePushA(buf);
        }
    }
    ~TraceRange()
    {
        if (on) roctxRangePop();
    }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

int n_params(int kind)
{
    switch (kind) {
    case HJX_HAM_NORMAL: return 1;
    case HJX_HAM_DUBINS3_PE: return 4;
    case HJX_HAM_DUBINS4: return 2;
    case HJX_HAM_ROCKETS: return 4;
    }
    return 0;
}

}  // namespace

struct hjx_problem {
    hjx_grid_desc grid;
    hjx_ham_desc ham;
    hjx_scheme_desc scheme;
    int device = 0;
    int64_t total = 0;
    double dx[kMaxDim] = {0, 0, 0, 0};
    size_t elem = 0;           // bytes per value
    void *tables = nullptr;    // device: per axis coord, cos, sin (elem bytes each)
    size_t table_off[kMaxDim][3] = {};
    void *ws[2] = {nullptr, nullptr};
    double *dalpha = nullptr;  // device: alpha[kMaxDim] + reduction partials
    int *dflag = nullptr;      // device: non-finite flags (input, output)
    double *hbuf = nullptr;    // pinned host: alpha[kMaxDim], flags
    hipEvent_t ev[2] = {nullptr, nullptr};
    Tile tile{};               // stage-kernel launch shape
    // alpha depends only on the grid tables and the parameters, both fixed
    // at create: reduced on the device once, then kept
    bool alpha_known = false;
    double alpha[kMaxDim] = {0, 0, 0, 0};
    // the stepping launches of hjx_solve, captured when the same solve
    // (arrays, times) is asked for a second time in a row, then replayed
    struct SolveKey {
        const void *phi0 = nullptr, *target = nullptr;
        void *out = nullptr;
        double t0 = 0.0, t1 = 0.0;
        bool operator==(const SolveKey &o) const
        {
            return phi0 == o.phi0 && target == o.target && out == o.out && t0 == o.t0 && t1 == o.t1;
        }
    };
    SolveKey last_key{};
    bool have_key = false;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

GridGeom geometry(const hjx_problem *p)
{
    GridGeom g{};
    g.dim = p->grid.dim;
    int s = 1;
    for (int d = g.dim - 1; d >= 0; --d) {
        g.n[d] = (int)p->grid.n[d];
        g.stride[d] = s;
        s *= g.n[d];
    }
    for (int d = g.dim; d < kMaxDim; ++d) {
        g.n[d] = 1;
        g.stride[d] = 0;
    }
    g.periodic = p->grid.periodic_mask;
    if (g.dim == 1) {
        g.plane = g.n[0];
        g.slow = 1;
    } else {
        g.plane = g.n[g.dim - 2] * g.n[g.dim - 1];
        g.slow = 1;
        for (int d = 0; d < g.dim - 2; ++d) g.slow *= g.n[d];
    }
    return g;
}

template <typename T>
AxisTables<T> tables(const hjx_problem *p)
{
    AxisTables<T> t{};
    const char *base = static_cast<const char *>(p->tables);
    for (int d = 0; d < p->grid.dim; ++d) {
        t.coord[d] = reinterpret_cast<const T *>(base + p->table_off[d][0]);
        t.cosv[d] = reinterpret_cast<const T *>(base + p->table_off[d][1]);
        t.sinv[d] = reinterpret_cast<const T *>(base + p->table_off[d][2]);
    }
    return t;
}

hjx_status validate_grid(const hjx_grid_desc *g)
{
    if (g->dim < 1 || g->dim > HJX_MAX_DIM)
        return fail(HJX_ERR_INVALID_ARG, "grid dim %d outside [1, %d]", g->dim, HJX_MAX_DIM);
    if (g->periodic_mask >> g->dim)
        return fail(HJX_ERR_INVALID_ARG, "periodic_mask 0x%x names an axis >= dim %d", g->periodic_mask, g->dim);
    int64_t total = 1;
    for (int d = 0; d < g->dim; ++d) {
        if (g->n[d] < 3) return fail(HJX_ERR_INVALID_ARG, "n[%d] = %lld < 3", d, (long long)g->n[d]);
        if (!std::isfinite(g->gmin[d]) || !std::isfinite(g->gmax[d]) || !(g->gmax[d] > g->gmin[d]))
            return fail(HJX_ERR_INVALID_ARG, "axis %d extent [%g, %g] is not a finite increasing interval", d,
                        g->gmin[d], g->gmax[d]);
        total *= g->n[d];
        if (total >= (int64_t(1) << 31))
            return fail(HJX_ERR_INVALID_ARG, "grid has 2^31 nodes or more");
    }
    return HJX_OK;
}

hjx_status validate(const hjx_grid_desc *g, const hjx_ham_desc *h, const hjx_scheme_desc *s)
{
    if (!g || !h || !s) return fail(HJX_ERR_INVALID_ARG, "NULL descriptor");
    hjx_status gst = validate_grid(g);
    if (gst != HJX_OK) return gst;
    const int np = n_params(h->kind);
    if (np == 0) return fail(HJX_ERR_INVALID_ARG, "unknown Hamiltonian kind %d", h->kind);
    if (h->dissipation != HJX_DISS_GLOBAL && h->dissipation != HJX_DISS_LOCAL && h->dissipation != HJX_DISS_GODUNOV)
        return fail(HJX_ERR_INVALID_ARG, "unknown dissipation %d", h->dissipation);
    if (h->dissipation == HJX_DISS_GODUNOV && h->kind != HJX_HAM_NORMAL)
        return fail(HJX_ERR_INVALID_ARG, "the Godunov Hamiltonian is built for NORMAL only");
    for (int k = 0; k < np; ++k)
        if (!std::isfinite(h->p[k])) return fail(HJX_ERR_INVALID_ARG, "Hamiltonian parameter %d is not finite", k);
    if (h->kind == HJX_HAM_DUBINS3_PE) {
        if (g->dim != 3) return fail(HJX_ERR_INVALID_ARG, "DUBINS3_PE needs dim 3, got %d", g->dim);
        if (h->p[2] < 0 || h->p[3] < 0) return fail(HJX_ERR_INVALID_ARG, "turn-rate bounds must be >= 0");
    }
    if (h->kind == HJX_HAM_DUBINS4) {
        if (g->dim != 4) return fail(HJX_ERR_INVALID_ARG, "DUBINS4 needs dim 4, got %d", g->dim);
        if (h->p[0] < 0 || h->p[1] < 0) return fail(HJX_ERR_INVALID_ARG, "control bounds must be >= 0");
    }
    if (h->kind == HJX_HAM_ROCKETS) {
        if (g->dim != 3) return fail(HJX_ERR_INVALID_ARG, "ROCKETS needs dim 3, got %d", g->dim);
        if (h->p[2] < 0 || h->p[3] < 0) return fail(HJX_ERR_INVALID_ARG, "control bounds must be >= 0");
    }
    if (s->deriv != HJX_DERIV_FIRST && s->deriv != HJX_DERIV_ENO2 && s->deriv != HJX_DERIV_ENO3 &&
        s->deriv != HJX_DERIV_WENO5)
        return fail(HJX_ERR_INVALID_ARG, "unknown derivative scheme %d", s->deriv);
    if (s->rk < 1 || s->rk > 3) return fail(HJX_ERR_INVALID_ARG, "rk order %d outside [1, 3]", s->rk);
    if (!(s->cfl > 0.0) || !(s->cfl <= 1.0)) return fail(HJX_ERR_INVALID_ARG, "cfl %g outside (0, 1]", s->cfl);
    if (s->dtype != HJX_F32 && s->dtype != HJX_F64) return fail(HJX_ERR_INVALID_ARG, "unknown dtype %d", s->dtype);
    if (s->restrict_update < HJX_RESTRICT_NONE || s->restrict_update > HJX_RESTRICT_POSITIVE)
        return fail(HJX_ERR_INVALID_ARG, "unknown restrict_update %d", s->restrict_update);
    return HJX_OK;
}

// ---------------------------------------------------------------- launches

// Default launch shape, from autotuner sweeps on MI355X: small grids (a few
// million nodes) do best with near-square plane tiles of ~256 threads and a
// march of 2 (many waves in flight); large grids with whole rows of the
// fastest axis (up to 128 nodes) and a march of 8 (fewer halo re-reads).
// hjx_tune refines the choice per problem.
// the direct variant addresses arrays through 32-bit byte offsets
bool direct_ok(const GridGeom &g, size_t elem)
{
    uint64_t total = 1;
    for (int d = 0; d < g.dim; ++d) total *= (uint64_t)g.n[d];
    return total * elem < (uint64_t(1) << 32);
}

// nodes one plane-march block may hold: 512 in 3-D and 4-D (the tile kernel,
// 512 threads, one node each), 256 in 1-D and 2-D (a thread per node)
int tile_max_nodes(const GridGeom &g) { return g.dim >= 3 ? 512 : 256; }

// In 3-D and 4-D the tile kernel addresses a plane of the two fastest axes
// through 32-bit offsets; in 1-D and 2-D every kernel addresses the whole
// array so.
bool tile_ok(const GridGeom &g, size_t elem)
{
    if (g.dim <= 2) return direct_ok(g, elem);
    const uint64_t planes = g.dim == 4 ? 7 : 1;  // 4-D: the seven planes of the gathered axis' stencil
    return planes * (uint64_t)g.n[g.dim - 1] * (uint64_t)g.n[g.dim - 2] * elem < (uint64_t(1) << 32);
}

// The steps variant's shape check: a 1-D or 2-D grid under 4 GiB, k = march
// whole steps with a halo H = k * rk * radius no deeper than a periodic axis,
// at most 2^20 values per LDS buffer and kStepsLdsMax bytes of LDS.  *area
// receives the values per buffer.
bool steps_shape(const GridGeom &g, size_t elem, int deriv, int rk, const Tile &t, long *area)
{
    if (g.dim > 2 || !direct_ok(g, elem) || t.tx < 1 || t.ty < 1 || t.march < 1 || (g.dim == 1 && t.ty != 1))
        return false;
    const int nx = g.n[g.dim - 1], ny = g.dim == 2 ? g.n[0] : 1;
    const bool perx = (g.periodic >> (g.dim - 1)) & 1u, pery = g.dim == 2 && (g.periodic & 1u);
    const long H = (long)t.march * rk * scheme_radius(deriv);
    if ((perx && H > nx) || (pery && H > ny)) return false;
    const long a = steps_area(t.tx, t.ty, H, nx, ny, perx, pery, g.dim == 2);
    if (a >= (1l << 20) || (size_t)steps_buffers(rk) * (size_t)a * elem > kStepsLdsMax) return false;
    if (area) *area = a;
    return true;
}

Tile default_tile(const GridGeom &g, size_t elem, int deriv, int rk)
{
    // small 1-D and 2-D grids: a few whole steps per launch (8 x 8 tiles,
    // about four stage radii of halo; the fastest shape the tuner finds for
    // the 101^2 first-order case, 1.5 us per step against 2.3 us with 16 x 16)
    long nodes = 1;
    for (int d = 0; d < g.dim; ++d) nodes *= g.n[d];
    if (g.dim <= 2 && nodes <= (1l << 16)) {
        const Tile st{g.dim == 1 ? 256 : 8, g.dim == 1 ? 1 : 8, std::max(1, 4 / (rk * scheme_radius(deriv))),
                      kVariantSteps};
        if (steps_shape(g, elem, deriv, rk, st, nullptr)) return st;
    }
    Tile t{};
    const int nf = g.n[g.dim - 1];
    const int nm = g.dim >= 2 ? g.n[g.dim - 2] : 1;
    long total = 1;
    for (int d = 0; d < g.dim; ++d) total *= g.n[d];
    const bool large = total >= (8l << 20);
    t.variant = large || !direct_ok(g, elem) ? kVariantPlaneMarch : kVariantDirect;
    const int width = large ? 128 : 16;
    const int pieces = (nf + width - 1) / width;
    const int maxn = tile_max_nodes(g);
    t.tx = std::min((nf + pieces - 1) / pieces, 256);
    t.ty = g.dim >= 2 ? std::max(1, std::min(maxn / t.tx, nm)) : 1;
    t.march = 1;
    if (g.dim >= 3) {  // the tile kernel marches axis 0: chunks of about 8 (large) or 2 planes, evenly
        const int want = large ? 8 : 2, chunks = std::max(1, (g.n[0] + want / 2) / want);
        t.march = (g.n[0] + chunks - 1) / chunks;
    }
    return t;
}

template <typename T>
StageArgs<T> stage_args(const hjx_problem *p, const double *alpha)
{
    StageArgs<T> a{};
    a.g = geometry(p);
    a.tile = p->tile;
    a.tab = tables<T>(p);
    for (int d = 0; d < kMaxDim; ++d) {
        a.inv_dx[d] = d < p->grid.dim ? T(1.0 / p->dx[d]) : T(0);
        a.dx[d] = d < p->grid.dim ? T(p->dx[d]) : T(0);
        a.alpha[d] = d < p->grid.dim ? T(alpha[d]) : T(0);
    }
    for (int k = 0; k < 8; ++k) a.hp[k] = T(p->ham.p[k]);
    a.diss = p->ham.dissipation;
    a.clip = p->scheme.restrict_update == HJX_RESTRICT_NONPOSITIVE ? -1
             : p->scheme.restrict_update == HJX_RESTRICT_POSITIVE  ? 1
                                                                   : 0;
    return a;
}

hipError_t launch_stage(const hjx_problem *p, const double *alpha, const void *in, const void *phin,
                        const void *target, void *out, double dt, double ca, double cb, bool rhs_only,
                        hipStream_t s)
{
    if (p->scheme.dtype == HJX_F32) {
        StageArgs<float> a = stage_args<float>(p, alpha);
        a.phi_in = static_cast<const float *>(in);
        a.phi_n = static_cast<const float *>(phin);
        a.target = static_cast<const float *>(target);
        a.out = static_cast<float *>(out);
        a.dt = float(dt);
        a.ca = float(ca);
        a.cb = float(cb);
        a.rhs_only = rhs_only;
        return launch_stage_f32(a, p->scheme.deriv, p->ham.kind, s);
    }
    StageArgs<double> a = stage_args<double>(p, alpha);
    a.phi_in = static_cast<const double *>(in);
    a.phi_n = static_cast<const double *>(phin);
    a.target = static_cast<const double *>(target);
    a.out = static_cast<double *>(out);
    a.dt = dt;
    a.ca = ca;
    a.cb = cb;
    a.rhs_only = rhs_only;
    return launch_stage_f64(a, p->scheme.deriv, p->ham.kind, s);
}

// k whole RK steps of the steps variant from in into out (different arrays),
// each of size dt but the last, of dt_last; the target after every step.
hipError_t launch_steps(const hjx_problem *p, const double *alpha, const void *in, const void *target, void *out,
                        int k, double dt, double dt_last, hipStream_t s, int *flag_in, int *flag_out)
{
    const GridGeom g = geometry(p);
    long area = 0;
    if (!steps_shape(g, p->elem, p->scheme.deriv, p->scheme.rk, p->tile, &area)) return hipErrorInvalidConfiguration;
    StepsLaunch l{};
    l.k = k;
    l.rk = p->scheme.rk;
    l.dt = dt;
    l.dt_last = dt_last;
    l.tx = p->tile.tx;
    l.ty = p->tile.ty;
    l.tiles_x = (g.n[g.dim - 1] + l.tx - 1) / l.tx;
    l.area_max = (int)area;
    l.flag_in = flag_in;
    l.flag_out = flag_out;
    // (area is for the tile's own number of steps; a launch of fewer has a
    // shallower halo and fits in it)
    if (p->scheme.dtype == HJX_F32) {
        StageArgs<float> a = stage_args<float>(p, alpha);
        a.phi_in = static_cast<const float *>(in);
        a.target = static_cast<const float *>(target);
        a.out = static_cast<float *>(out);
        return launch_steps_f32(a, l, p->scheme.deriv, p->ham.kind, s);
    }
    StageArgs<double> a = stage_args<double>(p, alpha);
    a.phi_in = static_cast<const double *>(in);
    a.target = static_cast<const double *>(target);
    a.out = static_cast<double *>(out);
    return launch_steps_f64(a, l, p->scheme.deriv, p->ham.kind, s);
}

hipError_t launch_copy(const hjx_problem *p, const void *src, void *dst, hipStream_t s)
{
    if (p->scheme.dtype == HJX_F32)
        return launch_copy_f32(static_cast<const float *>(src), static_cast<float *>(dst), (int)p->total, s);
    return launch_copy_f64(static_cast<const double *>(src), static_cast<double *>(dst), (int)p->total, s);
}

// One RK step of size dt: phi (in place) with the problem workspace.
hipError_t rk_step(const hjx_problem *p, const double *alpha, void *phi, const void *target, double dt,
                   hipStream_t s)
{
    hipError_t e;
    void *a = p->ws[0], *b = p->ws[1];
    switch (p->scheme.rk) {
    case 1:  // odeCFL1: phi + dt L(phi)
        if ((e = launch_stage(p, alpha, phi, nullptr, target, a, dt, 0.0, 1.0, false, s)) != hipSuccess) return e;
        return launch_copy(p, a, phi, s);
    case 2:  // odeCFL2: two Euler moves, then the average with phi^n
        if ((e = launch_stage(p, alpha, phi, nullptr, nullptr, a, dt, 0.0, 1.0, false, s)) != hipSuccess) return e;
        return launch_stage(p, alpha, a, phi, target, phi, dt, 0.5, 0.5, false, s);
    default:  // odeCFL3: Shu-Osher stages with averages 3/4, 1/4 and 1/3, 2/3
        if ((e = launch_stage(p, alpha, phi, nullptr, nullptr, a, dt, 0.0, 1.0, false, s)) != hipSuccess) return e;
        if ((e = launch_stage(p, alpha, a, phi, nullptr, b, dt, 0.75, 0.25, false, s)) != hipSuccess) return e;
        return launch_stage(p, alpha, b, phi, target, phi, dt, 1.0 / 3.0, 2.0 / 3.0, false, s);
    }
}

// alpha_d, the grid maximum of the partial bound: reduced on the device the
// first time (synchronises s), kept on the host afterwards.
hjx_status device_alpha(hjx_problem *p, hipStream_t s, double *alpha_host)
{
    if (p->alpha_known) {
        for (int d = 0; d < kMaxDim; ++d) alpha_host[d] = p->alpha[d];
        return HJX_OK;
    }
    hipError_t e;
    if (p->scheme.dtype == HJX_F32) {
        AlphaArgs<float> a{};
        a.g = geometry(p);
        a.tab = tables<float>(p);
        for (int k = 0; k < 8; ++k) a.hp[k] = float(p->ham.p[k]);
        a.ham = p->ham.kind;
        a.partial = p->dalpha + kMaxDim;
        a.total = (int)p->total;
        e = launch_alpha_f32(a, p->dalpha, s);
    } else {
        AlphaArgs<double> a{};
        a.g = geometry(p);
        a.tab = tables<double>(p);
        for (int k = 0; k < 8; ++k) a.hp[k] = p->ham.p[k];
        a.ham = p->ham.kind;
        a.partial = p->dalpha + kMaxDim;
        a.total = (int)p->total;
        e = launch_alpha_f64(a, p->dalpha, s);
    }
    HIP_TRY(e);
    HIP_TRY(hipMemcpyAsync(p->hbuf, p->dalpha, sizeof(double) * kMaxDim, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int d = 0; d < kMaxDim; ++d) p->alpha[d] = alpha_host[d] = d < p->grid.dim ? p->hbuf[d] : 0.0;
    p->alpha_known = true;
    return HJX_OK;
}

double cfl_dt(const hjx_problem *p, const double *alpha)
{
    double rate = 0.0;
    for (int d = 0; d < p->grid.dim; ++d) rate += alpha[d] / p->dx[d];
    if (!(rate > 0.0)) return INFINITY;
    return p->scheme.cfl / rate;
}

// any NaN/Inf in x?  synchronises s.
hjx_status any_nonfinite(hjx_problem *p, const void *x, hipStream_t s, bool *bad)
{
    HIP_TRY(hipMemsetAsync(p->dflag, 0, sizeof(int), s));
    if (p->scheme.dtype == HJX_F32)
        HIP_TRY(launch_nonfinite_f32(static_cast<const float *>(x), (int)p->total, p->dflag, s));
    else
        HIP_TRY(launch_nonfinite_f64(static_cast<const double *>(x), (int)p->total, p->dflag, s));
    int *hflag = reinterpret_cast<int *>(p->hbuf + kMaxDim);
    HIP_TRY(hipMemcpyAsync(hflag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *bad = *hflag != 0;
    return HJX_OK;
}

// launch the non-finite check of x into the flag word flag (0 = input,
// 1 = output); the flags must have been cleared on the same stream
hipError_t check_nonfinite(hjx_problem *p, const void *x, int flag, hipStream_t s)
{
    if (p->scheme.dtype == HJX_F32)
        return launch_nonfinite_f32(static_cast<const float *>(x), (int)p->total, p->dflag + flag, s);
    return launch_nonfinite_f64(static_cast<const double *>(x), (int)p->total, p->dflag + flag, s);
}

void drop_solve_graph(hjx_problem *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->have_key = false;
}

// The number of steps of a solve from t0 to t1 with CFL step dt and the
// size of the last one: steps of dt while they stay short of t1, the one
// that would reach t1 (or come within 1e-12 max(1, |t1|) of it) clamped to
// land on t1.
void schedule(double t0, double t1, double dt, int64_t *steps, double *dt_last)
{
    const double slack = 1e-12 * (std::fabs(t1) > 1.0 ? std::fabs(t1) : 1.0);
    double t = t0, h_last = 0.0;
    int64_t n = 0;
    while (t < t1) {
        double h = dt;
        bool last = false;
        if (t + h >= t1 - slack) {
            h = t1 - t;
            last = true;
        }
        ++n;
        h_last = h;
        t = last ? t1 : t + h;
    }
    *steps = n;
    *dt_last = h_last;
}

// The stepping launches of a solve: `steps` RK steps from phi0 into
// phi_out, the last of size dt_last, the others dt.  No copy of phi0: the
// first step reads it where it is.  Forward Euler alternates between
// phi_out and the workspace so that the last step lands in phi_out; the
// RK2/RK3 stages of the first step take phi0 as phi^n and write their last
// stage into phi_out, which later steps advance in place.
hipError_t enqueue_steps(const hjx_problem *p, const double *alpha, const void *phi0, const void *target,
                         void *phi_out, int64_t steps, double dt, double dt_last, hipStream_t s, int *flags)
{
    hipError_t e = hipSuccess;
    if (steps == 0) return phi_out == phi0 ? hipSuccess : launch_copy(p, phi0, phi_out, s);
    if (p->tile.variant == kVariantSteps) {
        // k steps per launch; launches alternate between the two workspaces
        // and the last lands in phi_out (through ws[0] and a copy when a
        // single launch would read and write phi_out).  With flags, the first
        // launch checks phi0 into flags[0] and the last its result into
        // flags[1] (the non-finite checks of hjx_solve).
        const int k = p->tile.march;
        const int64_t launches = (steps + k - 1) / k;
        const void *src = phi0;
        for (int64_t i = 0; i < launches && e == hipSuccess; ++i) {
            const bool final = i + 1 == launches;
            const int ki = (int)std::min<int64_t>(k, steps - i * k);
            void *dst = final ? phi_out : p->ws[i & 1];
            if (dst == src) dst = p->ws[0];
            e = launch_steps(p, alpha, src, target, dst, ki, dt, final ? dt_last : dt, s,
                             flags && i == 0 ? flags : nullptr, flags && final ? flags + 1 : nullptr);
            if (e == hipSuccess && final && dst != phi_out) e = launch_copy(p, dst, phi_out, s);
            src = dst;
        }
        return e;
    }
    if (p->scheme.rk == 1) {
        if (phi_out == phi0) {  // in place: each step through the workspace and back
            for (int64_t k = 0; k < steps && e == hipSuccess; ++k) {
                const double h = k + 1 == steps ? dt_last : dt;
                e = launch_stage(p, alpha, phi_out, nullptr, target, p->ws[0], h, 0.0, 1.0, false, s);
                if (e == hipSuccess) e = launch_copy(p, p->ws[0], phi_out, s);
            }
            return e;
        }
        // step k writes phi_out when steps - k is odd, else the workspace
        const void *cur = phi0;
        for (int64_t k = 0; k < steps && e == hipSuccess; ++k) {
            const double h = k + 1 == steps ? dt_last : dt;
            void *nxt = ((steps - k) & 1) ? phi_out : p->ws[0];
            e = launch_stage(p, alpha, cur, nullptr, target, nxt, h, 0.0, 1.0, false, s);
            cur = nxt;
        }
        return e;
    }
    const void *src = phi0;
    for (int64_t k = 0; k < steps && e == hipSuccess; ++k) {
        const double h = k + 1 == steps ? dt_last : dt;
        void *a = p->ws[0], *b = p->ws[1];
        if (p->scheme.rk == 2) {  // odeCFL2: two Euler moves, then the average with phi^n
            e = launch_stage(p, alpha, src, nullptr, nullptr, a, h, 0.0, 1.0, false, s);
            if (e == hipSuccess) e = launch_stage(p, alpha, a, src, target, phi_out, h, 0.5, 0.5, false, s);
        } else {  // odeCFL3: Shu-Osher stages with averages 3/4, 1/4 and 1/3, 2/3
            e = launch_stage(p, alpha, src, nullptr, nullptr, a, h, 0.0, 1.0, false, s);
            if (e == hipSuccess) e = launch_stage(p, alpha, a, src, nullptr, b, h, 0.75, 0.25, false, s);
            if (e == hipSuccess)
                e = launch_stage(p, alpha, b, src, target, phi_out, h, 1.0 / 3.0, 2.0 / 3.0, false, s);
        }
        src = phi_out;
    }
    return e;
}

// the stepping launches captured on the problem's own stream into a graph
hjx_status capture_steps(hjx_problem *p, const double *alpha, const void *phi0, const void *target, void *phi_out,
                         int64_t steps, double dt, double dt_last, int *flags)
{
    if (!p->cap) HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_steps(p, alpha, phi0, target, phi_out, steps, dt, dt_last, p->cap, flags);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(p->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(HJX_ERR_DEVICE, "solve graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    p->graph = g;
    const hipError_t e3 = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
        p->exec = nullptr;
        return fail(HJX_ERR_DEVICE, "solve graph instantiate: %s", hipGetErrorString(e3));
    }
    return HJX_OK;
}

// whether hjx_solve may capture and replay its launches (HJX_SOLVE_GRAPH=0
// turns it off: every solve then launches directly)
bool solve_graphs_on()
{
    const char *v = std::getenv("HJX_SOLVE_GRAPH");
    return !(v && v[0] == '0' && v[1] == 0);
}

void release(hjx_problem *p)
{
    if (!p) return;
    drop_solve_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->tables) (void)hipFree(p->tables);
    for (void *w : p->ws)
        if (w) (void)hipFree(w);
    if (p->dalpha) (void)hipFree(p->dalpha);
    if (p->dflag) (void)hipFree(p->dflag);
    if (p->hbuf) (void)hipHostFree(p->hbuf);
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

}  // namespace

// ==================================================================== ABI

extern "C" {

const char *hjx_version(void) { return "0.1.0"; }

const char *hjx_last_error(void) { return g_last_error.c_str(); }

hjx_status hjx_problem_create(const hjx_grid_desc *grid, const hjx_ham_desc *ham, const hjx_scheme_desc *scheme,
                              hjx_problem **out)
{
    if (!out) return fail(HJX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hjx_status st = validate(grid, ham, scheme);
    if (st != HJX_OK) return st;

    hjx_problem *p = new (std::nothrow) hjx_problem;
    if (!p) return fail(HJX_ERR_OOM, "host allocation failed");
    p->grid = *grid;
    p->ham = *ham;
    p->scheme = *scheme;
    p->total = 1;
    for (int d = 0; d < grid->dim; ++d) {
        p->total *= grid->n[d];
        const double len = grid->gmax[d] - grid->gmin[d];
        p->dx[d] = ((grid->periodic_mask >> d) & 1u) ? len / (double)grid->n[d] : len / (double)(grid->n[d] - 1);
    }
    p->elem = scheme->dtype == HJX_F32 ? sizeof(float) : sizeof(double);
    if (!tile_ok(geometry(p), p->elem)) {
        release(p);
        return fail(HJX_ERR_UNSUPPORTED, grid->dim <= 2   ? "a 1-D or 2-D grid's arrays must be under 4 GiB"
                                         : grid->dim == 3 ? "a plane of the two fastest axes must be under 4 GiB"
                                                          : "seven planes of the two fastest axes must be under 4 GiB");
    }

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        release(p);
        return fail(HJX_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }

    // per-axis tables: coordinates gmin + j dx, their cosine and sine
    size_t bytes = 0;
    for (int d = 0; d < grid->dim; ++d)
        for (int k = 0; k < 3; ++k) {
            p->table_off[d][k] = bytes;
            bytes += ((size_t)grid->n[d] * p->elem + 255) & ~size_t(255);
        }
    std::vector<unsigned char> host(bytes);
    for (int d = 0; d < grid->dim; ++d)
        for (int64_t j = 0; j < grid->n[d]; ++j) {
            const double x = grid->gmin[d] + (double)j * p->dx[d];
            const double v[3] = {x, std::cos(x), std::sin(x)};
            for (int k = 0; k < 3; ++k) {
                unsigned char *dst = host.data() + p->table_off[d][k] + (size_t)j * p->elem;
                if (p->elem == sizeof(float)) {
                    const float f = (float)v[k];
                    std::memcpy(dst, &f, sizeof f);
                } else {
                    std::memcpy(dst, &v[k], sizeof(double));
                }
            }
        }

    const size_t field = (size_t)p->total * p->elem;
    const int partials = alpha_blocks((int)p->total);
    size_t cap = 0;
    const size_t need = bytes + 2 * field + sizeof(double) * kMaxDim * (1 + (size_t)partials) + 2 * sizeof(int);
    if (over_workspace_cap(need, &cap)) {
        release(p);
        return fail(HJX_ERR_OOM, "problem workspace of %zu bytes exceeds HJX_MAX_WORKSPACE=%zu", need, cap);
    }
    if ((e = hipMalloc(&p->tables, bytes)) != hipSuccess ||
        (e = hipMemcpy(p->tables, host.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMalloc(&p->ws[0], field)) != hipSuccess || (e = hipMalloc(&p->ws[1], field)) != hipSuccess ||
        (e = hipMalloc(&p->dalpha, sizeof(double) * kMaxDim * (1 + (size_t)partials))) != hipSuccess ||
        (e = hipMalloc(&p->dflag, 2 * sizeof(int))) != hipSuccess ||
        (e = hipHostMalloc(&p->hbuf, sizeof(double) * (kMaxDim + 1), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreate(&p->ev[0])) != hipSuccess || (e = hipEventCreate(&p->ev[1])) != hipSuccess) {
        release(p);
        return fail(e == hipErrorOutOfMemory ? HJX_ERR_OOM : HJX_ERR_DEVICE, "problem allocation: %s",
                    hipGetErrorString(e));
    }
    p->tile = default_tile(geometry(p), p->elem, p->scheme.deriv, p->scheme.rk);
    *out = p;
    return ok();
}

hjx_status hjx_problem_destroy(hjx_problem *p)
{
    release(p);
    return ok();
}

hjx_status hjx_problem_set_params(hjx_problem *p, const double *params)
{
    if (!p || !params) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    hjx_ham_desc h = p->ham;
    const int np = n_params(h.kind);
    for (int k = 0; k < 8; ++k) h.p[k] = k < np ? params[k] : 0.0;
    hjx_status st = validate(&p->grid, &h, &p->scheme);
    if (st != HJX_OK) return st;
    if (std::memcmp(h.p, p->ham.p, sizeof h.p) == 0) return ok();
    p->ham = h;
    p->alpha_known = false;  // alpha and the captured launches carry the old values
    drop_solve_graph(p);
    return ok();
}

hjx_status hjx_problem_set_tile(hjx_problem *p, int32_t variant, int32_t tx, int32_t ty, int32_t march)
{
    if (!p) return fail(HJX_ERR_INVALID_ARG, "NULL problem");
    drop_solve_graph(p);  // its launches carry the old shape
    const GridGeom g = geometry(p);
    if (variant == HJX_TILE_DIRECT) {
        if (!direct_ok(g, p->elem)) return fail(HJX_ERR_UNSUPPORTED, "the direct variant needs arrays under 4 GiB");
        p->tile = Tile{256, 1, 1, kVariantDirect};
        return ok();
    }
    if (variant == HJX_TILE_STEPS) {
        if (g.dim > 2) return fail(HJX_ERR_UNSUPPORTED, "the steps variant takes 1-D and 2-D grids");
        if (!direct_ok(g, p->elem)) return fail(HJX_ERR_UNSUPPORTED, "the steps variant needs arrays under 4 GiB");
        const Tile t{tx, ty, march, kVariantSteps};
        if (!steps_shape(g, p->elem, p->scheme.deriv, p->scheme.rk, t, nullptr))
            return fail(HJX_ERR_INVALID_ARG,
                        "steps tile %d x %d, %d steps: needs tx, ty, steps >= 1 (ty = 1 in 1-D), a halo of "
                        "steps * rk * radius nodes no deeper than a periodic axis and at most %zu bytes of LDS",
                        tx, ty, march, kStepsLdsMax);
        p->tile = t;
        return ok();
    }
    if (variant != HJX_TILE_PLANE_MARCH) return fail(HJX_ERR_INVALID_ARG, "unknown tile variant %d", variant);
    const int maxn = tile_max_nodes(g);
    if (tx < 1 || ty < 1 || (int64_t)tx * ty > maxn)
        return fail(HJX_ERR_INVALID_ARG, "tile %d x %d: need 1 <= tx*ty <= %d", tx, ty, maxn);
    if (g.dim == 1 && ty != 1) return fail(HJX_ERR_INVALID_ARG, "a 1-D grid needs ty = 1");
    if (march < 1) return fail(HJX_ERR_INVALID_ARG, "march %d < 1", march);
    if (g.dim >= 3) {
        const int64_t blocks = (int64_t)((g.n[g.dim - 1] + tx - 1) / tx) * ((g.n[g.dim - 2] + ty - 1) / ty) *
                               ((g.n[0] + march - 1) / march) * (g.dim == 4 ? g.n[1] : 1);
        if (blocks > (int64_t(1) << 30))
            return fail(HJX_ERR_INVALID_ARG, "tile %d x %d march %d: %lld blocks (> 2^30)", tx, ty, march,
                        (long long)blocks);
    }
    p->tile = Tile{tx, ty, g.dim >= 3 ? march : 1, kVariantPlaneMarch};
    return ok();
}

hjx_status hjx_problem_get_tile(const hjx_problem *p, int32_t *variant, int32_t *tx, int32_t *ty, int32_t *march)
{
    if (!p || !variant || !tx || !ty || !march) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    *variant = p->tile.variant == kVariantDirect ? HJX_TILE_DIRECT
               : p->tile.variant == kVariantSteps  ? HJX_TILE_STEPS
                                                   : HJX_TILE_PLANE_MARCH;
    *tx = p->tile.tx;
    *ty = p->tile.ty;
    *march = p->tile.march;
    return ok();
}

}  // extern "C"

namespace {

// The autotuner's cache: a text file of one line per tuned problem,
//   hjx-tune 1 <arch> <compute units> <dtype> <dim> <n0>x..x<n3> <periodic>
//       <deriv> <rk> <ham> <dissipation> <restrict> | <variant> <tx> <ty> <march> <us>
// the part before '|' naming the device and everything the launch shape
// can depend on, the part after the shape and its time.  The last line with
// a problem's key wins; new results are appended.
std::string tune_key(const hjx_problem *p)
{
    hipDeviceProp_t prop{};
    const bool have = hipGetDeviceProperties(&prop, p->device) == hipSuccess;
    char buf[512];
    int o = std::snprintf(buf, sizeof buf, "hjx-tune 1 %s %d %s %d ", have ? prop.gcnArchName : "unknown",
                          have ? prop.multiProcessorCount : 0, p->scheme.dtype == HJX_F32 ? "f32" : "f64",
                          p->grid.dim);
    for (int d = 0; d < p->grid.dim; ++d)
        o += std::snprintf(buf + o, sizeof buf - o, d ? "x%lld" : "%lld", (long long)p->grid.n[d]);
    std::snprintf(buf + o, sizeof buf - o, " %u %d %d %d %d %d", p->grid.periodic_mask, p->scheme.deriv,
                  p->scheme.rk, p->ham.kind, p->ham.dissipation, p->scheme.restrict_update);
    return buf;
}

const char *tune_cache_path(const char *given)
{
    if (given) return given[0] ? given : nullptr;
    const char *env = std::getenv("HJX_TUNE_CACHE");
    return env && env[0] ? env : nullptr;
}

// the cached shape for key, if the file has one
bool tune_cache_find(const char *path, const std::string &key, Tile *tile, double *us)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string prefix = key + " | ";
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, prefix.c_str(), prefix.size()) != 0) continue;
        int v = 0, tx = 0, ty = 0, m = 0;
        double t = 0.0;
        if (std::sscanf(line + prefix.size(), "%d %d %d %d %lf", &v, &tx, &ty, &m, &t) == 5 &&
            (v == kVariantDirect || v == kVariantPlaneMarch || v == kVariantSteps)) {
            *tile = Tile{tx, ty, m, v};
            *us = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_add(const char *path, const std::string &key, const Tile &t, double us)
{
    FILE *f = std::fopen(path, "a");
    if (!f) return;  // a cache that cannot be written only costs the next call a retune
    std::fprintf(f, "%s | %d %d %d %d %.3f\n", key.c_str(), t.variant, t.tx, t.ty, t.march, us);
    std::fclose(f);
}

}  // namespace

extern "C" {

hjx_status hjx_tune(hjx_problem *p, const void *phi, int32_t reps, const char *cache_path, void *stream,
                    double *best_us)
{
    TraceRange trace_("hjx_tune");
    if (!p || !phi) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (reps < 1) return fail(HJX_ERR_INVALID_ARG, "reps %d < 1", reps);
    const char *cache = tune_cache_path(cache_path);
    const std::string key = cache ? tune_key(p) : std::string();
    if (cache) {
        Tile t{};
        double us = 0.0;
        if (tune_cache_find(cache, key, &t, &us)) {
            const int v = t.variant == kVariantDirect ? HJX_TILE_DIRECT
                          : t.variant == kVariantSteps  ? HJX_TILE_STEPS
                                                        : HJX_TILE_PLANE_MARCH;
            const hjx_status st = hjx_problem_set_tile(p, v, t.tx, t.ty, t.march);
            if (st == HJX_OK) {
                if (best_us) *best_us = us;
                return ok();
            }
            // a shape this problem rejects: tune again and append the new one
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double alpha[kMaxDim];
    hjx_status st = device_alpha(p, s, alpha);
    if (st != HJX_OK) return st;
    const double dt = cfl_dt(p, alpha);
    const double h = std::isfinite(dt) ? dt : 1.0;
    const GridGeom g = geometry(p);
    const int nf = g.n[g.dim - 1], nm = g.dim >= 2 ? g.n[g.dim - 2] : 1;
    const int nk = g.dim >= 3 ? g.n[0] : 1;  // the tile kernel marches axis 0
    const int outer = g.dim == 4 ? g.n[0] : 1;

    std::vector<Tile> cands;
    const int maxn = tile_max_nodes(g);
    for (int pieces = 1; pieces <= 8; ++pieces) {
        const int tx = (nf + pieces - 1) / pieces;
        if (tx > 256 || (pieces > 1 && tx < 8)) continue;
        // the tile kernel (3-D, 4-D) idles a thread per node short of 512:
        // only full tiles are worth timing there
        for (int nodes : {64, 128, 192, 256, 384, 512}) {
            if (nodes > maxn) break;
            if (g.dim >= 3 && nodes < 512) continue;
            int ty = g.dim >= 2 ? std::max(1, std::min(nodes / tx, nm)) : 1;
            if (tx * ty > maxn) continue;
            // march lengths: powers of two, and those that split axis 0 into
            // chunks of equal length (a last chunk of one plane pays a whole
            // block's set-up for it)
            std::vector<int> marches{1, 2, 4, 8, 16, 32};
            if (g.dim >= 3)
                for (int c = 1; c <= 64; ++c) {
                    const int m = (nk + c - 1) / c;
                    if (m <= 32 && nk % m == 0 && std::find(marches.begin(), marches.end(), m) == marches.end())
                        marches.push_back(m);
                }
            for (int m : marches) {
                if (g.dim < 3 && m > 1) break;
                if (m > nk && m > 1) continue;
                if (g.dim <= 2 && (long)((nk + m - 1) / m) * outer > 65535) continue;
                const Tile t{tx, ty, m, kVariantPlaneMarch};
                bool seen = false;
                for (const Tile &c : cands) seen |= c.tx == t.tx && c.ty == t.ty && c.march == t.march;
                if (!seen) cands.push_back(t);
            }
        }
    }
    if (direct_ok(g, p->elem)) cands.push_back(Tile{256, 1, 1, kVariantDirect});
    if (g.dim <= 2) {  // the steps variant: tiles of 64..1024 nodes, 1..8 steps per launch
        const int shapes[][2] = {{8, 8}, {16, 8}, {16, 16}, {32, 16}, {32, 32}, {64, 1}, {256, 1}, {1024, 1}};
        for (const auto &sh : shapes) {
            if ((g.dim == 1) != (sh[1] == 1)) continue;
            for (int k : {1, 2, 4, 8}) {
                const Tile t{sh[0], sh[1], k, kVariantSteps};
                if (steps_shape(g, p->elem, p->scheme.deriv, p->scheme.rk, t, nullptr)) cands.push_back(t);
            }
        }
    }
    const char *env = std::getenv("HJX_TUNE_VERBOSE");
    const bool verbose = env && env[0] && env[0] != '0';
    const Tile keep = p->tile;
    Tile best = keep;
    float best_ms = INFINITY;
    // time whole RK steps from phi into a temporary array, launched as a
    // solve launches them, without a target: a target adds one read to the
    // last stage of each step, half the traffic of a forward-Euler step, and
    // would favour shapes that hide it over those that are faster without
    void *work = nullptr;
    HIP_TRY(hipMalloc(&work, (size_t)p->total * p->elem));
    auto timed = [&](float *ms) -> hipError_t {
        hipError_t e;
        if ((e = enqueue_steps(p, alpha, phi, nullptr, work, reps, h, h, s, nullptr)) != hipSuccess) return e;  // untimed
        if ((e = hipEventRecord(p->ev[0], s)) != hipSuccess) return e;
        if ((e = enqueue_steps(p, alpha, phi, nullptr, work, reps, h, h, s, nullptr)) != hipSuccess) return e;
        if ((e = hipEventRecord(p->ev[1], s)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(p->ev[1])) != hipSuccess) return e;
        return hipEventElapsedTime(ms, p->ev[0], p->ev[1]);
    };
    for (const Tile &t : cands) {
        p->tile = t;
        // the faster of two timings: one launch's start-up latency and the
        // clock's ramp fall on a short timing unevenly across shapes
        float ms = 0.f, ms2 = 0.f;
        hipError_t e = timed(&ms);
        if (e == hipSuccess) e = timed(&ms2);
        ms = std::min(ms, ms2);
        if (e != hipSuccess) {
            (void)hipFree(work);
            p->tile = keep;
            return fail(HJX_ERR_DEVICE, "hjx_tune: %s", hipGetErrorString(e));
        }
        ms /= (float)p->scheme.rk;  // per stage launch
        if (verbose)
            fprintf(stderr, "hjx_tune: %s tile %3d x %3d march %2d: %9.2f us\n",
                    t.variant == kVariantDirect ? "direct" : (t.variant == kVariantSteps ? "steps " : "plane "), t.tx,
                    t.ty, t.march, (double)ms * 1e3 / reps);
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    HIP_TRY(hipFree(work));
    drop_solve_graph(p);
    p->tile = best;
    const double us = (double)best_ms * 1e3 / reps;
    if (cache) tune_cache_add(cache, key, best, us);
    if (best_us) *best_us = us;
    return ok();
}

hjx_status hjx_dissipation(hjx_problem *p, double *alpha_out, double *dt_out, void *stream)
{
    TraceRange trace_("hjx_dissipation");
    if (!p || !alpha_out || !dt_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    double alpha[kMaxDim];
    hjx_status st = device_alpha(p, static_cast<hipStream_t>(stream), alpha);
    if (st != HJX_OK) return st;
    for (int d = 0; d < p->grid.dim; ++d) alpha_out[d] = alpha[d];
    *dt_out = cfl_dt(p, alpha);
    return ok();
}

hjx_status hjx_rhs(hjx_problem *p, const void *phi, void *L_out, void *stream)
{
    TraceRange trace_("hjx_rhs");
    if (!p || !phi || !L_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (phi == L_out) return fail(HJX_ERR_INVALID_ARG, "phi and L_out alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double alpha[kMaxDim];
    hjx_status st = device_alpha(p, s, alpha);
    if (st != HJX_OK) return st;
    HIP_TRY(launch_stage(p, alpha, phi, nullptr, nullptr, L_out, 0.0, 0.0, 1.0, true, s));
    return ok();
}

hjx_status hjx_step(hjx_problem *p, void *phi, const void *target, double dt, void *stream)
{
    TraceRange trace_("hjx_step");
    if (!p || !phi) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (target == phi) return fail(HJX_ERR_INVALID_ARG, "target aliases phi");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HJX_ERR_INVALID_ARG, "dt %g is not a positive finite step", dt);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double alpha[kMaxDim];
    hjx_status st = device_alpha(p, s, alpha);
    if (st != HJX_OK) return st;
    HIP_TRY(rk_step(p, alpha, phi, target, dt, s));
    return ok();
}

hjx_status hjx_solve(hjx_problem *p, const void *phi0, const void *target, void *phi_out, double t0, double t1,
                     void *stream, hjx_stats *stats)
{
    TraceRange trace_("hjx_solve");
    if (!p || !phi0 || !phi_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (target && target == phi_out) return fail(HJX_ERR_INVALID_ARG, "target aliases phi_out");
    if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0))
        return fail(HJX_ERR_INVALID_ARG, "time span [%g, %g] is not finite and increasing", t0, t1);
    hipStream_t s = static_cast<hipStream_t>(stream);

    double alpha[kMaxDim];
    hjx_status st = device_alpha(p, s, alpha);
    if (st != HJX_OK) return st;
    const double dt = cfl_dt(p, alpha);
    int64_t steps = 0;
    double dt_last = 0.0;
    schedule(t0, t1, dt, &steps, &dt_last);

    // the input check, the stepping launches, the output check, then the
    // one host synchronisation of the call (the steps variant checks inside
    // its first and last launches: two launches fewer)
    const bool fused = p->tile.variant == kVariantSteps && steps > 0;
    int *flags = fused ? p->dflag : nullptr;
    HIP_TRY(hipMemsetAsync(p->dflag, 0, 2 * sizeof(int), s));
    if (!fused) HIP_TRY(check_nonfinite(p, phi0, 0, s));
    if (stats) HIP_TRY(hipEventRecord(p->ev[0], s));
    const hjx_problem::SolveKey key{phi0, target, phi_out, t0, t1};
    if (p->exec && p->have_key && key == p->last_key) {
        HIP_TRY(hipGraphLaunch(p->exec, s));
    } else if (solve_graphs_on() && steps > 1 && p->have_key && key == p->last_key) {
        // the same solve a second time in a row: capture it once, replay it from now on
        if ((st = capture_steps(p, alpha, phi0, target, phi_out, steps, dt, dt_last, flags)) != HJX_OK) return st;
        HIP_TRY(hipGraphLaunch(p->exec, s));
    } else {
        drop_solve_graph(p);
        HIP_TRY(enqueue_steps(p, alpha, phi0, target, phi_out, steps, dt, dt_last, s, flags));
        p->last_key = key;
        p->have_key = true;
    }
    if (stats) HIP_TRY(hipEventRecord(p->ev[1], s));
    if (!fused) HIP_TRY(check_nonfinite(p, phi_out, 1, s));
    int *hflag = reinterpret_cast<int *>(p->hbuf + kMaxDim);
    HIP_TRY(hipMemcpyAsync(hflag, p->dflag, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const bool bad_in = hflag[0] != 0, bad_out = hflag[1] != 0;

    if (stats) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
        stats->steps = steps;
        stats->dt = dt;
        stats->dt_last = dt_last;
        stats->t_final = steps > 0 ? t1 : t0;
        for (int d = 0; d < kMaxDim; ++d) stats->alpha[d] = alpha[d];
        stats->elapsed_ms = ms;
        // algorithmic bytes per step: every stage reads its input and writes
        // its output once; stages after the first also read phi^n; the last
        // stage reads the target.  Halo re-reads are not counted.
        const double f = (double)p->total * (double)p->elem;
        const int rk = p->scheme.rk;
        double per_step = rk == 1 ? 2.0 : (rk == 2 ? 2.0 + 3.0 : 2.0 + 3.0 + 3.0);
        if (target) per_step += 1.0;
        stats->alg_bytes = per_step * f * (double)steps;
    }
    if (bad_in) return fail(HJX_ERR_NONFINITE, "phi0 holds NaN or Inf");
    if (bad_out) return fail(HJX_ERR_NONFINITE, "the solution holds NaN or Inf");
    return ok();
}

}  // extern "C"

// ==================================================================== adjoint (host)

struct hjx_tape {
    hjx_problem *p = nullptr;
    double t0 = 0, t1 = 0, dt = 0, dt_last = 0, alpha[kMaxDim] = {0, 0, 0, 0};
    double hp[8] = {};                 // the problem's parameters when the tape was made
    int64_t steps = 0;
    int K = 1, nseg = 0;
    std::vector<void *> ckpt;          // phi at the start of every segment
    // replay workspace, two sets: the replay of one segment writes one set
    // while the reverse sweep of the next reads the other
    struct ReplaySet {
        std::vector<void *> phin, x1, xh;  // stage inputs of each step of a segment
        // the replay's decisions, a byte per node: bit 0 where the target was
        // the smaller, bit 1 where a restricted update clipped the rate.  One
        // array per step (its last stage) or, for a restricted update, per
        // stage (step i, stage k at i rk + k).
        std::vector<unsigned char *> mask;
        std::vector<void *> dp;            // p-, p+ of every stage (empty: recompute)
    } rs[2];
    void *lam[4] = {nullptr, nullptr, nullptr, nullptr};
    void *seed_m[kMaxDim] = {}, *seed_p[kMaxDim] = {};
    void *contrib[kMaxDim] = {};       // per-axis transpose contributions (dim >= 2)
    bool pending = false;              // contrib holds sums not yet added to the last lam_in
    size_t base_bytes = 0;             // device workspace without the derivative store
    double *acc = nullptr;             // per seed-kernel block
    int acc_blocks = 0;
    double *acc_out = nullptr;         // device, kAccCount
    double *hacc = nullptr;            // pinned, kAccCount
    const void *target = nullptr;
    bool solved = false;
    bool clip = false;                 // a restricted update: every stage keeps its mask

    // the mask stage k of step i of a replay set writes (and its reverse
    // reads), or null when that stage has no decision to keep
    unsigned char *mask_of(const ReplaySet &r, int i, int k) const
    {
        const int rk = p->scheme.rk;
        if (clip) return r.mask[(size_t)i * rk + k];
        return k == rk - 1 && target ? r.mask[i] : nullptr;
    }
};

namespace {

void tape_release(hjx_tape *t)
{
    if (!t) return;
    auto f = [](void *x) {
        if (x) (void)hipFree(x);
    };
    for (void *x : t->ckpt) f(x);
    for (auto &r : t->rs) {
        for (void *x : r.phin) f(x);
        for (void *x : r.x1) f(x);
        for (void *x : r.xh) f(x);
        for (unsigned char *x : r.mask) f(x);
        for (void *x : r.dp) f(x);
    }
    for (void *x : t->lam) f(x);
    for (int d = 0; d < kMaxDim; ++d) {
        f(t->seed_m[d]);
        f(t->seed_p[d]);
        f(t->contrib[d]);
    }
    f(t->acc);
    f(t->acc_out);
    if (t->hacc) (void)hipHostFree(t->hacc);
    delete t;
}

// bytes of the replay's derivative store: p-, p+ per axis for every stage
// of a segment, in both replay sets
size_t tape_dp_bytes(const hjx_problem *p, const hjx_tape *t)
{
    const int K = (int)std::min<int64_t>(t->K, std::max<int64_t>(t->steps, 1));
    return 2 * (size_t)K * (size_t)p->scheme.rk * 2 * (size_t)p->grid.dim * (size_t)p->total * p->elem;
}

void tape_free_dp(hjx_tape *t)
{
    for (auto &r : t->rs) {
        for (void *x : r.dp)
            if (x) (void)hipFree(x);
        r.dp.clear();
    }
}

hjx_status tape_alloc_dp(const hjx_problem *p, hjx_tape *t)
{
    const int K = (int)std::min<int64_t>(t->K, std::max<int64_t>(t->steps, 1));
    const size_t block = 2 * (size_t)p->grid.dim * (size_t)p->total * p->elem;
    for (auto &r : t->rs) {
        r.dp.assign((size_t)K * p->scheme.rk, nullptr);
        for (auto &x : r.dp) {
            const hipError_t e = hipMalloc(&x, block);
            if (e != hipSuccess) {
                tape_free_dp(t);
                return fail(e == hipErrorOutOfMemory ? HJX_ERR_OOM : HJX_ERR_DEVICE, "derivative store: %s",
                            hipGetErrorString(e));
            }
        }
    }
    return HJX_OK;
}

// dalpha_d / dtheta_m of the built-in bounds, differentiated at the first
// node where each maximum is attained (FP64, from the same node formula as
// the device tables)
void alpha_jacobian(const hjx_problem *p, double J[kMaxDim][8])
{
    for (int d = 0; d < kMaxDim; ++d)
        for (int m = 0; m < 8; ++m) J[d][m] = 0.0;
    auto node = [&](int d, int64_t j) { return p->grid.gmin[d] + (double)j * p->dx[d]; };
    auto sgn = [](double x) { return x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0); };
    const double *h = p->ham.p;
    if (p->ham.kind == HJX_HAM_NORMAL) {
        for (int d = 0; d < p->grid.dim; ++d) J[d][0] = sgn(h[0]);
    } else if (p->ham.kind == HJX_HAM_DUBINS3_PE) {
        // alpha_0 = max_th |-v_e + v_p cos th| + wbar_e max_y |y|
        // alpha_1 = max_th |v_p sin th| + wbar_e max_x |x|,  alpha_2 = wbar_e + wbar_p
        double b0 = -1, c0 = 0, b1 = -1, s1 = 0, ymax = 0, xmax = 0;
        for (int64_t k = 0; k < p->grid.n[2]; ++k) {
            const double th = node(2, k), c = std::cos(th), sn = std::sin(th);
            const double v0 = std::fabs(-h[0] + h[1] * c), v1 = std::fabs(h[1] * sn);
            if (v0 > b0) { b0 = v0; c0 = c; }
            if (v1 > b1) { b1 = v1; s1 = sn; }
        }
        for (int64_t j = 0; j < p->grid.n[1]; ++j) ymax = std::max(ymax, std::fabs(node(1, j)));
        for (int64_t i = 0; i < p->grid.n[0]; ++i) xmax = std::max(xmax, std::fabs(node(0, i)));
        const double g0 = sgn(-h[0] + h[1] * c0), g1 = sgn(h[1] * s1);
        J[0][0] = -g0;
        J[0][1] = g0 * c0;
        J[0][2] = ymax;
        J[1][1] = g1 * s1;
        J[1][2] = xmax;
        J[2][2] = 1.0;
        J[2][3] = 1.0;
    } else if (p->ham.kind == HJX_HAM_ROCKETS) {
        // alpha_0 = max_th |a cos th| + ubar_e max_x |x|
        // alpha_1 = max_th |a sin th + a - g| + ubar_p max_x |x|,  alpha_2 = ubar_e + ubar_p
        // (ubar_e, ubar_p >= 0, so each maximum splits over th and x)
        double b0 = -1, c0 = 0, b1 = -1, s1 = 0, xmax = 0;
        for (int64_t k = 0; k < p->grid.n[2]; ++k) {
            const double th = node(2, k), c = std::cos(th), sn = std::sin(th);
            const double v0 = std::fabs(h[0] * c), v1 = std::fabs(h[0] * sn + h[0] - h[1]);
            if (v0 > b0) { b0 = v0; c0 = c; }
            if (v1 > b1) { b1 = v1; s1 = sn; }
        }
        for (int64_t i = 0; i < p->grid.n[0]; ++i) xmax = std::max(xmax, std::fabs(node(0, i)));
        const double g0 = sgn(h[0] * c0), g1 = sgn(h[0] * s1 + h[0] - h[1]);
        J[0][0] = g0 * c0;
        J[0][2] = xmax;
        J[1][0] = g1 * (s1 + 1.0);
        J[1][1] = -g1;
        J[1][3] = xmax;
        J[2][2] = 1.0;
        J[2][3] = 1.0;
    } else {
        // alpha_0, alpha_1 = max |v cos th|, |v sin th| (no parameters); alpha_2 = wbar, alpha_3 = abar
        J[2][0] = 1.0;
        J[3][1] = 1.0;
    }
}

}  // namespace

extern "C" {

hjx_status hjx_tape_create(hjx_problem *p, double t0, double t1, int32_t ckpt_every, void *stream, hjx_tape **out)
{
    if (!p || !out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 >= t0))
        return fail(HJX_ERR_INVALID_ARG, "time span [%g, %g] is not finite and increasing", t0, t1);
    if (ckpt_every < 1) return fail(HJX_ERR_INVALID_ARG, "ckpt_every %d < 1", ckpt_every);
    if (!direct_ok(geometry(p), p->elem)) return fail(HJX_ERR_UNSUPPORTED, "the adjoint needs arrays under 4 GiB");
    hjx_tape *t = new (std::nothrow) hjx_tape;
    if (!t) return fail(HJX_ERR_OOM, "host allocation failed");
    t->p = p;
    std::memcpy(t->hp, p->ham.p, sizeof t->hp);
    t->t0 = t0;
    t->t1 = t1;
    t->K = ckpt_every;
    t->clip = p->scheme.restrict_update != HJX_RESTRICT_NONE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hjx_status st = device_alpha(p, s, t->alpha);
    if (st != HJX_OK) {
        tape_release(t);
        return st;
    }
    t->dt = cfl_dt(p, t->alpha);
    schedule(t0, t1, t->dt, &t->steps, &t->dt_last);
    t->nseg = (int)((t->steps + t->K - 1) / t->K);
    const size_t field = (size_t)p->total * p->elem;
    const int K = (int)std::min<int64_t>(t->K, std::max<int64_t>(t->steps, 1));
    {
        const int rk = p->scheme.rk;
        const size_t masks = (size_t)K * (t->clip ? rk : 1);
        const size_t sets = 2 * ((size_t)K * (1 + (rk >= 2) + (rk >= 3)) * field + masks * (size_t)p->total);
        const size_t need = (size_t)t->nseg * field + sets + 4 * field +
                            (size_t)p->grid.dim * (p->grid.dim >= 2 ? 3 : 2) * field +
                            sizeof(double) * kAccCount * ((size_t)adj_seed_blocks(geometry(p)) + 1);
        size_t cap = 0;
        if (over_workspace_cap(need, &cap)) {
            tape_release(t);
            return fail(HJX_ERR_OOM, "tape workspace of %zu bytes exceeds HJX_MAX_WORKSPACE=%zu", need, cap);
        }
        t->base_bytes = need;
    }
    hipError_t e = hipSuccess;
    auto grab = [&](void **x, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(x, bytes);
    };
    t->ckpt.assign(t->nseg, nullptr);
    for (auto &x : t->ckpt) grab(&x, field);
    for (auto &r : t->rs) {
        r.phin.assign(K + 1, nullptr);
        for (int i = 1; i <= K; ++i) grab(&r.phin[i], field);  // phin[0] is the checkpoint itself
        if (p->scheme.rk >= 2) {
            r.x1.assign(K, nullptr);
            for (auto &x : r.x1) grab(&x, field);
        }
        if (p->scheme.rk >= 3) {
            r.xh.assign(K, nullptr);
            for (auto &x : r.xh) grab(&x, field);
        }
        r.mask.assign((size_t)K * (t->clip ? p->scheme.rk : 1), nullptr);
        for (auto &x : r.mask) grab(reinterpret_cast<void **>(&x), (size_t)p->total);
    }
    for (auto &x : t->lam) grab(&x, field);
    for (int d = 0; d < p->grid.dim; ++d) {
        grab(&t->seed_m[d], field);
        grab(&t->seed_p[d], field);
        if (p->grid.dim >= 2) grab(&t->contrib[d], field);
    }
    t->acc_blocks = adj_seed_blocks(geometry(p));
    grab(reinterpret_cast<void **>(&t->acc), sizeof(double) * kAccCount * (size_t)t->acc_blocks);
    grab(reinterpret_cast<void **>(&t->acc_out), sizeof(double) * kAccCount);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&t->hacc), sizeof(double) * kAccCount,
                                           hipHostMallocDefault);
    if (e != hipSuccess) {
        tape_release(t);
        return fail(e == hipErrorOutOfMemory ? HJX_ERR_OOM : HJX_ERR_DEVICE, "tape allocation: %s",
                    hipGetErrorString(e));
    }
    // keep the replay's derivatives when they take at most a quarter of the
    // free device memory
    size_t free_b = 0, total_b = 0, cap = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && tape_dp_bytes(p, t) <= free_b / 4 &&
        !over_workspace_cap(t->base_bytes + tape_dp_bytes(p, t), &cap)) {
        st = tape_alloc_dp(p, t);
        if (st != HJX_OK) {
            tape_release(t);
            return st;
        }
    }
    *out = t;
    return ok();
}

hjx_status hjx_tape_set_mode(hjx_tape *tape, int32_t mode)
{
    if (!tape) return fail(HJX_ERR_INVALID_ARG, "NULL tape");
    if (mode != HJX_TAPE_RECOMPUTE && mode != HJX_TAPE_STORE_DERIVS)
        return fail(HJX_ERR_INVALID_ARG, "mode %d: HJX_TAPE_RECOMPUTE or HJX_TAPE_STORE_DERIVS", mode);
    if (mode == HJX_TAPE_RECOMPUTE) {
        tape_free_dp(tape);
        return ok();
    }
    if (!tape->rs[0].dp.empty()) return ok();
    size_t cap = 0;
    if (over_workspace_cap(tape->base_bytes + tape_dp_bytes(tape->p, tape), &cap))
        return fail(HJX_ERR_OOM, "the derivative store would exceed HJX_MAX_WORKSPACE=%zu", cap);
    const hjx_status st = tape_alloc_dp(tape->p, tape);
    return st == HJX_OK ? ok() : st;
}

hjx_status hjx_tape_get_mode(const hjx_tape *tape, int32_t *mode)
{
    if (!tape || !mode) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    *mode = tape->rs[0].dp.empty() ? HJX_TAPE_RECOMPUTE : HJX_TAPE_STORE_DERIVS;
    return ok();
}

hjx_status hjx_tape_destroy(hjx_tape *tape)
{
    tape_release(tape);
    return ok();
}

hjx_status hjx_solve_taped(hjx_problem *p, hjx_tape *tape, const void *phi0, const void *target, void *phi_out,
                           void *stream, hjx_stats *stats)
{
    TraceRange trace_("hjx_solve_taped");
    if (!p || !tape || !phi0 || !phi_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (tape->p != p) return fail(HJX_ERR_INVALID_ARG, "the tape belongs to another problem");
    if (std::memcmp(tape->hp, p->ham.p, sizeof tape->hp) != 0)
        return fail(HJX_ERR_INVALID_ARG, "the problem's parameters changed since the tape was made");
    if (target && target == phi_out) return fail(HJX_ERR_INVALID_ARG, "target aliases phi_out");
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool bad = false;
    hjx_status st = any_nonfinite(p, phi0, s, &bad);
    if (st != HJX_OK) return st;
    if (bad) return fail(HJX_ERR_NONFINITE, "phi0 holds NaN or Inf");
    if (phi_out != phi0) HIP_TRY(launch_copy(p, phi0, phi_out, s));
    if (stats) HIP_TRY(hipEventRecord(p->ev[0], s));
    for (int64_t n = 0; n < tape->steps; ++n) {
        if (n % tape->K == 0) HIP_TRY(launch_copy(p, phi_out, tape->ckpt[n / tape->K], s));
        const double h = n == tape->steps - 1 ? tape->dt_last : tape->dt;
        if (p->scheme.rk == 1) {
            HIP_TRY(launch_stage(p, tape->alpha, phi_out, nullptr, target, p->ws[0], h, 0.0, 1.0, false, s));
            HIP_TRY(launch_copy(p, p->ws[0], phi_out, s));
        } else {
            HIP_TRY(rk_step(p, tape->alpha, phi_out, target, h, s));
        }
    }
    if (stats) HIP_TRY(hipEventRecord(p->ev[1], s));
    if ((st = any_nonfinite(p, phi_out, s, &bad)) != HJX_OK) return st;
    tape->target = target;
    tape->solved = true;
    if (stats) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
        stats->steps = tape->steps;
        stats->dt = tape->dt;
        stats->dt_last = tape->dt_last;
        stats->t_final = tape->t1;
        for (int d = 0; d < kMaxDim; ++d) stats->alpha[d] = tape->alpha[d];
        stats->elapsed_ms = ms;
        stats->alg_bytes = 0.0;
    }
    if (bad) return fail(HJX_ERR_NONFINITE, "the solution holds NaN or Inf");
    return ok();
}

}  // extern "C"

namespace {

// One forward stage of a replay: out = ca phin + cb (in + h L(in)), min with
// the target when target is set; the stage's decisions go to mask (the
// tape's mask_of; nullable) and p-, p+ to dp (nullable).
struct ReplayStage {
    const void *in, *phin, *target;
    void *out;
    double h, ca, cb;
    unsigned char *mask;
    void *dp;
};

template <typename T>
StageArgs<T> replay_args(const hjx_problem *p, const double *alpha, const ReplayStage &r)
{
    StageArgs<T> a = stage_args<T>(p, alpha);
    a.dp_out = static_cast<T *>(r.dp);
    a.dp_stride = (int)p->total;
    a.phi_in = static_cast<const T *>(r.in);
    a.phi_n = static_cast<const T *>(r.phin);
    a.target = static_cast<const T *>(r.target);
    a.out = static_cast<T *>(r.out);
    a.dt = T(r.h);
    a.ca = T(r.ca);
    a.cb = T(r.cb);
    a.mask = r.mask;
    return a;
}

hipError_t replay_stage(const hjx_problem *p, const double *alpha, const ReplayStage &r, hipStream_t s)
{
    if (p->scheme.dtype == HJX_F32)
        return launch_stage_f32(replay_args<float>(p, alpha, r), p->scheme.deriv, p->ham.kind, s);
    return launch_stage_f64(replay_args<double>(p, alpha, r), p->scheme.deriv, p->ham.kind, s);
}

// Reverse one stage.  rep (nullable): a forward stage of the replay of the
// preceding segment, evaluated in the same launch as the seed pass.
template <typename T>
hipError_t reverse_stage_t(const hjx_problem *p, hjx_tape *t, const void *in, const void *lam_out,
                           const unsigned char *mask, void *lam_target, void *lam_in, int in_mode, void *lam_n,
                           int n_mode, double ca, double cb, double h, int h_slot, const void *dp,
                           const ReplayStage *rep, hipStream_t s)
{
    AdjSeedArgs<T> a{};
    a.dp_in = static_cast<const T *>(dp);
    a.dp_stride = (int)p->total;
    // lam_out is the lam_in of the stage reversed just before, whose per-axis
    // contributions are still pending
    if (t->pending)
        for (int d = 0; d < p->grid.dim; ++d) a.lam_add[a.n_add++] = static_cast<const T *>(t->contrib[d]);
    a.st = stage_args<T>(p, t->alpha);
    a.st.phi_in = static_cast<const T *>(in);
    a.lam_out = static_cast<const T *>(lam_out);
    a.mask = mask;
    a.lam_target = static_cast<T *>(lam_target);
    for (int d = 0; d < kMaxDim; ++d) {
        a.seed_m[d] = static_cast<T *>(t->seed_m[d]);
        a.seed_p[d] = static_cast<T *>(t->seed_p[d]);
    }
    a.lam_in = static_cast<T *>(lam_in);
    a.in_mode = in_mode;
    a.lam_n = static_cast<T *>(lam_n);
    a.n_mode = n_mode;
    a.ca = T(ca);
    a.cb = T(cb);
    a.h = T(h);
    a.acc = t->acc;
    a.h_slot = h_slot;
    StageArgs<T> ra;
    if (rep) ra = replay_args<T>(p, t->alpha, *rep);
    hipError_t e;
    if constexpr (std::is_same<T, float>::value)
        e = launch_adj_seed_f32(a, rep ? &ra : nullptr, p->scheme.deriv, p->ham.kind, s);
    else
        e = launch_adj_seed_f64(a, rep ? &ra : nullptr, p->scheme.deriv, p->ham.kind, s);
    if (e != hipSuccess) return e;
    // the transposes of all axes in one launch; with several axes each
    // writes its own contribution, added to lam_in afterwards in axis order
    const GridGeom g = geometry(p);
    AdjAxesArgs<T> xs{};
    xs.nax = g.dim;
    AdjCombineArgs<T> cmb{};
    cmb.n = g.dim >= 2 ? g.dim : 0;
    for (int d = 0; d < g.dim; ++d) {
        AdjAxisArgs<T> &x = xs.ax[d];
        x.phi = static_cast<const T *>(in);
        x.seed_m = static_cast<const T *>(t->seed_m[d]);
        x.seed_p = static_cast<const T *>(t->seed_p[d]);
        x.lam = static_cast<T *>(lam_in);
        x.out = g.dim >= 2 ? static_cast<T *>(t->contrib[d]) : nullptr;
        cmb.c[d] = x.out;
        x.g = g;
        x.d = d;
        // cross axis: the fastest axis (coalesced rows), or the second-fastest
        // when the line itself is the fastest axis
        x.c = d != g.dim - 1 ? g.dim - 1 : (g.dim >= 2 ? g.dim - 2 : -1);
        int r = 0;
        x.rest[0] = x.rest[1] = -1;
        for (int k = 0; k < g.dim; ++k)
            if (k != d && k != x.c) x.rest[r++] = k;
        x.inv_dx = T(1.0 / p->dx[d]);
        x.dx = T(p->dx[d]);
        const int nd = g.n[d], nc = x.c >= 0 ? g.n[x.c] : 1;
        // line tiles split each axis into equal pieces of at most 64 (fastest
        // axis, along the lanes) or 32 nodes (other axes, up to 8 columns of
        // the fastest axis per block): each piece transposes its tl + 5
        // intervals, and tw lines are taken so that those (tl + 5) tw
        // intervals fit the block's 256 threads, one each
        const int cap = d == g.dim - 1 ? 64 : 32;
        const int pieces = (nd + cap - 1) / cap;
        x.tl = std::max(2, (nd + pieces - 1) / pieces);
        const int fit = std::max(1, 256 / (x.tl + 5));
        if (d == g.dim - 1)
            x.tw = std::max(1, std::min(fit, nc));
        else {  // a power of two (the kernel shifts instead of dividing)
            x.tw = std::min(nc >= 8 ? 8 : (nc >= 4 ? 4 : (nc >= 2 ? 2 : 1)), fit);
            while (x.tw & (x.tw - 1)) --x.tw;
        }
    }
    if constexpr (std::is_same<T, float>::value)
        e = launch_adj_axes_f32(xs, p->scheme.deriv, s);
    else
        e = launch_adj_axes_f64(xs, p->scheme.deriv, s);
    // with several axes the contributions stay in contrib: the next seed
    // kernel (or the final combine) adds them to lam_in as it reads it
    t->pending = cmb.n > 0;
    return e;
}

// lam += the pending per-axis contributions
hipError_t flush_contrib(const hjx_problem *p, hjx_tape *t, void *lam, hipStream_t s)
{
    if (!t->pending) return hipSuccess;
    t->pending = false;
    if (p->scheme.dtype == HJX_F32) {
        AdjCombineArgs<float> c{};
        for (int d = 0; d < p->grid.dim; ++d) c.c[c.n++] = static_cast<const float *>(t->contrib[d]);
        return launch_combine_f32(static_cast<float *>(lam), c, (int)p->total, s);
    }
    AdjCombineArgs<double> c{};
    for (int d = 0; d < p->grid.dim; ++d) c.c[c.n++] = static_cast<const double *>(t->contrib[d]);
    return launch_combine_f64(static_cast<double *>(lam), c, (int)p->total, s);
}

hipError_t reverse_stage(const hjx_problem *p, hjx_tape *t, const void *in, const void *lam_out,
                         const unsigned char *mask, void *lam_target, void *lam_in, int in_mode, void *lam_n,
                         int n_mode, double ca, double cb, double h, int h_slot, const void *dp,
                         const ReplayStage *rep, hipStream_t s)
{
    if (p->scheme.dtype == HJX_F32)
        return reverse_stage_t<float>(p, t, in, lam_out, mask, lam_target, lam_in, in_mode, lam_n, n_mode, ca, cb,
                                      h, h_slot, dp, rep, s);
    return reverse_stage_t<double>(p, t, in, lam_out, mask, lam_target, lam_in, in_mode, lam_n, n_mode, ca, cb, h,
                                   h_slot, dp, rep, s);
}

hipError_t zero(const hjx_problem *p, void *x, hipStream_t s)
{
    if (p->scheme.dtype == HJX_F32) return launch_zero_f32(static_cast<float *>(x), (int)p->total, s);
    return launch_zero_f64(static_cast<double *>(x), (int)p->total, s);
}

}  // namespace

extern "C" {

hjx_status hjx_adjoint(hjx_problem *p, hjx_tape *t, const void *dL_dphiT, void *dL_dphi0, void *dL_dtarget,
                       double *dL_dparams, void *stream)
{
    TraceRange trace_("hjx_adjoint");
    if (!p || !t || !dL_dphiT || !dL_dphi0) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (t->p != p) return fail(HJX_ERR_INVALID_ARG, "the tape belongs to another problem");
    if (!t->solved) return fail(HJX_ERR_INVALID_ARG, "the tape holds no solve (call hjx_solve_taped first)");
    if (dL_dtarget && !t->target) return fail(HJX_ERR_INVALID_ARG, "dL_dtarget given but the solve had no target");
    if (std::memcmp(t->hp, p->ham.p, sizeof t->hp) != 0)
        return fail(HJX_ERR_INVALID_ARG, "the problem's parameters changed since the tape was made");
    // dL_dtarget == dL_dphi0: the gradient through phi0 when phi0 is also the
    // target, written as the sum of the two
    const bool summed = dL_dtarget && dL_dtarget == dL_dphi0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int rk = p->scheme.rk;
    // stage k of the forward step: out = ca phi_n + cb (in_k + h L(in_k))
    static const double kCa[3][3] = {{0, 0, 0}, {0, 0.5, 0}, {0, 0.75, 1.0 / 3.0}};
    static const double kCb[3][3] = {{1, 0, 0}, {1, 0.5, 0}, {1, 0.25, 2.0 / 3.0}};

    void *lbar = t->lam[0], *lnew = t->lam[1];
    t->pending = false;
    HIP_TRY(launch_copy(p, dL_dphiT, lbar, s));
    if (dL_dtarget) HIP_TRY(zero(p, dL_dtarget, s));
    HIP_TRY(launch_zero_f64acc(t->acc, kAccCount * t->acc_blocks, s));

    // The replay of segment seg - 1 only reads its checkpoint and writes the
    // other replay set, so it is independent of the reverse sweep of segment
    // seg: each reversed stage carries one of its forward stages in the
    // launch of its seed pass (memory-bound work beside arithmetic-bound
    // work), and the stages left over, if any, follow the sweep.  Only the
    // last segment's replay runs on its own.
    auto plan = [&](int seg) {
        std::vector<ReplayStage> v;
        const int64_t s0 = (int64_t)seg * t->K, s1 = std::min<int64_t>(t->steps, s0 + t->K);
        const int len = (int)(s1 - s0);
        hjx_tape::ReplaySet &R = t->rs[seg & 1];
        auto phin = [&](int i) -> void * { return i == 0 ? t->ckpt[seg] : R.phin[i]; };
        auto dp = [&](int i, int k) -> void * { return R.dp.empty() ? nullptr : R.dp[(size_t)i * rk + k]; };
        for (int i = 0; i < len; ++i) {
            const double h = s0 + i == t->steps - 1 ? t->dt_last : t->dt;
            if (rk == 1) {
                v.push_back({phin(i), nullptr, t->target, phin(i + 1), h, 0, 1, t->mask_of(R, i, 0), dp(i, 0)});
            } else if (rk == 2) {
                v.push_back({phin(i), nullptr, nullptr, R.x1[i], h, 0, 1, t->mask_of(R, i, 0), dp(i, 0)});
                v.push_back(
                    {R.x1[i], phin(i), t->target, phin(i + 1), h, 0.5, 0.5, t->mask_of(R, i, 1), dp(i, 1)});
            } else {
                v.push_back({phin(i), nullptr, nullptr, R.x1[i], h, 0, 1, t->mask_of(R, i, 0), dp(i, 0)});
                v.push_back({R.x1[i], phin(i), nullptr, R.xh[i], h, 0.75, 0.25, t->mask_of(R, i, 1), dp(i, 1)});
                v.push_back({R.xh[i], phin(i), t->target, phin(i + 1), h, 1.0 / 3.0, 2.0 / 3.0,
                             t->mask_of(R, i, 2), dp(i, 2)});
            }
        }
        return v;
    };
    if (t->nseg > 0) {
        TraceRange trace_rep("hjx_adjoint replay of segment %ld", (long)(t->nseg - 1));
        for (const ReplayStage &r : plan(t->nseg - 1)) HIP_TRY(replay_stage(p, t->alpha, r, s));
    }
    for (int seg = t->nseg - 1; seg >= 0; --seg) {
        TraceRange trace_seg("hjx_adjoint reverse segment %ld", (long)seg);
        const std::vector<ReplayStage> next = seg > 0 ? plan(seg - 1) : std::vector<ReplayStage>();
        size_t carried = 0;
        const int64_t s0 = (int64_t)seg * t->K, s1 = std::min<int64_t>(t->steps, s0 + t->K);
        const int len = (int)(s1 - s0);
        hjx_tape::ReplaySet &R = t->rs[seg & 1];
        auto phin = [&](int i) -> void * { return i == 0 ? t->ckpt[seg] : R.phin[i]; };
        auto dp = [&](int i, int k) -> void * { return R.dp.empty() ? nullptr : R.dp[(size_t)i * rk + k]; };
        // reverse steps
        for (int i = len - 1; i >= 0; --i) {
            const int64_t n = s0 + i;
            const double h = n == t->steps - 1 ? t->dt_last : t->dt;
            const int slot = n == t->steps - 1 ? kAccDhLast : kAccDhMain;
            const void *inputs[3] = {phin(i), rk >= 2 ? R.x1[i] : nullptr, rk >= 3 ? R.xh[i] : nullptr};
            bool n_written = false;
            const void *lout = lbar;
            void *stage_lam[2] = {t->lam[2], t->lam[3]};
            for (int k = rk - 1; k >= 0; --k) {
                const bool last = k == rk - 1;
                const unsigned char *mk = t->mask_of(R, i, k);
                void *ltgt = last && t->target ? dL_dtarget : nullptr;
                const double ca = kCa[rk - 1][k], cb = kCb[rk - 1][k];
                void *lin;
                int in_mode;
                if (k == 0) {
                    lin = lnew;
                    in_mode = n_written ? 1 : 0;
                } else {
                    lin = stage_lam[k & 1];
                    in_mode = 0;
                }
                int n_mode = 0;
                if (k != 0 && ca != 0.0) {
                    n_mode = n_written ? 2 : 1;
                    n_written = true;
                }
                const ReplayStage *rep = carried < next.size() ? &next[carried++] : nullptr;
                HIP_TRY(reverse_stage(p, t, inputs[k], lout, mk, ltgt, lin, in_mode, lnew, n_mode, ca, cb, h, slot,
                                      dp(i, k), rep, s));
                lout = lin;
            }
            std::swap(lbar, lnew);
        }
        for (; carried < next.size(); ++carried) HIP_TRY(replay_stage(p, t->alpha, next[carried], s));
    }
    HIP_TRY(flush_contrib(p, t, lbar, s));
    if (summed) {  // dL/dphi0 = dL/dtarget + lam at t0
        if (p->scheme.dtype == HJX_F32) {
            AdjCombineArgs<float> c{};
            c.c[c.n++] = static_cast<const float *>(lbar);
            HIP_TRY(launch_combine_f32(static_cast<float *>(dL_dphi0), c, (int)p->total, s));
        } else {
            AdjCombineArgs<double> c{};
            c.c[c.n++] = static_cast<const double *>(lbar);
            HIP_TRY(launch_combine_f64(static_cast<double *>(dL_dphi0), c, (int)p->total, s));
        }
    } else {
        HIP_TRY(launch_copy(p, lbar, dL_dphi0, s));
    }

    HIP_TRY(launch_acc_reduce(t->acc, t->acc_blocks, t->acc_out, s));
    HIP_TRY(hipMemcpyAsync(t->hacc, t->acc_out, sizeof(double) * kAccCount, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (dL_dparams) {
        // the step size depends on alpha: dt = cfl / sum_d alpha_d / dx_d for
        // every step but the last, which is t1 - t0 - (N-1) dt
        double ddt = 0.0;
        if (std::isfinite(t->dt) && t->steps > 0)
            ddt = t->hacc[kAccDhMain] - (double)(t->steps - 1) * t->hacc[kAccDhLast];
        double J[kMaxDim][8];
        alpha_jacobian(p, J);
        for (int m = 0; m < 8; ++m) {
            double gsum = t->hacc[kAccTheta + m];
            for (int d = 0; d < p->grid.dim; ++d) {
                double dalpha = t->hacc[kAccAlpha + d];
                if (std::isfinite(t->dt))
                    dalpha += ddt * (-t->dt * t->dt / (p->scheme.cfl * p->dx[d]));
                gsum += dalpha * J[d][m];
            }
            dL_dparams[m] = m < n_params(p->ham.kind) ? gsum : 0.0;
        }
    }
    return ok();
}

hjx_status hjx_loss_volume(hjx_problem *p, const void *phi, double eps, double *loss, void *dL_dphi, void *stream)
{
    if (!p || !phi || !loss) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(HJX_ERR_INVALID_ARG, "eps %g is not positive", eps);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double vol = 1.0;
    for (int d = 0; d < p->grid.dim; ++d) vol *= p->dx[d];
    const int blocks = alpha_blocks((int)p->total);
    double *partial = p->dalpha + kMaxDim;
    if (p->scheme.dtype == HJX_F32)
        HIP_TRY(launch_loss_f32(static_cast<const float *>(phi), (int)p->total, eps, vol, static_cast<float *>(dL_dphi),
                                partial, blocks, p->dalpha, s));
    else
        HIP_TRY(launch_loss_f64(static_cast<const double *>(phi), (int)p->total, eps, vol,
                                static_cast<double *>(dL_dphi), partial, blocks, p->dalpha, s));
    HIP_TRY(hipMemcpyAsync(p->hbuf, p->dalpha, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *loss = p->hbuf[0];
    return ok();
}

}  // extern "C"

// ==================================================================== batch (host)

struct hjx_batch {
    int n = 0;
    int device = 0;
    int dtype = 0, deriv = 0, rk = 0;
    int clip = 0;                     // some member has a restricted update
    int ext = 0;                      // some member plays the rockets game or takes the local form or Godunov
    size_t elem = 0, inst_bytes = 0;
    std::vector<hjx_problem *> probs;
    std::vector<double> alpha;        // n * kMaxDim
    std::vector<double> hp;           // n * 8: each member's parameters at create
    std::vector<double> dt;           // CFL step of each problem
    void *dinst = nullptr;            // device descriptors (sorted order)
    void *hinst = nullptr;            // pinned host copy
    int *dflag = nullptr;             // device, per sorted instance
    int *hflag = nullptr;             // pinned
    int item_nodes = 1024, blocks = 0, blocks_max = 0;
    // schedule behind the captured graph
    std::vector<int64_t> steps;       // per problem
    std::vector<double> dt_last;      // per problem
    std::vector<int> order;           // sorted position -> problem
    std::vector<int> item0;           // sorted position -> first item; n+1 entries
    int64_t max_steps = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_ok = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace {

constexpr int64_t kBatchMaxSteps = 1 << 20;

void batch_drop_graph(hjx_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ok = false;
}

void batch_release(hjx_batch *b)
{
    if (!b) return;
    batch_drop_graph(b);
    if (b->dinst) (void)hipFree(b->dinst);
    if (b->hinst) (void)hipHostFree(b->hinst);
    if (b->dflag) (void)hipFree(b->dflag);
    if (b->hflag) (void)hipHostFree(b->hflag);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

// one whole-batch or stage launch
hipError_t batch_launch(const hjx_batch *b, int n_active, int s, int stage, hipStream_t st)
{
    const int items = b->item0[n_active];
    if (b->dtype == HJX_F32) {
        BatchArgs<float> a{static_cast<const BatchInst<float> *>(b->dinst), b->dflag, n_active, items, s, stage,
                           b->rk, b->item_nodes, b->clip, b->ext};
        return launch_batch_f32(a, b->deriv, b->blocks, st);
    }
    BatchArgs<double> a{static_cast<const BatchInst<double> *>(b->dinst), b->dflag, n_active, items, s, stage,
                        b->rk, b->item_nodes, b->clip, b->ext};
    return launch_batch_f64(a, b->deriv, b->blocks, st);
}

// the launches of one horizon: copy in, rk stages of every global step over
// the instances still active, copy out (RK1)
hipError_t batch_enqueue(const hjx_batch *b, hipStream_t st)
{
    hipError_t e = batch_launch(b, b->n, 0, kBatchCopyIn, st);
    int active = b->n;
    for (int64_t s = 0; s < b->max_steps && e == hipSuccess; ++s) {
        while (active > 0 && b->steps[b->order[active - 1]] <= s) --active;
        for (int k = 0; k < b->rk && e == hipSuccess; ++k) e = batch_launch(b, active, (int)s, k, st);
    }
    if (e == hipSuccess && b->rk == 1) e = batch_launch(b, b->n, 0, kBatchCopyOut, st);
    return e;
}

hjx_status batch_build_graph(hjx_batch *b)
{
    batch_drop_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const hipError_t e = batch_enqueue(b, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(HJX_ERR_DEVICE, "batch graph capture: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_ok = true;
    return HJX_OK;
}

template <typename T>
void batch_descriptors(hjx_batch *b, const void *const *phi0, const void *const *target, void *const *phi_out)
{
    BatchInst<T> *I = static_cast<BatchInst<T> *>(b->hinst);
    for (int k = 0; k < b->n; ++k) {
        const int i = b->order[k];
        const hjx_problem *p = b->probs[i];
        BatchInst<T> x{};
        x.st = stage_args<T>(p, &b->alpha[(size_t)i * kMaxDim]);
        x.phi0 = static_cast<const T *>(phi0[i]);
        x.target = target ? static_cast<const T *>(target[i]) : nullptr;
        x.phi = static_cast<T *>(phi_out[i]);
        x.ws0 = static_cast<T *>(p->ws[0]);
        x.ws1 = static_cast<T *>(p->ws[1]);
        x.dt = T(b->dt[i]);
        x.dt_last = T(b->dt_last[i]);
        x.steps = (int)b->steps[i];
        x.ham = p->ham.kind;
        x.total = (int)p->total;
        x.item0 = b->item0[k];
        I[k] = x;
    }
}

// the schedule of every instance for horizons t1; (re)builds the order,
// the work list and the graph when they change
hjx_status batch_schedule(hjx_batch *b, const double *t1)
{
    std::vector<int64_t> steps(b->n);
    std::vector<double> last(b->n);
    int64_t mx = 0;
    for (int i = 0; i < b->n; ++i) {
        if (!std::isfinite(t1[i]) || !(t1[i] >= 0.0))
            return fail(HJX_ERR_INVALID_ARG, "t1[%d] = %g is not finite and >= 0", i, t1[i]);
        if (t1[i] > 0.0 && (double)kBatchMaxSteps * b->dt[i] < t1[i])
            return fail(HJX_ERR_UNSUPPORTED, "instance %d needs more than %lld steps", i, (long long)kBatchMaxSteps);
        schedule(0.0, t1[i], b->dt[i], &steps[i], &last[i]);
        mx = std::max(mx, steps[i]);
    }
    b->dt_last = last;
    if (b->graph_ok && steps == b->steps) return HJX_OK;
    b->steps = steps;
    b->max_steps = mx;
    b->order.resize(b->n);
    for (int i = 0; i < b->n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return steps[x] > steps[y]; });
    b->item0.assign(b->n + 1, 0);
    int64_t acc = 0;
    for (int k = 0; k < b->n; ++k) {
        b->item0[k] = (int)acc;
        acc += (b->probs[b->order[k]]->total + b->item_nodes - 1) / b->item_nodes;
    }
    if (acc > INT32_MAX) return fail(HJX_ERR_UNSUPPORTED, "batch work list too long");
    b->item0[b->n] = (int)acc;
    return batch_build_graph(b);
}

// flags of the last check -> first bad problem index or -1; synchronises
hjx_status batch_check(hjx_batch *b, int mode, hipStream_t s, int *first_bad)
{
    HIP_TRY(hipMemsetAsync(b->dflag, 0, sizeof(int) * b->n, s));
    HIP_TRY(batch_launch(b, b->n, 0, mode, s));
    HIP_TRY(hipMemcpyAsync(b->hflag, b->dflag, sizeof(int) * b->n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *first_bad = -1;
    for (int k = 0; k < b->n; ++k)
        if (b->hflag[k] && (*first_bad < 0 || b->order[k] < *first_bad)) *first_bad = b->order[k];
    return HJX_OK;
}

}  // namespace

extern "C" {

hjx_status hjx_batch_create(int32_t n, hjx_problem *const *problems, void *stream, hjx_batch **out)
{
    if (!out) return fail(HJX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !problems) return fail(HJX_ERR_INVALID_ARG, "need n >= 1 problems");
    for (int i = 0; i < n; ++i)
        if (!problems[i]) return fail(HJX_ERR_INVALID_ARG, "problems[%d] is NULL", i);
    const hjx_problem *p0 = problems[0];
    {
        std::vector<const hjx_problem *> seen(problems, problems + n);
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            return fail(HJX_ERR_INVALID_ARG, "a problem appears twice in the batch");
    }
    for (int i = 0; i < n; ++i) {
        const hjx_problem *p = problems[i];
        if (p->scheme.dtype != p0->scheme.dtype || p->scheme.deriv != p0->scheme.deriv ||
            p->scheme.rk != p0->scheme.rk)
            return fail(HJX_ERR_INVALID_ARG, "problems[%d]: every problem of a batch needs the same dtype, "
                        "derivative scheme and RK order", i);
        if (p->device != p0->device) return fail(HJX_ERR_INVALID_ARG, "problems[%d] is on another device", i);
        if (!direct_ok(geometry(p), p->elem))
            return fail(HJX_ERR_UNSUPPORTED, "problems[%d]: arrays of 4 GiB or more", i);
    }
    {
        const size_t need = (p0->scheme.dtype == HJX_F32 ? sizeof(BatchInst<float>) : sizeof(BatchInst<double>)) *
                                (size_t)n + sizeof(int) * (size_t)n;
        size_t cap = 0;
        if (over_workspace_cap(need, &cap))
            return fail(HJX_ERR_OOM, "batch workspace of %zu bytes exceeds HJX_MAX_WORKSPACE=%zu", need, cap);
    }
    hjx_batch *b = new (std::nothrow) hjx_batch;
    if (!b) return fail(HJX_ERR_OOM, "host allocation failed");
    b->n = n;
    b->device = p0->device;
    b->dtype = p0->scheme.dtype;
    b->deriv = p0->scheme.deriv;
    b->rk = p0->scheme.rk;
    for (int i = 0; i < n; ++i) {
        b->clip |= problems[i]->scheme.restrict_update != HJX_RESTRICT_NONE;
        b->ext |= problems[i]->ham.kind == HJX_HAM_ROCKETS || problems[i]->ham.dissipation != HJX_DISS_GLOBAL;
    }
    b->elem = p0->elem;
    b->inst_bytes = b->dtype == HJX_F32 ? sizeof(BatchInst<float>) : sizeof(BatchInst<double>);
    b->probs.assign(problems, problems + n);
    b->alpha.assign((size_t)n * kMaxDim, 0.0);
    b->hp.assign((size_t)n * 8, 0.0);
    for (int i = 0; i < n; ++i) std::memcpy(&b->hp[(size_t)i * 8], problems[i]->ham.p, sizeof(double) * 8);
    b->dt.assign(n, 0.0);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) {
        hjx_status st = device_alpha(b->probs[i], s, &b->alpha[(size_t)i * kMaxDim]);
        if (st != HJX_OK) {
            batch_release(b);
            return st;
        }
        b->dt[i] = cfl_dt(b->probs[i], &b->alpha[(size_t)i * kMaxDim]);
    }
    int cus = 0;
    hipError_t e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device)) != hipSuccess ||
        (e = hipMalloc(&b->dinst, b->inst_bytes * n)) != hipSuccess ||
        (e = hipHostMalloc(&b->hinst, b->inst_bytes * n, hipHostMallocDefault)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void **>(&b->dflag), sizeof(int) * n)) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&b->hflag), sizeof(int) * n, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreate(&b->ev[0])) != hipSuccess || (e = hipEventCreate(&b->ev[1])) != hipSuccess) {
        batch_release(b);
        return fail(e == hipErrorOutOfMemory ? HJX_ERR_OOM : HJX_ERR_DEVICE, "batch allocation: %s",
                    hipGetErrorString(e));
    }
    const int per_cu = batch_blocks_per_cu(b->dtype == HJX_F64, b->deriv, b->clip, b->ext);
    b->blocks_max = std::max(1, cus) * per_cu;
    b->blocks = b->blocks_max;
    *out = b;
    return ok();
}

hjx_status hjx_batch_destroy(hjx_batch *b)
{
    batch_release(b);
    return ok();
}

hjx_status hjx_batch_set_shape(hjx_batch *b, int32_t item_nodes, int32_t blocks)
{
    if (!b) return fail(HJX_ERR_INVALID_ARG, "NULL batch");
    if (item_nodes < 256 || item_nodes > (1 << 20) || item_nodes % 256)
        return fail(HJX_ERR_INVALID_ARG, "item_nodes %d: a multiple of 256 in [256, 2^20]", item_nodes);
    if (blocks < 1 || blocks > b->blocks_max)
        return fail(HJX_ERR_INVALID_ARG, "blocks %d: in [1, %d] (resident blocks)", blocks, b->blocks_max);
    if (item_nodes != b->item_nodes || blocks != b->blocks) batch_drop_graph(b);
    b->item_nodes = item_nodes;
    b->blocks = blocks;
    return ok();
}

hjx_status hjx_batch_get_shape(const hjx_batch *b, int32_t *item_nodes, int32_t *blocks, int32_t *blocks_max)
{
    if (!b) return fail(HJX_ERR_INVALID_ARG, "NULL batch");
    if (item_nodes) *item_nodes = b->item_nodes;
    if (blocks) *blocks = b->blocks;
    if (blocks_max) *blocks_max = b->blocks_max;
    return ok();
}

hjx_status hjx_batch_solve(hjx_batch *b, const void *const *phi0, const void *const *target, void *const *phi_out,
                           const double *t1, void *stream, hjx_stats *stats)
{
    TraceRange trace_("hjx_batch_solve");
    if (!b || !phi0 || !phi_out || !t1) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i < b->n; ++i) {
        if (!phi0[i] || !phi_out[i]) return fail(HJX_ERR_INVALID_ARG, "phi0[%d] or phi_out[%d] is NULL", i, i);
        if (target && target[i] && target[i] == phi_out[i])
            return fail(HJX_ERR_INVALID_ARG, "target[%d] aliases phi_out[%d]", i, i);
        if (std::memcmp(&b->hp[(size_t)i * 8], b->probs[i]->ham.p, sizeof(double) * 8) != 0)
            return fail(HJX_ERR_INVALID_ARG, "member %d's parameters changed since the batch was made", i);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hjx_status st = batch_schedule(b, t1);
    if (st != HJX_OK) return st;
    if (b->dtype == HJX_F32) batch_descriptors<float>(b, phi0, target, phi_out);
    else batch_descriptors<double>(b, phi0, target, phi_out);
    HIP_TRY(hipMemcpyAsync(b->dinst, b->hinst, b->inst_bytes * b->n, hipMemcpyHostToDevice, s));

    int bad = -1;
    if ((st = batch_check(b, kBatchCheckIn, s, &bad)) != HJX_OK) return st;
    if (bad >= 0) return fail(HJX_ERR_NONFINITE, "phi0[%d] holds NaN or Inf", bad);

    HIP_TRY(hipEventRecord(b->ev[0], s));
    HIP_TRY(hipGraphLaunch(b->exec, s));
    HIP_TRY(hipEventRecord(b->ev[1], s));

    if ((st = batch_check(b, kBatchCheckOut, s, &bad)) != HJX_OK) return st;
    if (stats) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
        for (int i = 0; i < b->n; ++i) {
            const hjx_problem *p = b->probs[i];
            hjx_stats &x = stats[i];
            x.steps = b->steps[i];
            x.dt = b->dt[i];
            x.dt_last = b->steps[i] ? b->dt_last[i] : 0.0;
            x.t_final = t1[i];
            for (int d = 0; d < kMaxDim; ++d) x.alpha[d] = b->alpha[(size_t)i * kMaxDim + d];
            x.elapsed_ms = ms;  // the whole batch
            const double f = (double)p->total * (double)p->elem;
            double per_step = b->rk == 1 ? 2.0 : (b->rk == 2 ? 5.0 : 8.0);
            if (target && target[i]) per_step += 1.0;
            x.alg_bytes = per_step * f * (double)b->steps[i];
        }
    }
    if (bad >= 0) return fail(HJX_ERR_NONFINITE, "the solution of instance %d holds NaN or Inf", bad);
    return ok();
}

hjx_status hjx_batch_tune(hjx_batch *b, const void *const *phi0, const void *const *target, void *const *phi_out,
                          const double *t1, int32_t reps, void *stream, double *best_ms)
{
    TraceRange trace_("hjx_batch_tune");
    if (!b) return fail(HJX_ERR_INVALID_ARG, "NULL batch");
    if (reps < 1) return fail(HJX_ERR_INVALID_ARG, "reps must be >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cus =
        std::max(1, b->blocks_max / std::max(1, batch_blocks_per_cu(b->dtype == HJX_F64, b->deriv, b->clip, b->ext)));
    std::vector<std::pair<int, int>> cand;
    for (int items : {256, 1024, 4096}) {
        for (int per_cu : {1, 2, 4}) {
            const int blocks = per_cu * cus;
            if (blocks < b->blocks_max) cand.push_back({items, blocks});
        }
        cand.push_back({items, b->blocks_max});
    }
    if (cand.empty()) cand.push_back({b->item_nodes, b->blocks_max});
    const bool verbose = std::getenv("HJX_TUNE_VERBOSE") != nullptr;
    double best = INFINITY;
    std::pair<int, int> win = cand[0];
    for (const auto &c : cand) {
        hjx_status st = hjx_batch_set_shape(b, c.first, c.second);
        if (st != HJX_OK) return st;
        if ((st = hjx_batch_solve(b, phi0, target, phi_out, t1, stream, nullptr)) != HJX_OK) return st;  // capture
        double total = 0.0;
        for (int r = 0; r < reps; ++r) {
            HIP_TRY(hipEventRecord(b->ev[0], s));
            HIP_TRY(hipGraphLaunch(b->exec, s));
            HIP_TRY(hipEventRecord(b->ev[1], s));
            HIP_TRY(hipEventSynchronize(b->ev[1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
            total += ms;
        }
        const double mean = total / reps;
        if (verbose) std::fprintf(stderr, "hjx_batch_tune items=%d blocks=%d: %.3f ms\n", c.first, c.second, mean);
        if (mean < best) {
            best = mean;
            win = c;
        }
    }
    hjx_status st = hjx_batch_set_shape(b, win.first, win.second);
    if (st != HJX_OK) return st;
    if (best_ms) *best_ms = best;
    return ok();
}

}  // extern "C"

// ==================================================================== conservation laws

struct hjx_claw {
    hjx_grid_desc grid{};
    int flux = 0, dtype = 0;
    double c[kMaxDim] = {0, 0, 0, 0};
    double cfl = 0.0;
    double dx[kMaxDim] = {0, 0, 0, 0};
    int64_t total = 0;
    size_t elem = 0;
    int device = 0;
    void *tmp = nullptr;                  // work array of the grid's size
    unsigned long long *dmax = nullptr;   // device: max |v| (double bits), then the NaN/Inf flag
    unsigned long long *hmax = nullptr;   // pinned host copy
};

namespace {

void claw_release(hjx_claw *h)
{
    if (!h) return;
    if (h->tmp) (void)hipFree(h->tmp);
    if (h->dmax) (void)hipFree(h->dmax);
    if (h->hmax) (void)hipHostFree(h->hmax);
    delete h;
}

template <typename T>
ClawArgs<T> claw_args(const hjx_claw *h, const void *v, void *out, double dt)
{
    ClawArgs<T> a{};
    a.v = static_cast<const T *>(v);
    a.out = static_cast<T *>(out);
    a.dim = h->grid.dim;
    int st = 1;
    for (int d = h->grid.dim - 1; d >= 0; --d) {
        a.n[d] = (int)h->grid.n[d];
        a.stride[d] = st;
        st *= a.n[d];
    }
    a.periodic = h->grid.periodic_mask;
    a.rows = (int)(h->total / h->grid.n[h->grid.dim - 1]);
    for (int d = 0; d < h->grid.dim; ++d) {
        a.c[d] = T(h->c[d]);
        a.half_lam[d] = T(dt / h->dx[d] / 2.0);
    }
    a.inv_2n = T(1.0 / (2.0 * h->grid.dim));
    return a;
}

hipError_t claw_launch(const hjx_claw *h, const void *v, void *out, double dt, hipStream_t s)
{
    if (h->dtype == HJX_F32) return launch_claw_f32(claw_args<float>(h, v, out, dt), h->flux, s);
    return launch_claw_f64(claw_args<double>(h, v, out, dt), h->flux, s);
}

// max |v| over the grid (synchronises s)
hjx_status claw_maxabs(hjx_claw *h, const void *v, hipStream_t s, double *out)
{
    if (h->dtype == HJX_F32)
        HIP_TRY(launch_maxabs_f32(static_cast<const float *>(v), (int)h->total, h->dmax, s));
    else
        HIP_TRY(launch_maxabs_f64(static_cast<const double *>(v), (int)h->total, h->dmax, s));
    HIP_TRY(hipMemcpyAsync(h->hmax, h->dmax, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(out, h->hmax, sizeof(double));
    return HJX_OK;
}

// whether v holds NaN or Inf (synchronises s)
hjx_status claw_nonfinite(hjx_claw *h, const void *v, hipStream_t s, bool *bad)
{
    int *flag = reinterpret_cast<int *>(h->dmax + 1);
    HIP_TRY(launch_zero_f64acc(reinterpret_cast<double *>(h->dmax + 1), 1, s));
    if (h->dtype == HJX_F32)
        HIP_TRY(launch_nonfinite_f32(static_cast<const float *>(v), (int)h->total, flag, s));
    else
        HIP_TRY(launch_nonfinite_f64(static_cast<const double *>(v), (int)h->total, flag, s));
    HIP_TRY(hipMemcpyAsync(h->hmax + 1, h->dmax + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int host_flag = 0;
    std::memcpy(&host_flag, h->hmax + 1, sizeof(int));
    *bad = host_flag != 0;
    return HJX_OK;
}

hjx_status claw_dt(hjx_claw *h, const void *v, hipStream_t s, double *dt)
{
    double vmax = 1.0;
    if (h->flux == HJX_FLUX_BURGERS) {
        hjx_status st = claw_maxabs(h, v, s, &vmax);
        if (st != HJX_OK) return st;
    }
    double best = INFINITY;
    for (int d = 0; d < h->grid.dim; ++d) {
        const double speed = std::fabs(h->c[d]) * vmax;
        if (speed > 0) best = std::min(best, h->cfl * h->dx[d] / ((double)h->grid.dim * speed));
    }
    *dt = best;
    return HJX_OK;
}

}  // namespace

extern "C" {

hjx_status hjx_claw_create(const hjx_grid_desc *grid, int32_t flux, const double *c, int32_t dtype, double cfl,
                           hjx_claw **out)
{
    if (!out) return fail(HJX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !c) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    hjx_status st = validate_grid(grid);
    if (st != HJX_OK) return st;
    if (flux != HJX_FLUX_LINEAR && flux != HJX_FLUX_BURGERS) return fail(HJX_ERR_INVALID_ARG, "unknown flux %d", flux);
    for (int d = 0; d < grid->dim; ++d)
        if (!std::isfinite(c[d])) return fail(HJX_ERR_INVALID_ARG, "flux coefficient %d is not finite", d);
    if (!(cfl > 0.0) || !(cfl <= 1.0)) return fail(HJX_ERR_INVALID_ARG, "cfl %g outside (0, 1]", cfl);
    if (dtype != HJX_F32 && dtype != HJX_F64) return fail(HJX_ERR_INVALID_ARG, "unknown dtype %d", dtype);

    hjx_claw *h = new (std::nothrow) hjx_claw;
    if (!h) return fail(HJX_ERR_OOM, "host allocation failed");
    h->grid = *grid;
    h->flux = flux;
    h->dtype = dtype;
    h->cfl = cfl;
    h->total = 1;
    for (int d = 0; d < grid->dim; ++d) {
        h->c[d] = c[d];
        h->total *= grid->n[d];
        const double len = grid->gmax[d] - grid->gmin[d];
        h->dx[d] = ((grid->periodic_mask >> d) & 1u) ? len / (double)grid->n[d] : len / (double)(grid->n[d] - 1);
    }
    h->elem = dtype == HJX_F32 ? sizeof(float) : sizeof(double);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        claw_release(h);
        return fail(HJX_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    const size_t need = (size_t)h->total * h->elem;
    size_t cap = 0;
    if (over_workspace_cap(need, &cap)) {
        claw_release(h);
        return fail(HJX_ERR_OOM, "work array of %zu bytes exceeds HJX_MAX_WORKSPACE=%zu", need, cap);
    }
    if ((e = hipMalloc(&h->tmp, need)) != hipSuccess || (e = hipMalloc(&h->dmax, 2 * sizeof(unsigned long long))) !=
                                                                hipSuccess ||
        (e = hipHostMalloc(&h->hmax, 2 * sizeof(unsigned long long))) != hipSuccess) {
        claw_release(h);
        return fail(e == hipErrorOutOfMemory ? HJX_ERR_OOM : HJX_ERR_DEVICE, "allocation: %s", hipGetErrorString(e));
    }
    *out = h;
    return ok();
}

hjx_status hjx_claw_destroy(hjx_claw *h)
{
    claw_release(h);
    return ok();
}

hjx_status hjx_claw_dt(hjx_claw *h, const void *v, double *dt_out, void *stream)
{
    if (!h || !dt_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (!v && h->flux == HJX_FLUX_BURGERS) return fail(HJX_ERR_INVALID_ARG, "v is NULL (the Burgers flux needs it)");
    hjx_status st = claw_dt(h, v, static_cast<hipStream_t>(stream), dt_out);
    return st != HJX_OK ? st : ok();
}

hjx_status hjx_claw_step(hjx_claw *h, const void *v, void *v_out, double dt, void *stream)
{
    if (!h || !v || !v_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (v == v_out) return fail(HJX_ERR_INVALID_ARG, "v_out aliases v");
    if (!std::isfinite(dt) || dt < 0) return fail(HJX_ERR_INVALID_ARG, "dt %g is not finite and >= 0", dt);
    HIP_TRY(claw_launch(h, v, v_out, dt, static_cast<hipStream_t>(stream)));
    return ok();
}

hjx_status hjx_claw_solve(hjx_claw *h, const void *v0, void *v_out, double t1, void *stream, int64_t *steps_out,
                          double *dt_out)
{
    if (!h || !v0 || !v_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (v0 == v_out) return fail(HJX_ERR_INVALID_ARG, "v_out aliases v0");
    if (!std::isfinite(t1) || t1 < 0) return fail(HJX_ERR_INVALID_ARG, "t1 %g is not finite and >= 0", t1);
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool bad = false;
    hjx_status st = claw_nonfinite(h, v0, s, &bad);
    if (st != HJX_OK) return st;
    if (bad) return fail(HJX_ERR_NONFINITE, "v0 holds NaN or Inf");
    double dt = 0.0;
    if ((st = claw_dt(h, v0, s, &dt)) != HJX_OK) return st;

    // the step sizes first, so that the ping-pong between v_out and the work
    // array ends in v_out
    std::vector<double> hs;
    const double slack = 1e-12 * (std::fabs(t1) > 1.0 ? std::fabs(t1) : 1.0);
    for (double t = 0.0; t < t1;) {
        double step = dt;
        bool last = false;
        if (t + step >= t1 - slack) {
            step = t1 - t;
            last = true;
        }
        hs.push_back(step);
        t = last ? t1 : t + step;
    }
    const size_t n = hs.size();
    if (n == 0) {
        HIP_TRY(hipMemcpyAsync(v_out, v0, (size_t)h->total * h->elem, hipMemcpyDeviceToDevice, s));
    }
    const void *src = v0;
    for (size_t k = 0; k < n; ++k) {
        void *dst = ((n - k) & 1) ? v_out : h->tmp;
        HIP_TRY(claw_launch(h, src, dst, hs[k], s));
        src = dst;
    }
    if ((st = claw_nonfinite(h, v_out, s, &bad)) != HJX_OK) return st;
    if (steps_out) *steps_out = (int64_t)n;
    if (dt_out) *dt_out = dt;
    if (bad) return fail(HJX_ERR_NONFINITE, "the solution holds NaN or Inf");
    return ok();
}

}  // extern "C"

// ==================================================================== shapes

namespace {

// validate one shape on one grid and fill its kernel arguments
hjx_status shape_args(const hjx_grid_desc *grid, const hjx_shape_desc *shape, ShapeArgs *out)
{
    hjx_status st = validate_grid(grid);
    if (st != HJX_OK) return st;
    if (shape->kind != HJX_SHAPE_BALL && shape->kind != HJX_SHAPE_ELLIPSOID)
        return fail(HJX_ERR_INVALID_ARG, "unknown shape kind %d", shape->kind);
    if (shape->axis_mask == 0 || (shape->axis_mask >> grid->dim))
        return fail(HJX_ERR_INVALID_ARG, "axis_mask 0x%x names no axis or an axis >= dim %d", shape->axis_mask,
                    grid->dim);
    if (!std::isfinite(shape->radius)) return fail(HJX_ERR_INVALID_ARG, "radius is not finite");
    ShapeArgs a{};
    a.dim = grid->dim;
    a.kind = shape->kind;
    a.mask = shape->axis_mask;
    a.total = 1;
    for (int d = 0; d < grid->dim; ++d) {
        if (!std::isfinite(shape->center[d]) || (shape->kind == HJX_SHAPE_ELLIPSOID && !std::isfinite(shape->weights[d])))
            return fail(HJX_ERR_INVALID_ARG, "center or weight %d is not finite", d);
        a.n[d] = (int)grid->n[d];
        a.total *= a.n[d];
        const double len = grid->gmax[d] - grid->gmin[d];
        a.gmin[d] = grid->gmin[d];
        a.dx[d] = ((grid->periodic_mask >> d) & 1u) ? len / (double)grid->n[d] : len / (double)(grid->n[d] - 1);
        a.center[d] = shape->center[d];
        a.weights[d] = shape->weights[d];
    }
    a.radius = shape->radius;
    a.rows = (int)(a.total / a.n[grid->dim - 1]);
    *out = a;
    return HJX_OK;
}

}  // namespace

extern "C" {

hjx_status hjx_shape(const hjx_grid_desc *grid, const hjx_shape_desc *shape, int32_t dtype, void *phi_out,
                     void *stream)
{
    if (!grid || !shape || !phi_out) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (dtype != HJX_F32 && dtype != HJX_F64) return fail(HJX_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    ShapeArgs a{};
    hjx_status st = shape_args(grid, shape, &a);
    if (st != HJX_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == HJX_F32) HIP_TRY(launch_shape_f32(a, static_cast<float *>(phi_out), s));
    else HIP_TRY(launch_shape_f64(a, static_cast<double *>(phi_out), s));
    return ok();
}

hjx_status hjx_shape_batch(int32_t n, const hjx_grid_desc *grids, const hjx_shape_desc *shapes, int32_t dtype,
                           void *const *phi_out, void *stream)
{
    if (n < 1 || n > 65535 || !grids || !shapes || !phi_out)
        return fail(HJX_ERR_INVALID_ARG, "need 1 <= n <= 65535 and no NULL array");
    if (dtype != HJX_F32 && dtype != HJX_F64) return fail(HJX_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    std::vector<ShapeMember> host((size_t)n);
    long largest = 0;
    for (int k = 0; k < n; ++k) {
        if (!phi_out[k]) return fail(HJX_ERR_INVALID_ARG, "phi_out[%d] is NULL", k);
        hjx_status st = shape_args(&grids[k], &shapes[k], &host[k].a);
        if (st != HJX_OK) return fail(st, "member %d: %s", k, hjx_last_error());
        host[k].out = phi_out[k];
        largest = std::max(largest, host[k].a.total);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ShapeMember *dev = nullptr;
    HIP_TRY(hipMalloc(&dev, host.size() * sizeof(ShapeMember)));
    hipError_t e = hipMemcpyAsync(dev, host.data(), host.size() * sizeof(ShapeMember), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = dtype == HJX_F32 ? launch_shape_batch_f32(dev, n, largest, s) : launch_shape_batch_f64(dev, n, largest, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dev);
    if (e != hipSuccess) return fail(HJX_ERR_DEVICE, "hjx_shape_batch: %s", hipGetErrorString(e));
    return ok();
}

hjx_status hjx_shape_batch_noalloc(int32_t n, const hjx_grid_desc *grids, const hjx_shape_desc *shapes,
                                   int32_t dtype, void *const *phi_out, void *stream)
{
    static_assert(HJX_SHAPE_NOALLOC_MAX == kShapeNoAllocMax, "the header states the array's size");
    if (n < 1 || n > HJX_SHAPE_NOALLOC_MAX)
        return fail(HJX_ERR_INVALID_ARG, "n = %d outside [1, %d], the size of the fixed descriptor array", n,
                    HJX_SHAPE_NOALLOC_MAX);
    if (!grids || !shapes || !phi_out) return fail(HJX_ERR_INVALID_ARG, "NULL array");
    if (dtype != HJX_F32 && dtype != HJX_F64) return fail(HJX_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    // host staging in static storage too: the call allocates nothing anywhere;
    // one call at a time per process holds it and the device array
    static std::mutex mu;
    static ShapeMember host[kShapeNoAllocMax];
    std::lock_guard<std::mutex> lock(mu);
    long largest = 0;
    for (int k = 0; k < n; ++k) {
        if (!phi_out[k]) return fail(HJX_ERR_INVALID_ARG, "phi_out[%d] is NULL", k);
        hjx_status st = shape_args(&grids[k], &shapes[k], &host[k].a);
        if (st != HJX_OK) return fail(st, "member %d: %s", k, hjx_last_error());
        host[k].out = phi_out[k];
        largest = std::max(largest, host[k].a.total);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ShapeMember *dev = nullptr;
    HIP_TRY(shape_noalloc_scratch(&dev));
    HIP_TRY(hipMemcpyAsync(dev, host, (size_t)n * sizeof(ShapeMember), hipMemcpyHostToDevice, s));
    HIP_TRY(dtype == HJX_F32 ? launch_shape_batch_f32(dev, n, largest, s) : launch_shape_batch_f64(dev, n, largest, s));
    HIP_TRY(hipStreamSynchronize(s));
    return ok();
}

hjx_status hjx_shape_op(int32_t op, int32_t dtype, const void *a, const void *b, void *out, int64_t n, void *stream)
{
    if (op < HJX_OP_UNION || op > HJX_OP_SUBTRACTION) return fail(HJX_ERR_INVALID_ARG, "unknown shape op %d", op);
    if (!a || !out || (op != HJX_OP_COMPLEMENT && !b)) return fail(HJX_ERR_INVALID_ARG, "NULL argument");
    if (dtype != HJX_F32 && dtype != HJX_F64) return fail(HJX_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if (n < 0) return fail(HJX_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0) return ok();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (op == HJX_OP_COMPLEMENT) b = a;  // unused by the kernel
    if (dtype == HJX_F32)
        HIP_TRY(launch_shape_op_f32(op, static_cast<const float *>(a), static_cast<const float *>(b),
                                    static_cast<float *>(out), (long)n, s));
    else
        HIP_TRY(launch_shape_op_f64(op, static_cast<const double *>(a), static_cast<const double *>(b),
                                    static_cast<double *>(out), (long)n, s));
    return ok();
}

}  // extern "C"
