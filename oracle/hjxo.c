/*
 * hjxo -- plain, slow FP64 CPU oracle for explicit Hamilton-Jacobi level-set
 * time stepping (LevelSetPy, arXiv 2411.03501).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no source with the HIP
 * library: it builds its own grid, coordinate tables, ghost values, stencils,
 * Hamiltonians, reductions and integrator, written straight from the paper.
 *
 * What is computed, and where the paper defines it:
 *   grid and spacing ............. Sec. III-B (grid layout, Listing 1)
 *   ghost cells .................. Sec. III-B item (iv) (periodic; otherwise
 *                                  linear extrapolation -- the paper does not
 *                                  state the non-periodic rule)
 *   one-sided differences ........ Sec. IV, eq. (fwd_bck_differencing), with
 *                                  the standard labels: D- looks left,
 *                                  D+ looks right (the printed labels are
 *                                  swapped; Sec. IV-A and the WENO stencils
 *                                  only make sense this way round)
 *   first-order upwinding ........ Sec. IV-A
 *   ENO2 / ENO3 .................. Sec. IV-B (divided-difference table, the
 *                                  smaller-|D^2| and smaller-|D^3| choices;
 *                                  k* is the leftmost node of the chosen
 *                                  three-point stencil)
 *   WENO5 ........................ Sec. IV-C (three substencils, smoothness
 *                                  indicators, eps, weights), with the
 *                                  printed typos read as: third substencil
 *                                  starts with +1/3; sigma_2 uses -2 D+v_{i-1};
 *                                  alpha_3 has numerator 0.3; eps uses the
 *                                  squares of the five differences.  The
 *                                  right-biased value is the mirror image.
 *   Lax-Friedrichs Hamiltonian ... Sec. IV-D: Hhat = H(x, pbar)
 *                                  - sum_d alpha_d (p+_d - p-_d) / 2, with
 *                                  alpha_d the grid-wide maximum of the
 *                                  partial bound (global LF dissipation,
 *                                  Listing 4 'artificialDissipationGLF')
 *   local LF dissipation ......... alpha_d taken at the node itself (the
 *                                  partial bound there) instead of its grid
 *                                  maximum; the CFL step still uses the
 *                                  maximum.  Not in the paper, which names
 *                                  only the global form (Listing 4); the
 *                                  standard local variant of it.
 *   Godunov normal motion ........ for H = a|p| only, the Godunov numerical
 *                                  Hamiltonian in place of Lax-Friedrichs:
 *                                  the extremum of H over the interval
 *                                  between p- and p+ on each axis (min for
 *                                  the convex a >= 0, max for a < 0), which
 *                                  for |p| reduces per axis to
 *                                  q = max(max(p-, 0), -min(p+, 0)) (a >= 0)
 *                                  or max(-min(p-, 0), max(p+, 0)) (a < 0)
 *                                  and Hhat = a sqrt(sum q^2).  Not in the
 *                                  paper: the monotone scheme its upwind
 *                                  discussion leads to for this Hamiltonian.
 *   CFL time step ................ Sec. IV-D (lambda max|f'| <= 1) and Sec. V
 *   TVD-RK 1/2/3 ................. Sec. V (odeCFL1/2/3 averaging steps)
 *   min-with-target .............. Sec. VI, variational HJ PDE (tube form)
 *   conservation-law LF scheme ... Sec. IV-D: v_t + sum_d f_d(v)_{x_d} = 0 by
 *                                  the Lax-Friedrichs scheme (hjxo_claw_*),
 *                                  with the CFL condition of the same section
 *   restricted update ............ Sec. VI: the variational form with
 *                                  min[0, H], and the 'positive' field of
 *                                  the rockets listing (Listing 4).  Read
 *                                  as a clip of the rate of every Euler
 *                                  move: L <- min(L, 0) (phi may only fall
 *                                  in tau, the zero sublevel set only
 *                                  grows) or L <- max(L, 0) (phi may only
 *                                  rise).  The paper does not define the
 *                                  flag; this is the reading.
 *
 * Conventions: time-to-go tau >= 0, phi_tau + H(x, grad phi) = 0,
 * phi(., 0) = phi0; the right-hand side is L(phi) = -Hhat.
 *
 * The same source is compiled twice: once with real = double (exports
 * hjxo_*), once with real = double complex (-DHJXO_CSTEP, exports
 * hjxo_cs_*).  The complex build is the complex-step method of
 * Squire & Trapp (SIAM Rev. 1998): seeding an imaginary perturbation i*h*delta
 * and reading Im(out)/h gives the exact directional derivative of the scheme
 * to rounding.  Every branch (|.|, max, ENO choice, loop exit) is decided on
 * the real part only, so both builds take identical decisions.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef HJXO_CSTEP
#include <complex.h>
typedef double _Complex real;
#define RE(x) creal(x)
#define API(name) hjxo_cs_##name
#else
typedef double real;
#define RE(x) (x)
#define API(name) hjxo_##name
#endif

#define MAXD 4
#define R 3 /* widest stencil radius (ENO3 / WENO5) */

enum { SCHEME_FIRST = 1, SCHEME_ENO2 = 2, SCHEME_ENO3 = 3, SCHEME_WENO5 = 5 };
enum { HAM_NORMAL = 0, HAM_DUBINS3_PE = 1, HAM_DUBINS4 = 2, HAM_ROCKETS = 3 };
enum { RESTRICT_NONE = 0, RESTRICT_NONPOSITIVE = 1, RESTRICT_POSITIVE = 2 };
enum { DISS_GLOBAL = 0, DISS_LOCAL = 1, DISS_GODUNOV = 2 };

/* Problem description, laid out for ctypes. */
typedef struct {
    int dim;
    double gmin[MAXD], gmax[MAXD];
    long n[MAXD];
    unsigned periodic_mask;
    int ham_kind;
    double hp[8];   /* Hamiltonian parameters (see ham_value) */
    int scheme;     /* 1, 2, 3 or 5 */
    int rk;         /* 1, 2 or 3 */
    double cfl;
    int restrict_update; /* RESTRICT_NONE, RESTRICT_NONPOSITIVE or RESTRICT_POSITIVE */
    int dissipation;     /* DISS_GLOBAL, DISS_LOCAL or DISS_GODUNOV */
    int decide_f32;      /* ENO stencil choices taken in binary32 (see eno_choice) */
} hjxo_problem;

/* ------------------------------------------------------------------ */
/* elementary helpers: every decision looks at the real part only       */

static real r_abs(real x)
{
    if (RE(x) > 0) return x;
    if (RE(x) < 0) return -x;
    return (real)0.0; /* sign(0) = 0 */
}

/* the larger of a, b; ties keep a (the earlier one) */
static real r_max(real a, real b) { return RE(b) > RE(a) ? b : a; }

static real r_sq(real x) { return x * x; }

static real r_sqrt(real x)
{
    if (RE(x) <= 0) return (real)0.0; /* |p| at p = 0: value 0, tangent 0 */
#ifdef HJXO_CSTEP
    return csqrt(x);
#else
    return sqrt(x);
#endif
}

static real r_exp(real x)
{
#ifdef HJXO_CSTEP
    return cexp(x);
#else
    return exp(x);
#endif
}

/* ------------------------------------------------------------------ */
/* Grid (Sec. III-B): a non-periodic axis has its end points on gmin and
 * gmax; a periodic axis is the half-open [gmin, gmax). */

static int is_periodic(const hjxo_problem *P, int d) { return (P->periodic_mask >> d) & 1u; }

static double spacing(const hjxo_problem *P, int d)
{
    double len = P->gmax[d] - P->gmin[d];
    return is_periodic(P, d) ? len / (double)P->n[d] : len / (double)(P->n[d] - 1);
}

static double coord(const hjxo_problem *P, int d, long j)
{
    return P->gmin[d] + (double)j * spacing(P, d);
}

static long npoints(const hjxo_problem *P)
{
    long p = 1;
    for (int d = 0; d < P->dim; ++d) p *= P->n[d];
    return p;
}

/* row-major: the last axis is the fastest */
static long stride(const hjxo_problem *P, int d)
{
    long s = 1;
    for (int e = d + 1; e < P->dim; ++e) s *= P->n[e];
    return s;
}

/* multi-index of flat index f */
static void unflatten(const hjxo_problem *P, long f, long idx[MAXD])
{
    for (int d = P->dim - 1; d >= 0; --d) {
        idx[d] = f % P->n[d];
        f /= P->n[d];
    }
}

/* ------------------------------------------------------------------ */
/* Ghost cells (Sec. III-B): copy one grid line into ext[R + j], j = 0..n-1,
 * and fill R ghost values on each side. */

static void fill_line(const real *phi, long start, long step, long n, int periodic, real *ext)
{
    for (long j = 0; j < n; ++j) ext[R + j] = phi[start + j * step];
    for (long k = 1; k <= R; ++k) {
        if (periodic) {
            ext[R - k] = ext[R + n - k];
            ext[R + n - 1 + k] = ext[R + k - 1];
        } else {
            /* linear extrapolation from the two end nodes */
            ext[R - k] = ext[R] + (double)k * (ext[R] - ext[R + 1]);
            ext[R + n - 1 + k] = ext[R + n - 1] + (double)k * (ext[R + n - 1] - ext[R + n - 2]);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Divided differences (Sec. IV-B) on an extended line e (E(j) = e[R + j]).
 *   D1(j) = D^1_{j+1/2} = (E(j+1) - E(j)) / dx      (= D+ phi_j)
 *   D2(j) = D^2_j       = (D1(j) - D1(j-1)) / (2 dx)
 *   D3(j) = D^3_{j+1/2} = (D2(j+1) - D2(j)) / (3 dx)                      */

static real D1(const real *e, long j, double dx) { return (e[R + j + 1] - e[R + j]) / dx; }
static real D2(const real *e, long j, double dx) { return (D1(e, j, dx) - D1(e, j - 1, dx)) / (2.0 * dx); }
static real D3(const real *e, long j, double dx) { return (D2(e, j + 1, dx) - D2(e, j, dx)) / (3.0 * dx); }

/* The ENO choices (Sec. IV-B) turn floating-point comparisons into a
 * stencil, an integer decision.  A solver that computes in binary32 takes
 * them in binary32, so the oracle can take them the same way: with 'ef' the
 * line rounded to binary32 (ghosts extrapolated in binary32, one fused
 * multiply-add each) and h the binary32 reciprocal of the spacing,
 *   d1(j) = (E(j+1) - E(j)) h,  d2(j) = (d1(j) - d1(j-1)) (h/2),
 *   d3(j) = (d2(j+1) - d2(j)) (h * fl32(1/3)),
 * every operation rounded to binary32.  Only the choice is taken from these
 * values; the derivative itself is still formed in double from the double
 * line.  With ef == NULL the choices compare the double D2 and D3 above. */
static void fill_line_f32(const real *e, long n, int periodic, float *ef)
{
    for (long j = 0; j < n; ++j) ef[R + j] = (float)RE(e[R + j]);
    for (long k = 1; k <= R; ++k) {
        if (periodic) {
            ef[R - k] = ef[R + n - k];
            ef[R + n - 1 + k] = ef[R + k - 1];
        } else {
            ef[R - k] = fmaf((float)k, ef[R] - ef[R + 1], ef[R]);
            ef[R + n - 1 + k] = fmaf((float)k, ef[R + n - 1] - ef[R + n - 2], ef[R + n - 1]);
        }
    }
}

static float d1f(const float *ef, long j, float h) { return (ef[R + j + 1] - ef[R + j]) * h; }
static float d2f(const float *ef, long j, float h) { return (d1f(ef, j, h) - d1f(ef, j - 1, h)) * (0.5f * h); }
static float d3f(const float *ef, long j, float h)
{
    return (d2f(ef, j + 1, h) - d2f(ef, j, h)) * (h * (float)(1.0 / 3.0));
}

/* does the smaller-|D^o| rule pick the left candidate (D2 at j vs j+1 for
 * o = 2, D3 at j vs j+1 for o = 3)?  Ties go left, as printed. */
static int eno_choice(const real *e, const float *ef, long j, int o, double dx, float h)
{
    if (ef) {
        const float a = o == 2 ? d2f(ef, j, h) : d3f(ef, j, h);
        const float b = o == 2 ? d2f(ef, j + 1, h) : d3f(ef, j + 1, h);
        return fabsf(a) <= fabsf(b);
    }
    const real a = o == 2 ? D2(e, j, dx) : D3(e, j, dx);
    const real b = o == 2 ? D2(e, j + 1, dx) : D3(e, j + 1, dx);
    return RE(r_abs(a)) <= RE(r_abs(b));
}

/* ENO derivative at node i from the stencil that starts at interval k
 * (k = i-1 for the left-biased value, k = i for the right-biased one),
 * grown to 'order' points + 1 by the smaller-divided-difference rule. */
static real eno_derivative(const real *e, const float *ef, float h, long i, long k, int order, double dx)
{
    real p = D1(e, k, dx); /* Q1'(x_i) */
    if (order == 1) return p;

    real c;
    long kstar;
    if (eno_choice(e, ef, k, 2, dx, h)) { /* |D2_k| <= |D2_{k+1}|: ties go left */
        c = D2(e, k, dx);
        kstar = k - 1;
    } else {
        c = D2(e, k + 1, dx);
        kstar = k;
    }
    p = p + c * (double)(2 * (i - k) - 1) * dx; /* Q2'(x_i) */
    if (order == 2) return p;

    real cstar;
    if (eno_choice(e, ef, kstar, 3, dx, h))
        cstar = D3(e, kstar, dx);     /* D^3_{k*+1/2} */
    else
        cstar = D3(e, kstar + 1, dx); /* D^3_{k*+3/2} */
    long m = i - kstar;
    p = p + cstar * (double)(3 * m * m - 6 * m + 2) * dx * dx; /* Q3'(x_i) */
    return p;
}

/* WENO5 (Sec. IV-C) from five consecutive one-sided differences v1..v5,
 * ordered so that the result approximates the derivative at the node that
 * sits between v3 and v4 on the upwind side. */
static real weno5(real v1, real v2, real v3, real v4, real v5)
{
    /* the three third-order substencils */
    real f0 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
    real f1 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
    real f2 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;

    /* smoothness of each substencil */
    real s0 = 13.0 / 12.0 * r_sq(v1 - 2.0 * v2 + v3) + 0.25 * r_sq(v1 - 4.0 * v2 + 3.0 * v3);
    real s1 = 13.0 / 12.0 * r_sq(v2 - 2.0 * v3 + v4) + 0.25 * r_sq(v2 - v4);
    real s2 = 13.0 / 12.0 * r_sq(v3 - 2.0 * v4 + v5) + 0.25 * r_sq(3.0 * v3 - 4.0 * v4 + v5);

    real vmax2 = r_sq(v1);
    vmax2 = r_max(vmax2, r_sq(v2));
    vmax2 = r_max(vmax2, r_sq(v3));
    vmax2 = r_max(vmax2, r_sq(v4));
    vmax2 = r_max(vmax2, r_sq(v5));
    real eps = 1e-6 * vmax2 + 1e-99;

    real a0 = 0.1 / r_sq(s0 + eps);
    real a1 = 0.6 / r_sq(s1 + eps);
    real a2 = 0.3 / r_sq(s2 + eps);
    return (a0 * f0 + a1 * f1 + a2 * f2) / (a0 + a1 + a2);
}

/* Left (pm) and right (pp) derivative approximations at every node of one
 * extended line. */
static void derivative_line(int scheme, const real *e, const float *ef, long n, double dx, real *pm, real *pp)
{
    const float h = (float)(1.0 / dx); /* used only with ef */
    for (long i = 0; i < n; ++i) {
        switch (scheme) {
        case SCHEME_FIRST: /* Sec. IV-A: D- and D+ */
            pm[i] = (e[R + i] - e[R + i - 1]) / dx;
            pp[i] = (e[R + i + 1] - e[R + i]) / dx;
            break;
        case SCHEME_ENO2:
            pm[i] = eno_derivative(e, ef, h, i, i - 1, 2, dx);
            pp[i] = eno_derivative(e, ef, h, i, i, 2, dx);
            break;
        case SCHEME_ENO3:
            pm[i] = eno_derivative(e, ef, h, i, i - 1, 3, dx);
            pp[i] = eno_derivative(e, ef, h, i, i, 3, dx);
            break;
        case SCHEME_WENO5:
            /* left-biased: v_m = D+ phi_{i-4+m}, m = 1..5 */
            pm[i] = weno5(D1(e, i - 3, dx), D1(e, i - 2, dx), D1(e, i - 1, dx),
                          D1(e, i, dx), D1(e, i + 1, dx));
            /* right-biased: the mirror image */
            pp[i] = weno5(D1(e, i + 2, dx), D1(e, i + 1, dx), D1(e, i, dx),
                          D1(e, i - 1, dx), D1(e, i - 2, dx));
            break;
        }
    }
}

/* pm, pp along axis d at every node of the grid */
static void derivative_axis(const hjxo_problem *P, const real *phi, int d, real *pm, real *pp)
{
    long n = P->n[d], s = stride(P, d), total = npoints(P);
    long nlines = total / n;
    double dx = spacing(P, d);
    int per = is_periodic(P, d);
#pragma omp parallel
    {
        real *ext = (real *)malloc(sizeof(real) * (size_t)(n + 2 * R));
        float *extf = P->decide_f32 ? (float *)malloc(sizeof(float) * (size_t)(n + 2 * R)) : NULL;
        real *lm = (real *)malloc(sizeof(real) * (size_t)n);
        real *lp = (real *)malloc(sizeof(real) * (size_t)n);
#pragma omp for schedule(static)
        for (long line = 0; line < nlines; ++line) {
            long outer = line / s, inner = line % s;
            long start = outer * n * s + inner;
            fill_line(phi, start, s, n, per, ext);
            if (extf) fill_line_f32(ext, n, per, extf);
            derivative_line(P->scheme, ext, extf, n, dx, lm, lp);
            for (long j = 0; j < n; ++j) {
                pm[start + j * s] = lm[j];
                pp[start + j * s] = lp[j];
            }
        }
        free(ext);
        free(extf);
        free(lm);
        free(lp);
    }
}

/* ------------------------------------------------------------------ */
/* Hamiltonians (convention: phi_tau + H = 0, tau = time to go).
 *
 * HAM_NORMAL     hp = [a]: motion at speed a along the outward normal,
 *                H = a |p|; partial bound alpha_d = |a|.
 * HAM_DUBINS3_PE hp = [v_e, v_p, wbar_e, wbar_p]: pursuit-evasion of two
 *                unicycles in the evader's frame, state (x, y, theta):
 *                  xdot = -v_e + v_p cos th + w_e y
 *                  ydot =  v_p sin th - w_e x
 *                  thdot = w_p - w_e,  |w_e| <= wbar_e, |w_p| <= wbar_p;
 *                the evader maximises and the pursuer minimises p.f, so
 *                H = -[p1(-v_e + v_p cos th) + p2 v_p sin th
 *                      + wbar_e |p1 y - p2 x - p3| - wbar_p |p3|].
 * HAM_DUBINS4    hp = [wbar, abar]: car with speed state (x, y, theta, v),
 *                xdot = v cos th, ydot = v sin th, thdot = w, vdot = a;
 *                the control minimises p.f (reach), so
 *                H = -v(p1 cos th + p2 sin th) + wbar |p3| + abar |p4|.
 * HAM_ROCKETS    hp = [a, g, ubar_e, ubar_p]: the two-rocket game of Sec. VI,
 *                state (x, z, theta), with the vector field inside the
 *                max-min of eq. (ham_def) and a_e = a_p = a:
 *                  xdot = a cos th + u_e x
 *                  zdot = a sin th + a + u_p x - g
 *                  thdot = u_p - u_e,  |u_e| <= ubar_e, |u_p| <= ubar_p;
 *                the evader maximises and the pursuer minimises p.f.  The
 *                terms in u_e and u_p separate, so
 *                H = -[a p1 cos th + p2 (a sin th + a - g)
 *                      + ubar_e |p1 x - p3| - ubar_p |p2 x + p3|].
 *                (The closed form printed as eq. (rocket_hamfunc) differs
 *                from this in the sign of the p2 term and of both absolute
 *                values; the definition is followed.)                       */

static real ham_value(const hjxo_problem *P, const real *hp, const double *x, const real *p)
{
    switch (P->ham_kind) {
    case HAM_NORMAL: {
        real s = 0.0;
        for (int d = 0; d < P->dim; ++d) s = s + r_sq(p[d]);
        return hp[0] * r_sqrt(s);
    }
    case HAM_DUBINS3_PE: {
        double c = cos(x[2]), sn = sin(x[2]);
        real ve = hp[0], vp = hp[1], we = hp[2], wp = hp[3];
        real drift = p[0] * (-ve + vp * c) + p[1] * (vp * sn);
        return -(drift + we * r_abs(p[0] * x[1] - p[1] * x[0] - p[2]) - wp * r_abs(p[2]));
    }
    case HAM_DUBINS4: {
        double c = cos(x[2]), sn = sin(x[2]);
        real wb = hp[0], ab = hp[1];
        return -x[3] * (p[0] * c + p[1] * sn) + wb * r_abs(p[2]) + ab * r_abs(p[3]);
    }
    case HAM_ROCKETS: {
        double c = cos(x[2]), sn = sin(x[2]);
        real a = hp[0], g = hp[1], ue = hp[2], up = hp[3];
        real drift = a * c * p[0] + (a * sn + a - g) * p[1];
        return -(drift + ue * r_abs(p[0] * x[0] - p[2]) - up * r_abs(p[1] * x[0] + p[2]));
    }
    }
    return 0.0;
}

/* bound on |dH/dp_d| at one node, over all admissible controls */
static real partial_bound(const hjxo_problem *P, const real *hp, const double *x, int d)
{
    switch (P->ham_kind) {
    case HAM_NORMAL:
        return r_abs(hp[0]);
    case HAM_DUBINS3_PE: {
        real ve = hp[0], vp = hp[1], we = hp[2], wp = hp[3];
        if (d == 0) return r_abs(-ve + vp * cos(x[2])) + we * fabs(x[1]);
        if (d == 1) return r_abs(vp * sin(x[2])) + we * fabs(x[0]);
        return we + wp;
    }
    case HAM_DUBINS4: {
        real wb = hp[0], ab = hp[1];
        if (d == 0) return r_abs((real)(x[3] * cos(x[2])));
        if (d == 1) return r_abs((real)(x[3] * sin(x[2])));
        if (d == 2) return wb;
        return ab;
    }
    case HAM_ROCKETS: {
        real a = hp[0], g = hp[1], ue = hp[2], up = hp[3];
        if (d == 0) return r_abs(a * cos(x[2])) + ue * fabs(x[0]);
        if (d == 1) return r_abs(a * sin(x[2]) + a - g) + up * fabs(x[0]);
        return ue + up;
    }
    }
    return 0.0;
}

/* alpha_d = max over grid nodes of the partial bound (global LF) */
static void dissipation_alpha(const hjxo_problem *P, const real *hp, real alpha[MAXD])
{
    long total = npoints(P);
    for (int d = 0; d < P->dim; ++d) alpha[d] = 0.0;
    for (long f = 0; f < total; ++f) {
        long idx[MAXD];
        double x[MAXD];
        unflatten(P, f, idx);
        for (int d = 0; d < P->dim; ++d) x[d] = coord(P, d, idx[d]);
        for (int d = 0; d < P->dim; ++d) alpha[d] = r_max(alpha[d], partial_bound(P, hp, x, d));
    }
}

/* CFL step: cfl / sum_d alpha_d / dx_d (infinite if nothing moves) */
static real cfl_dt(const hjxo_problem *P, const real alpha[MAXD])
{
    real rate = 0.0;
    for (int d = 0; d < P->dim; ++d) rate = rate + alpha[d] / spacing(P, d);
    if (RE(rate) <= 0) return (real)INFINITY;
    return P->cfl / rate;
}

/* ------------------------------------------------------------------ */
/* L(phi) = -Hhat(phi): the Lax-Friedrichs right-hand side */

static void lf_rhs(const hjxo_problem *P, const real *hp, const real *phi, const real alpha[MAXD],
                   real *L, real *pm[MAXD], real *pp[MAXD])
{
    long total = npoints(P);
    for (int d = 0; d < P->dim; ++d) derivative_axis(P, phi, d, pm[d], pp[d]);
#pragma omp parallel for schedule(static)
    for (long f = 0; f < total; ++f) {
        long idx[MAXD];
        double x[MAXD];
        real pbar[MAXD];
        unflatten(P, f, idx);
        for (int d = 0; d < P->dim; ++d) {
            x[d] = coord(P, d, idx[d]);
            pbar[d] = (pm[d][f] + pp[d][f]) / 2.0;
        }
        if (P->dissipation == DISS_GODUNOV) { /* normal motion only (check_problem) */
            real s = 0.0;
            for (int d = 0; d < P->dim; ++d) {
                real m = pm[d][f], p = pp[d][f], q;
                if (RE(hp[0]) >= 0) {
                    real up = RE(m) > 0 ? m : (real)0.0, dn = RE(p) < 0 ? -p : (real)0.0;
                    q = r_max(up, dn);
                } else {
                    real dn = RE(m) < 0 ? -m : (real)0.0, up = RE(p) > 0 ? p : (real)0.0;
                    q = r_max(dn, up);
                }
                s = s + q * q;
            }
            L[f] = -(hp[0] * r_sqrt(s));
            continue;
        }
        real hhat = ham_value(P, hp, x, pbar);
        for (int d = 0; d < P->dim; ++d) {
            real a = P->dissipation == DISS_LOCAL ? partial_bound(P, hp, x, d) : alpha[d];
            hhat = hhat - a * (pp[d][f] - pm[d][f]) / 2.0;
        }
        L[f] = -hhat;
    }
}

/* ------------------------------------------------------------------ */
/* TVD Runge-Kutta (Sec. V) with optional min-with-target (Sec. VI) */

typedef struct {
    real *L, *a, *b, *pm[MAXD], *pp[MAXD];
} workspace;

static int ws_alloc(const hjxo_problem *P, workspace *w)
{
    size_t bytes = sizeof(real) * (size_t)npoints(P);
    memset(w, 0, sizeof(*w));
    w->L = (real *)malloc(bytes);
    w->a = (real *)malloc(bytes);
    w->b = (real *)malloc(bytes);
    int ok = w->L && w->a && w->b;
    for (int d = 0; d < P->dim; ++d) {
        w->pm[d] = (real *)malloc(bytes);
        w->pp[d] = (real *)malloc(bytes);
        ok = ok && w->pm[d] && w->pp[d];
    }
    return ok;
}

static void ws_free(workspace *w)
{
    free(w->L);
    free(w->a);
    free(w->b);
    for (int d = 0; d < MAXD; ++d) {
        free(w->pm[d]);
        free(w->pp[d]);
    }
}

/* The rate of an Euler move under the restricted update (Sec. VI):
 * min[0, .] of the variational form keeps only rates that lower phi; the
 * 'positive' flag keeps only rates that raise it.  A clipped rate is an
 * exact zero (value and complex-step tangent). */
static real restricted_rate(const hjxo_problem *P, real L)
{
    if (P->restrict_update == RESTRICT_NONPOSITIVE && RE(L) > 0) return (real)0.0;
    if (P->restrict_update == RESTRICT_POSITIVE && RE(L) < 0) return (real)0.0;
    return L;
}

/* one Euler move: out = in + dt * L(in), L restricted as above */
static void euler(const hjxo_problem *P, const real *hp, const real *in, const real alpha[MAXD],
                  real dt, real *out, workspace *w)
{
    long total = npoints(P);
    lf_rhs(P, hp, in, alpha, w->L, w->pm, w->pp);
    for (long f = 0; f < total; ++f) out[f] = in[f] + dt * restricted_rate(P, w->L[f]);
}

/* advance phi by one step of size dt (in place) */
static void rk_step(const hjxo_problem *P, const real *hp, real *phi, const real *target, real dt,
                    workspace *w)
{
    long total = npoints(P);
    real alpha[MAXD];
    dissipation_alpha(P, hp, alpha);

    if (P->rk == 1) { /* odeCFL1: forward Euler */
        euler(P, hp, phi, alpha, dt, w->a, w);
        for (long f = 0; f < total; ++f) phi[f] = w->a[f];
    } else if (P->rk == 2) { /* odeCFL2: two Euler moves, then average */
        euler(P, hp, phi, alpha, dt, w->a, w);
        euler(P, hp, w->a, alpha, dt, w->b, w);
        for (long f = 0; f < total; ++f) phi[f] = (phi[f] + w->b[f]) / 2.0;
    } else { /* odeCFL3: Shu-Osher three stages */
        euler(P, hp, phi, alpha, dt, w->a, w);
        euler(P, hp, w->a, alpha, dt, w->b, w);
        for (long f = 0; f < total; ++f) w->a[f] = (3.0 * phi[f] + w->b[f]) / 4.0;
        euler(P, hp, w->a, alpha, dt, w->b, w);
        for (long f = 0; f < total; ++f) phi[f] = (phi[f] + 2.0 * w->b[f]) / 3.0;
    }
    if (target)
        for (long f = 0; f < total; ++f)
            if (RE(target[f]) < RE(phi[f])) phi[f] = target[f]; /* ties keep phi */
}

/* time loop from t0 to t1 with the CFL step; the step that would reach
 * (or come within 1e-12 relative of) t1 is clamped to land on t1.  With
 * max_steps >= 0 the loop stops after that many steps and *t_reached (if
 * not NULL) says where, so that a later call from there continues the same
 * schedule. */
static long solve(const hjxo_problem *P, const real *hp, real *phi, const real *target, double t0,
                  double t1, workspace *w, double *dt_first, long max_steps, double *t_reached)
{
    real t = t0;
    long steps = 0;
    double slack = 1e-12 * (fabs(t1) > 1.0 ? fabs(t1) : 1.0);
    while (RE(t) < t1 && (max_steps < 0 || steps < max_steps)) {
        real alpha[MAXD];
        dissipation_alpha(P, hp, alpha);
        real dt = cfl_dt(P, alpha);
        int last = 0;
        if (RE(t + dt) >= t1 - slack) {
            dt = t1 - t;
            last = 1;
        }
        if (steps == 0 && dt_first) *dt_first = RE(dt);
        rk_step(P, hp, phi, target, dt, w);
        ++steps;
        t = last ? (real)t1 : t + dt;
    }
    if (t_reached) *t_reached = RE(t);
    return steps;
}

static int check_problem(const hjxo_problem *P)
{
    if (P->dim < 1 || P->dim > MAXD) return -1;
    for (int d = 0; d < P->dim; ++d) {
        if (P->n[d] < 3) return -1;
        if (!(P->gmax[d] > P->gmin[d])) return -1;
    }
    if (P->scheme != SCHEME_FIRST && P->scheme != SCHEME_ENO2 && P->scheme != SCHEME_ENO3 &&
        P->scheme != SCHEME_WENO5)
        return -1;
    if (P->rk < 1 || P->rk > 3) return -1;
    if (P->restrict_update < RESTRICT_NONE || P->restrict_update > RESTRICT_POSITIVE) return -1;
    if (P->dissipation != DISS_GLOBAL && P->dissipation != DISS_LOCAL && P->dissipation != DISS_GODUNOV) return -1;
    if (P->dissipation == DISS_GODUNOV && P->ham_kind != HAM_NORMAL) return -1;
    if (P->ham_kind == HAM_DUBINS3_PE && P->dim != 3) return -1;
    if (P->ham_kind == HAM_DUBINS4 && P->dim != 4) return -1;
    if (P->ham_kind == HAM_ROCKETS && P->dim != 3) return -1;
    if (P->ham_kind < 0 || P->ham_kind > 3) return -1;
    return 0;
}

/* ================================================================== */
/* exported entry points                                                */

#ifndef HJXO_CSTEP

void hjxo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int hjxo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* spacing and node coordinates of axis d */
int hjxo_grid(const hjxo_problem *P, int d, double *dx, double *coords)
{
    if (check_problem(P) || d < 0 || d >= P->dim) return -1;
    *dx = spacing(P, d);
    if (coords)
        for (long j = 0; j < P->n[d]; ++j) coords[j] = coord(P, d, j);
    return 0;
}

/* derivative approximations along a single line of n nodes */
int hjxo_deriv_line(int scheme, const double *phi, long n, int periodic, double dx, double *pm,
                    double *pp)
{
    if (n < 3 || !(dx > 0)) return -1;
    if (scheme != SCHEME_FIRST && scheme != SCHEME_ENO2 && scheme != SCHEME_ENO3 &&
        scheme != SCHEME_WENO5)
        return -1;
    double *ext = (double *)malloc(sizeof(double) * (size_t)(n + 2 * R));
    fill_line(phi, 0, 1, n, periodic, ext);
    derivative_line(scheme, ext, NULL, n, dx, pm, pp);
    free(ext);
    return 0;
}

/* WENO5 combination of five given differences (left-biased ordering) */
double hjxo_weno5(double v1, double v2, double v3, double v4, double v5)
{
    return weno5(v1, v2, v3, v4, v5);
}

/* derivative approximations along axis d of the whole grid */
int hjxo_deriv_axis(const hjxo_problem *P, const double *phi, int d, double *pm, double *pp)
{
    if (check_problem(P) || d < 0 || d >= P->dim) return -1;
    derivative_axis(P, phi, d, pm, pp);
    return 0;
}

/* H(x_f, p) at flat node f */
double hjxo_ham(const hjxo_problem *P, long f, const double *p)
{
    long idx[MAXD];
    double x[MAXD];
    unflatten(P, f, idx);
    for (int d = 0; d < P->dim; ++d) x[d] = coord(P, d, idx[d]);
    return ham_value(P, P->hp, x, p);
}

int hjxo_alpha(const hjxo_problem *P, double *alpha)
{
    if (check_problem(P)) return -1;
    real a[MAXD];
    dissipation_alpha(P, P->hp, a);
    for (int d = 0; d < P->dim; ++d) alpha[d] = a[d];
    return 0;
}

double hjxo_cfl_dt(const hjxo_problem *P)
{
    real a[MAXD];
    dissipation_alpha(P, P->hp, a);
    return cfl_dt(P, a);
}

/* L = -Hhat at every node */
int hjxo_rhs(const hjxo_problem *P, const double *phi, double *L)
{
    if (check_problem(P)) return -1;
    workspace w;
    if (!ws_alloc(P, &w)) { ws_free(&w); return -2; }
    real alpha[MAXD];
    dissipation_alpha(P, P->hp, alpha);
    lf_rhs(P, P->hp, phi, alpha, L, w.pm, w.pp);
    ws_free(&w);
    return 0;
}

/* one step of size dt, in place; target may be NULL */
int hjxo_step(const hjxo_problem *P, double *phi, const double *target, double dt)
{
    if (check_problem(P)) return -1;
    workspace w;
    if (!ws_alloc(P, &w)) { ws_free(&w); return -2; }
    rk_step(P, P->hp, phi, target, dt, &w);
    ws_free(&w);
    return 0;
}

/* full solve from t0 to t1; returns the number of steps (< 0 on error) */
long hjxo_solve(const hjxo_problem *P, const double *phi0, const double *target, double t0,
                double t1, double *phi_out, double *dt_first)
{
    if (check_problem(P) || !(t1 >= t0)) return -1;
    workspace w;
    if (!ws_alloc(P, &w)) { ws_free(&w); return -2; }
    long total = npoints(P);
    if (phi_out != phi0) memcpy(phi_out, phi0, sizeof(double) * (size_t)total);
    long steps = solve(P, P->hp, phi_out, target, t0, t1, &w, dt_first, -1, NULL);
    ws_free(&w);
    return steps;
}

/* At most max_steps >= 1 steps of the solve from t0 towards t1, in place on
 * phi; *t_reached is where they end.  Calling again from there (t0 =
 * *t_reached) until it equals t1 takes exactly the steps of one hjxo_solve,
 * so a long solve can report progress between calls.  Returns the number of
 * steps taken (< 0 on error). */
long hjxo_solve_part(const hjxo_problem *P, double *phi, const double *target, double t0, double t1,
                     long max_steps, double *t_reached)
{
    if (check_problem(P) || !(t1 >= t0) || max_steps < 1 || !t_reached) return -1;
    workspace w;
    if (!ws_alloc(P, &w)) { ws_free(&w); return -2; }
    long steps = solve(P, P->hp, phi, target, t0, t1, &w, NULL, max_steps, t_reached);
    ws_free(&w);
    return steps;
}

/* ------------------------------------------------------------------ */
/* Scalar conservation laws v_t + sum_d f_d(v)_{x_d} = 0 (Sec. IV-D).
 *
 * The paper gives the Lax-Friedrichs scheme in one dimension,
 *   v_j^{n+1} = v_j^n - (lambda/2) (f(v_{j+1}) - f(v_{j-1}))
 *               + (1/2) (v_{j+1} - 2 v_j + v_{j-1}),   lambda = dt/dx,
 * monotone when lambda max |f'| <= 1.  In N dimensions (the reading used
 * here) the new value is the mean of the 2N axis neighbours minus the
 * central flux differences of every axis,
 *   v^{n+1} = (1/2N) sum_d (v_{+d} + v_{-d}) - sum_d (lambda_d/2) (f_d(v_{+d}) - f_d(v_{-d})),
 * which is monotone when lambda_d max |f_d'| <= 1/N on every axis, and is the
 * printed scheme for N = 1.  Periodic axes wrap; on the others the value
 * beyond the edge is the edge value.
 *
 * Fluxes: CLAW_LINEAR f_d(v) = c_d v; CLAW_BURGERS f_d(v) = c_d v^2 / 2.   */

enum { CLAW_LINEAR = 0, CLAW_BURGERS = 1 };

typedef struct {
    int dim;
    double gmin[MAXD], gmax[MAXD];
    long n[MAXD];
    unsigned periodic_mask;
    int flux;        /* CLAW_LINEAR or CLAW_BURGERS */
    double c[MAXD];  /* flux coefficient per axis */
    double cfl;      /* 0 < cfl <= 1 */
} hjxo_claw;

/* the grid of a conservation law as a problem (for the grid helpers) */
static hjxo_problem claw_grid(const hjxo_claw *C)
{
    hjxo_problem P;
    memset(&P, 0, sizeof P);
    P.dim = C->dim;
    for (int d = 0; d < MAXD; ++d) {
        P.gmin[d] = C->gmin[d];
        P.gmax[d] = C->gmax[d];
        P.n[d] = C->n[d];
    }
    P.periodic_mask = C->periodic_mask;
    P.scheme = SCHEME_FIRST;
    P.rk = 1;
    P.cfl = C->cfl;
    return P;
}

static int claw_check(const hjxo_claw *C)
{
    if (C->dim < 1 || C->dim > MAXD) return -1;
    for (int d = 0; d < C->dim; ++d)
        if (C->n[d] < 3 || !(C->gmax[d] > C->gmin[d])) return -1;
    if (C->flux != CLAW_LINEAR && C->flux != CLAW_BURGERS) return -1;
    if (!(C->cfl > 0) || !(C->cfl <= 1)) return -1;
    return 0;
}

static double claw_flux(const hjxo_claw *C, int d, double v)
{
    if (C->flux == CLAW_LINEAR) return C->c[d] * v;
    return C->c[d] * v * v / 2.0;
}

/* value of the neighbour of flat node f at offset s (+1 or -1) along axis d */
static double claw_neighbour(const hjxo_problem *G, const double *v, long f, const long idx[MAXD], int d, int s)
{
    long stride = 1;
    for (int e = G->dim - 1; e > d; --e) stride *= G->n[e];
    long j = idx[d] + s;
    if (j < 0 || j >= G->n[d]) {
        if ((G->periodic_mask >> d) & 1u) j = j < 0 ? j + G->n[d] : j - G->n[d];
        else j = idx[d];  /* the edge value */
    }
    return v[f + (j - idx[d]) * stride];
}

/* the CFL step of the data v: cfl * min_d dx_d / (N max |f_d'|), with
 * max |f_d'| = |c_d| (linear) or |c_d| max |v| (Burgers); +inf if nothing moves */
double hjxo_claw_dt(const hjxo_claw *C, const double *v)
{
    if (claw_check(C)) return -1.0;
    hjxo_problem G = claw_grid(C);
    double vmax = 0.0;
    if (C->flux == CLAW_BURGERS)
        for (long f = 0; f < npoints(&G); ++f) vmax = fabs(v[f]) > vmax ? fabs(v[f]) : vmax;
    double dt = INFINITY;
    for (int d = 0; d < C->dim; ++d) {
        double speed = C->flux == CLAW_LINEAR ? fabs(C->c[d]) : fabs(C->c[d]) * vmax;
        if (speed > 0) {
            double h = C->cfl * spacing(&G, d) / ((double)C->dim * speed);
            dt = h < dt ? h : dt;
        }
    }
    return dt;
}

/* one Lax-Friedrichs step of size dt from v into out (no aliasing) */
int hjxo_claw_step(const hjxo_claw *C, const double *v, double *out, double dt)
{
    if (claw_check(C) || !(dt >= 0) || v == out) return -1;
    hjxo_problem G = claw_grid(C);
    long total = npoints(&G);
#pragma omp parallel for schedule(static)
    for (long f = 0; f < total; ++f) {
        long idx[MAXD];
        unflatten(&G, f, idx);
        double mean = 0.0, flux = 0.0;
        for (int d = 0; d < C->dim; ++d) {
            double vp = claw_neighbour(&G, v, f, idx, d, +1), vm = claw_neighbour(&G, v, f, idx, d, -1);
            mean += vp + vm;
            flux += (dt / spacing(&G, d)) / 2.0 * (claw_flux(C, d, vp) - claw_flux(C, d, vm));
        }
        out[f] = mean / (2.0 * C->dim) - flux;
    }
    return 0;
}

/* solve from 0 to t1 with the CFL step of v0 (the scheme is monotone, so
 * max |v| and with it every speed bound never grows); the step that would
 * reach t1 (or come within 1e-12 relative of it) lands on t1.  Returns the
 * number of steps. */
long hjxo_claw_solve(const hjxo_claw *C, const double *v0, double t1, double *out, double *dt_out)
{
    if (claw_check(C) || !(t1 >= 0)) return -1;
    hjxo_problem G = claw_grid(C);
    long total = npoints(&G);
    double dt = hjxo_claw_dt(C, v0);
    if (dt_out) *dt_out = dt;
    double *a = (double *)malloc(sizeof(double) * (size_t)total);
    if (!a) return -2;
    memcpy(out, v0, sizeof(double) * (size_t)total);
    double t = 0.0, slack = 1e-12 * (fabs(t1) > 1.0 ? fabs(t1) : 1.0);
    long steps = 0;
    while (t < t1) {
        double h = dt;
        int last = 0;
        if (t + h >= t1 - slack) {
            h = t1 - t;
            last = 1;
        }
        hjxo_claw_step(C, out, a, h);
        memcpy(out, a, sizeof(double) * (size_t)total);
        ++steps;
        t = last ? t1 : t + h;
    }
    free(a);
    return steps;
}

#else /* HJXO_CSTEP: complex-step directional derivatives */

/* Smoothed-Heaviside volume of {phi <= 0}:
 *   loss = cell volume * sum_f sigma(-phi_f / eps_h),  sigma(z) = 1/(1+e^-z) */
static real sigmoid_volume(const hjxo_problem *P, const real *phi, double eps_h)
{
    long total = npoints(P);
    double vol = 1.0;
    for (int d = 0; d < P->dim; ++d) vol *= spacing(P, d);
    real acc = 0.0;
    for (long f = 0; f < total; ++f) acc = acc + 1.0 / (1.0 + r_exp(phi[f] / eps_h));
    return vol * acc;
}

/* Solve from phi0 + i h dphi0 with parameters hp + i h dhp (target = phi0
 * when with_target != 0, perturbed alike); returns the loss value and its
 * directional derivative Im(loss)/h.  phi_T_re/phi_T_tan (optional) get
 * the final state and its tangent. */
long hjxo_cs_solve_loss(const hjxo_problem *P, const double *phi0, const double *dphi0,
                        const double *dhp, int with_target, double t0, double t1, double eps_h,
                        double h, double *loss, double *dloss, double *phi_T_re, double *phi_T_tan)
{
    if (check_problem(P) || !(t1 >= t0) || !(h > 0)) return -1;
    long total = npoints(P);
    real hp[8];
    for (int k = 0; k < 8; ++k) hp[k] = P->hp[k] + I * h * (dhp ? dhp[k] : 0.0);
    real *phi = (real *)malloc(sizeof(real) * (size_t)total);
    real *tgt = with_target ? (real *)malloc(sizeof(real) * (size_t)total) : NULL;
    workspace w;
    if (!phi || (with_target && !tgt) || !ws_alloc(P, &w)) {
        free(phi);
        free(tgt);
        return -2;
    }
    for (long f = 0; f < total; ++f) {
        phi[f] = phi0[f] + I * h * (dphi0 ? dphi0[f] : 0.0);
        if (tgt) tgt[f] = phi[f];
    }
    long steps = solve(P, hp, phi, tgt, t0, t1, &w, NULL, -1, NULL);
    real L = sigmoid_volume(P, phi, eps_h);
    *loss = creal(L);
    *dloss = cimag(L) / h;
    for (long f = 0; f < total; ++f) {
        if (phi_T_re) phi_T_re[f] = creal(phi[f]);
        if (phi_T_tan) phi_T_tan[f] = cimag(phi[f]) / h;
    }
    ws_free(&w);
    free(phi);
    free(tgt);
    return steps;
}

#endif
