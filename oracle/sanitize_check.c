/*
 * A run of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure: built and run by tests/test_oracle_sanitized.py with
 * gcc on the host; nothing else uses it).  The real build of hjxo.c is
 * compiled into this file; the complex-step build is linked beside it.
 * Every Hamiltonian, derivative scheme and RK order takes a few steps on
 * tiny grids (n = 3 to 9, periodic and not), with the restricted updates and
 * the local, Godunov and global dissipations, and the complex-step loss runs
 * once; the conservation-law scheme steps every dimension and flux; any
 * invalid access or undefined operation aborts the program.
 */
#include "hjxo.c"

#include <stdio.h>

long hjxo_cs_solve_loss(const hjxo_problem *P, const double *phi0, const double *dphi0, const double *dhp,
                        int with_target, double t0, double t1, double eps_h, double h, double *loss,
                        double *dloss, double *phi_T_re, double *phi_T_tan);

static int run_opts(int dim, const long *n, unsigned per, int ham, int scheme, int rk, int restrict_update,
                    int dissipation)
{
    hjxo_problem P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    for (int d = 0; d < dim; ++d) {
        P.gmin[d] = d == 2 ? 0.0 : -1.0;
        P.gmax[d] = d == 2 ? 6.283185307179586 : 1.5;
        P.n[d] = n[d];
    }
    P.periodic_mask = per;
    P.ham_kind = ham;
    if (ham == 0) P.hp[0] = 1.0;
    if (ham == 1) { P.hp[0] = 1.0; P.hp[1] = 1.2; P.hp[2] = 0.5; P.hp[3] = 0.7; }
    if (ham == 2) { P.hp[0] = 1.0; P.hp[1] = 0.8; }
    if (ham == 3) { P.hp[0] = 1.0; P.hp[1] = 3.0; P.hp[2] = 0.5; P.hp[3] = 0.7; }
    P.restrict_update = restrict_update;
    P.dissipation = dissipation;
    P.scheme = scheme;
    P.rk = rk;
    P.cfl = 0.75;
    long total = 1;
    for (int d = 0; d < dim; ++d) total *= n[d];
    double *phi = malloc(sizeof(double) * total), *tg = malloc(sizeof(double) * total),
           *out = malloc(sizeof(double) * total), *dphi = malloc(sizeof(double) * total);
    for (long f = 0; f < total; ++f) {
        phi[f] = sin(0.7 * f) + 0.1 * (double)(f % 5) - 0.3;
        tg[f] = phi[f] + 0.05;
        dphi[f] = cos(0.3 * f);
    }
    const double dt = hjxo_cfl_dt(&P);
    const double t1 = isfinite(dt) ? 3.5 * dt : 0.1;
    long steps = hjxo_solve(&P, phi, tg, 0.0, t1, out, NULL);
    int bad = steps < 0;
    for (long f = 0; f < total && !bad; ++f) bad = !isfinite(out[f]);
    double L = 0.0, dL = 0.0, dhp[8] = {1, 0, 0, 0, 0, 0, 0, 0};
    if (!bad && hjxo_cs_solve_loss(&P, phi, dphi, dhp, 1, 0.0, t1, 0.3, 1e-20, &L, &dL, NULL, NULL) < 0) bad = 1;
    if (!bad && !(isfinite(L) && isfinite(dL))) bad = 1;
    free(phi); free(tg); free(out); free(dphi);
    if (bad)
        fprintf(stderr, "failed: dim %d ham %d scheme %d rk %d restrict %d dissipation %d\n", dim, ham, scheme, rk,
                restrict_update, dissipation);
    return bad;
}

static int run(int dim, const long *n, unsigned per, int ham, int scheme, int rk)
{
    return run_opts(dim, n, per, ham, scheme, rk, 0, 0);
}

/* a few Lax-Friedrichs steps of a conservation law on a tiny grid */
static int run_claw(int dim, const long *n, unsigned per, int flux)
{
    hjxo_claw C;
    memset(&C, 0, sizeof C);
    C.dim = dim;
    for (int d = 0; d < dim; ++d) {
        C.gmin[d] = -1.0;
        C.gmax[d] = 1.0 + 0.5 * d;
        C.n[d] = n[d];
        C.c[d] = d % 2 ? -0.7 : 1.1;
    }
    C.periodic_mask = per;
    C.flux = flux;
    C.cfl = 0.9;
    long total = 1;
    for (int d = 0; d < dim; ++d) total *= n[d];
    double *v = malloc(sizeof(double) * total), *out = malloc(sizeof(double) * total);
    for (long f = 0; f < total; ++f) v[f] = sin(0.9 * f) + 0.2;
    double dt = 0.0;
    long steps = hjxo_claw_solve(&C, v, 4.5 * hjxo_claw_dt(&C, v), out, &dt);
    int bad = steps != 5;
    for (long f = 0; f < total && !bad; ++f) bad = !isfinite(out[f]);
    free(v); free(out);
    if (bad) fprintf(stderr, "failed: claw dim %d flux %d\n", dim, flux);
    return bad;
}

int main(void)
{
    hjxo_set_threads(2);
    const int schemes[4] = {1, 2, 3, 5};
    int bad = 0;
    for (int s = 0; s < 4; ++s)
        for (int rk = 1; rk <= 3; ++rk) {
            const long n1[1] = {3}, n2[2] = {4, 9}, n3[3] = {5, 4, 6}, n4[4] = {3, 4, 5, 3};
            bad |= run(1, n1, 1u, 0, schemes[s], rk);
            bad |= run(2, n2, 0u, 0, schemes[s], rk);
            bad |= run(3, n3, 4u, 1, schemes[s], rk);
            bad |= run(4, n4, 4u, 2, schemes[s], rk);
            bad |= run(3, n3, 0u, 3, schemes[s], rk);
            for (int r = 1; r <= 2; ++r) bad |= run_opts(2, n2, 1u, 0, schemes[s], rk, r, 0);
            bad |= run_opts(3, n3, 4u, 1, schemes[s], rk, 0, 1);
            bad |= run_opts(3, n3, 0u, 3, schemes[s], rk, 2, 1);
            bad |= run_opts(2, n2, 2u, 0, schemes[s], rk, 0, 2);
            bad |= run_opts(1, n1, 0u, 0, schemes[s], rk, 1, 2);
        }
    for (int flux = 0; flux <= 1; ++flux) {
        const long c1[1] = {3}, c2[2] = {4, 7}, c3[3] = {3, 5, 4}, c4[4] = {3, 3, 4, 5};
        bad |= run_claw(1, c1, 1u, flux);
        bad |= run_claw(2, c2, 0u, flux);
        bad |= run_claw(3, c3, 5u, flux);
        bad |= run_claw(4, c4, 15u, flux);
    }
    for (int s = 0; s < 4; ++s)
        for (long n = 3; n <= 9; ++n)
            for (int per = 0; per <= 1; ++per) {
                double line[9], pm[9], pp[9];
                for (long i = 0; i < n; ++i) line[i] = (double)(i * i) - 0.5 * (double)i;
                bad |= hjxo_deriv_line(schemes[s], line, n, per, 0.25, pm, pp) != 0;
            }
    printf(bad ? "oracle sanitized run: FAILED\n" : "oracle sanitized run: ok\n");
    return bad;
}
