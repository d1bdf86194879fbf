"""Pins of the oracle's Godunov numerical Hamiltonian for normal motion,
H = a|p| (the dissipation kind "godunov"): on each axis the extremum of H
over the interval between p- and p+ -- the minimum for the convex a >= 0, the
maximum for a < 0 -- combined as a sqrt(sum q_d^2).

Fixed by properties, not the formula: consistency (p- = p+ = p gives a|p|),
pure upwinding for monotone data, brute force over the interval in one
dimension, the comparison principle, and convergence to the closed-form
expanding and shrinking circles with less error than Lax-Friedrichs.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2411_03501_amd import inputs

SCHEMES = ["first", "eno2", "eno3", "weno5"]


def _p(n, a, scheme="first", rk=1, diss="godunov", lo=-1.0, hi=1.0, periodic=()):
    d = len(n)
    return O.make_problem([lo] * d, [hi] * d, n, periodic=list(periodic), ham="normal", params=(a,), scheme=scheme,
                          rk=rk, dissipation=diss)


@pytest.mark.parametrize("a", [1.3, -0.7])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_consistency_on_linear_data(scheme, a):
    """p- = p+ = grad phi for linear data, so Hhat = a |grad phi| exactly
    (to rounding) at every node, and L = -a |grad phi|."""
    P = _p((17, 13), a, scheme)
    x = np.linspace(-1, 1, 17)[:, None]
    y = np.linspace(-1, 1, 13)[None, :]
    phi = 0.6 * x - 0.8 * y + 0.1
    np.testing.assert_allclose(O.rhs(P, phi), -a * 1.0 + 0 * phi, rtol=0, atol=1e-13)


def _interval_bruteforce(pm, pp, a, k=2001):
    """Godunov's flux in one dimension: min of a|p| over [pm, pp] if pm <= pp,
    max over [pp, pm] otherwise (a grid that contains both ends and 0)."""
    lo, hi = min(pm, pp), max(pm, pp)
    ps = np.concatenate([np.linspace(lo, hi, k), [0.0] if lo <= 0 <= hi else []])
    h = a * np.abs(ps)
    return h.min() if pm <= pp else h.max()


@pytest.mark.parametrize("a", [1.0, -1.0, 2.5, -0.4])
def test_one_dimensional_flux_is_the_extremum_over_the_interval(a):
    """On a 1-D line with first-order differences, -L at node j is the
    extremum of a|p| over the interval between the two one-sided slopes."""
    rng = np.random.default_rng(5)
    n = 41
    P = _p((n,), a, periodic=(0,))
    phi = rng.normal(size=n)
    dx = 2.0 / n
    L = O.rhs(P, phi)
    for j in range(n):
        pm = (phi[j] - phi[j - 1]) / dx
        pp = (phi[(j + 1) % n] - phi[j]) / dx
        assert -L[j] == pytest.approx(_interval_bruteforce(pm, pp, a), rel=1e-12, abs=1e-12), j


def test_monotone_data_is_pure_upwinding():
    """phi increasing along the line, a > 0: information comes from the left,
    and Hhat = a p- (the backward difference); a < 0: Hhat = a p+."""
    n = 30
    x = np.linspace(-1, 1, n)
    phi = np.exp(x) + x
    dx = 2.0 / (n - 1)
    pm = np.diff(phi)[:-1] / dx     # backward difference at nodes 1..n-2
    pp = np.diff(phi)[1:] / dx      # forward difference at nodes 1..n-2
    np.testing.assert_allclose(-O.rhs(_p((n,), 1.5), phi)[1:-1], 1.5 * pm, rtol=1e-13)
    np.testing.assert_allclose(-O.rhs(_p((n,), -1.5), phi)[1:-1], -1.5 * pp, rtol=1e-13)


@pytest.mark.parametrize("a", [1.0, -1.0])
def test_comparison_principle(a):
    """Godunov's flux is monotone (nonincreasing in p+, nondecreasing in p-),
    so under the CFL step phi <= psi gives S(phi) <= S(psi)."""
    n = (23, 19)
    P = _p(n, a, periodic=(0, 1))
    dt = O.cfl_dt(P)
    rng = np.random.default_rng(13)
    for trial in range(3):
        phi = rng.uniform(-1, 1, size=n) * (1 + 3 * trial)
        psi = phi + rng.uniform(0, 0.4, size=n) * (rng.uniform(size=n) < 0.3)
        assert (O.step(P, phi, dt) <= O.step(P, psi, dt) + 1e-12).all(), trial


@pytest.mark.parametrize("a", [1.0, -1.0])
def test_circle_converges_to_the_closed_form_with_less_error_than_lf(a):
    """phi0 = |x| - 0.5: expanding (a = 1), phi = max(|x| - tau, 0) - 0.5;
    shrinking (a = -1), phi = |x| - 0.5 + tau away from the centre.  First
    order, forward Euler; the error on nodes away from the centre (where
    the expanding solution is flat and the kink sits) and more than tau from
    the edges (a shrinking front carries the ghost cells' error inwards)
    falls at first order and stays below Lax-Friedrichs's."""
    tau = 0.3
    errs = {"godunov": [], "global": []}
    for n in (41, 81, 161):
        w = inputs.NORMAL2D.with_(n=(n, n))
        ax = inputs.node_axes(w)
        X, Y = np.meshgrid(*ax, indexing="ij")
        r = np.hypot(X, Y)
        phi0 = r - 0.5
        exact = (np.maximum(r - tau, 0) - 0.5) if a > 0 else (r - 0.5 + tau)
        mask = (r >= 0.45) & (np.abs(X) <= 0.6) & (np.abs(Y) <= 0.6)
        for diss in errs:
            out, _, _ = O.solve(_p((n, n), a, diss=diss), phi0, tau)
            errs[diss].append(np.abs(out - exact)[mask].max())
    rates = [math.log2(errs["godunov"][i] / errs["godunov"][i + 1]) for i in range(2)]
    assert all(0.7 < r_ < 1.4 for r_ in rates), (errs, rates)
    assert all(g < l for g, l in zip(errs["godunov"], errs["global"])), errs


def test_godunov_needs_normal_motion():
    P = O.make_problem([0, 0, 0], [1, 1, 1], [5, 5, 5], ham="dubins3_pe", params=(1, 1, 1, 1), dissipation="godunov")
    with pytest.raises(ValueError):
        O.rhs(P, np.zeros((5, 5, 5)))
