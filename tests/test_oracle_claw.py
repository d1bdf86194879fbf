"""Pins of the oracle's conservation-law Lax-Friedrichs scheme (Sec. IV-D):
v_t + sum_d f_d(v)_{x_d} = 0 with linear (f = c v) and Burgers (f = c v^2/2)
fluxes.

Each pin is fixed by the mathematics, not by the scheme's own formula: at
lambda c = +-1 the scheme is the exact shift of linear advection; a periodic
grid conserves the sum; a monotone scheme obeys the maximum principle; the
Burgers shock moves at the Rankine-Hugoniot speed and the rarefaction
approaches the self-similar fan; linear data under a linear flux is advected
exactly away from the edges; the CFL step is the printed condition.
"""
import math

import numpy as np
import pytest

import oracle as O


def _line(n, flux, c, cfl, periodic=True, lo=0.0, hi=1.0):
    return O.make_claw([lo], [hi], [n], periodic=[0] if periodic else [], flux=flux, c=[c], cfl=cfl)


@pytest.mark.parametrize("c", [1.0, -1.0])
def test_linear_advection_at_cfl_one_is_the_exact_shift(c):
    """lambda c = +-1: (v_{j+1} + v_{j-1})/2 -+ (v_{j+1} - v_{j-1})/2 is
    v_{j-1} or v_{j+1}: the exact solution on the grid."""
    n = 64
    C = _line(n, "linear", c, 1.0)
    x = np.arange(n) / n
    v = np.exp(np.sin(2 * np.pi * x)) + 0.3 * np.cos(6 * np.pi * x)
    dt = O.claw_dt(C, v)
    assert dt == pytest.approx(1.0 / n, rel=1e-15)
    out, steps, _ = O.claw_solve(C, v, 17 * dt)
    assert steps == 17
    np.testing.assert_allclose(out, np.roll(v, 17 if c > 0 else -17), rtol=0, atol=1e-13)


def test_edge_value_flows_in_through_a_non_periodic_edge():
    """Beyond a non-periodic edge the value is the edge value, so at
    lambda c = 1 the inflow node keeps its value and the exact shift carries
    it in: v_j^n = v_{max(j - n, 0)}^0."""
    n = 40
    C = _line(n, "linear", 1.0, 1.0, periodic=False)
    v = np.cos(np.arange(n) * 0.37) + 2.0
    dt = O.claw_dt(C, v)
    out, steps, _ = O.claw_solve(C, v, 9 * dt)
    assert steps == 9
    np.testing.assert_allclose(out, v[np.maximum(np.arange(n) - 9, 0)], rtol=0, atol=1e-14)


@pytest.mark.parametrize("flux", ["linear", "burgers"])
@pytest.mark.parametrize("shape", [(97,), (23, 19), (9, 8, 7)])
def test_periodic_grid_conserves_the_sum(flux, shape):
    """sum_j v_j^{n+1} = sum_j v_j^n: the neighbour means sum to the total
    and the flux differences telescope around a periodic grid."""
    rng = np.random.default_rng(3)
    C = O.make_claw([0] * len(shape), [1] * len(shape), shape, periodic=list(range(len(shape))), flux=flux,
                    c=[0.7, -1.3, 0.4][:len(shape)], cfl=0.9)
    v = rng.normal(size=shape)
    out, steps, _ = O.claw_solve(C, v, 6.5 * O.claw_dt(C, v))
    assert steps == 7
    assert abs(out.sum() - v.sum()) < 1e-12 * np.abs(v).sum()


@pytest.mark.parametrize("flux", ["linear", "burgers"])
@pytest.mark.parametrize("shape,periodic", [((101,), ()), ((31, 27), (0,)), ((12, 11, 10), (0, 1, 2))])
def test_monotone_scheme_obeys_the_maximum_principle(flux, shape, periodic):
    """Under the CFL condition every new value is a convex combination of
    old neighbour values (for Burgers, by the mean value theorem), so the
    range never widens; rough data makes the check bite."""
    rng = np.random.default_rng(11)
    C = O.make_claw([0] * len(shape), [1] * len(shape), shape, periodic=list(periodic), flux=flux,
                    c=[1.0, -0.6, 0.8][:len(shape)], cfl=0.8)   # below 1: not the exact shift
    v = rng.uniform(-1, 2, size=shape)
    dt = O.claw_dt(C, v)
    cur = v
    for _ in range(6):
        nxt = O.claw_step(C, cur, dt)
        assert nxt.min() >= cur.min() - 1e-14 and nxt.max() <= cur.max() + 1e-14
        cur = nxt
    assert cur.max() < v.max() - 0.1 and cur.min() > v.min() + 0.1


def test_linear_data_is_advected_exactly_away_from_the_edges():
    """v = a + b.x with f_d = c_d v: the neighbour mean is v itself and the
    central differences are exact, so v^{n+1} = v - dt c.b at every node
    whose neighbours are inside the grid."""
    C = O.make_claw([-1, 0], [1, 3], [21, 17], flux="linear", c=[0.8, -1.7], cfl=0.8)
    x = np.linspace(-1, 1, 21)[:, None]
    y = np.linspace(0, 3, 17)[None, :]
    v = 0.3 + 1.1 * x - 0.4 * y
    dt = O.claw_dt(C, v)
    out = O.claw_step(C, v, dt)
    want = v - dt * (0.8 * 1.1 + (-1.7) * (-0.4))
    np.testing.assert_allclose(out[1:-1, 1:-1], want[1:-1, 1:-1], rtol=0, atol=1e-14)


def test_cfl_step_is_the_printed_condition():
    """dt = cfl min_d dx_d / (N max|f_d'|): lambda_d max|f_d'| <= 1/N per
    axis, the printed lambda max|f'| <= 1 for one axis."""
    C = O.make_claw([0, 0], [2, 1], [41, 21], flux="burgers", c=[1.5, 0.5], cfl=0.8)
    v = np.zeros((41, 21))
    v[3, 4] = -2.5
    dxs = [2 / 40, 1 / 20]
    want = 0.8 * min(dxs[0] / (2 * 1.5 * 2.5), dxs[1] / (2 * 0.5 * 2.5))
    assert O.claw_dt(C, v) == pytest.approx(want, rel=1e-15)
    assert O.claw_dt(C, np.zeros((41, 21))) == math.inf


def _riemann(n, ul, ur, t):
    C = _line(n, "burgers", 1.0, 0.9, periodic=False, lo=-1.0, hi=1.0)
    x = np.linspace(-1, 1, n)
    v0 = np.where(x < 0, ul, ur)
    out, _, _ = O.claw_solve(C, v0, t)
    return x, out


def test_burgers_shock_moves_at_the_rankine_hugoniot_speed():
    """u_L = 1, u_R = 0: the shock speed is (u_L + u_R)/2 = 1/2, so at
    t = 0.6 the jump sits at x = 0.3; the smeared profile crosses 1/2 there
    to within a few cells, and the L1 error falls as the grid is refined."""
    errs = []
    for n in (201, 801):
        x, v = _riemann(n, 1.0, 0.0, 0.6)
        exact = np.where(x < 0.3, 1.0, 0.0)
        k = np.argmax(v < 0.5)
        assert abs(x[k] - 0.3) < 4 * (x[1] - x[0])
        errs.append(np.abs(v - exact).mean() * 2)
    assert errs[1] < errs[0] / 2


def test_burgers_rarefaction_approaches_the_fan():
    """u_L = 0, u_R = 1: v = clamp(x/t, 0, 1); the L1 error falls with the
    grid (a first-order scheme through the fan's corners: about dx^0.5 or
    better)."""
    errs = []
    for n in (101, 401, 1601):
        x, v = _riemann(n, 0.0, 1.0, 0.5)
        exact = np.clip(x / 0.5, 0.0, 1.0)
        errs.append(np.abs(v - exact).mean() * 2)
    rates = [math.log2(errs[i] / errs[i + 1]) / 2 for i in range(2)]
    assert all(r > 0.4 for r in rates), (errs, rates)


def test_bad_arguments_are_rejected():
    C = _line(10, "burgers", 1.0, 0.9)
    v = np.zeros(10)
    C.cfl = 1.5
    with pytest.raises(ValueError):
        O.claw_step(C, v, 0.01)
    C = _line(10, "burgers", 1.0, 0.9)
    C.flux = 7
    with pytest.raises(ValueError):
        O.claw_dt(C, v)
