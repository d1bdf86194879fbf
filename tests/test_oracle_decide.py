"""Pins of the oracle's binary32 ENO choices (make_problem(decide="f32")).

The ENO rules of Sec. IV-B compare |D^2| (and |D^3|) of two candidate
stencils and keep the smaller; that comparison turns floating-point values
into a stencil, an integer decision.  A solver that computes in binary32
takes it in binary32, and where the two candidates are closer than binary32
rounding the choice may legitimately go the other way.  The oracle can take
the choice in binary32 too (the derivative itself is still formed in
double).  These tests pin that mode against the classical construction:
away from near ties it chooses as the double mode does, every value it
returns is the derivative of one of the interpolants the ENO rule may grow,
and on a tie that only binary32 rounding creates it goes left, as printed.
"""
import itertools

import numpy as np
import pytest

import oracle as O


def _divided_difference(x, f):
    if len(x) == 1:
        return f[0]
    return (_divided_difference(x[1:], f[1:]) - _divided_difference(x[:-1], f[:-1])) / (x[-1] - x[0])


def _eno_candidates(x, f, i, side, order):
    """Derivative at node i of every interpolant the ENO rule can grow from
    the interval next to node i (side < 0: the left one), each growth step
    going either way: {(value, ambiguity)} where ambiguity is the smallest
    relative gap between the compared |divided differences| on that path."""
    out = []
    for path in itertools.product((0, 1), repeat=order - 1):
        a = i - 1 if side < 0 else i
        b = a + 1
        gap = np.inf
        for go_left in path:
            left = abs(_divided_difference(x[a - 1:b + 1], f[a - 1:b + 1]))
            right = abs(_divided_difference(x[a:b + 2], f[a:b + 2]))
            gap = min(gap, abs(left - right) / max(left, right, 1e-300))
            if go_left:
                a -= 1
            else:
                b += 1
        coef = np.polyfit(x[a:b + 1] - x[i], f[a:b + 1], b - a)
        out.append((np.polyder(coef)[-1], gap, path))
    return out


def _line_problem(n, scheme, decide):
    return O.make_problem([0.0], [float(n - 1)], [n], scheme=scheme, decide=decide)


@pytest.mark.parametrize("scheme,order", [("eno2", 2), ("eno3", 3)])
def test_binary32_choices_are_admissible_and_agree_away_from_ties(scheme, order):
    """Rough binary32 data on 1-D lines: both modes return the derivative of
    an interpolant the ENO rule may grow; they agree wherever every compared
    pair differs by more than 1e-5 relative; where they differ the binary32
    mode's choice is one the double mode did not take."""
    rng = np.random.default_rng(23)
    n = 16
    x = np.arange(n, dtype=np.float64)
    differ = 0
    for trial in range(300):
        # data on a coarse lattice makes near ties frequent
        f = (rng.integers(-40, 41, size=n) / 8.0 + rng.normal(size=n) * 1e-7 * (trial % 2))
        f = f.astype(np.float32).astype(np.float64)
        Pd = _line_problem(n, scheme, "f64")
        Pf = _line_problem(n, scheme, "f32")
        pm_d, pp_d = O.deriv_axis(Pd, f, 0)
        pm_f, pp_f = O.deriv_axis(Pf, f, 0)
        for i in range(4, n - 4):
            for side, vd, vf in ((-1, pm_d[i], pm_f[i]), (1, pp_d[i], pp_f[i])):
                cands = _eno_candidates(x, f, i, side, order)
                assert any(abs(vf - c) <= 1e-9 * (1 + abs(c)) for c, _, _ in cands), (trial, i, side)
                assert any(abs(vd - c) <= 1e-9 * (1 + abs(c)) for c, _, _ in cands), (trial, i, side)
                if vd != vf:
                    differ += 1
                    # the double mode's own path must have had a near tie
                    own = [g for c, g, _ in cands if abs(vd - c) <= 1e-9 * (1 + abs(c))]
                    assert min(own) <= 1e-5, (trial, i, side, own)
    assert differ > 0  # the lattice data do produce binary32-only ties


def test_tie_created_by_binary32_rounding_goes_left():
    """phi = (0, 0, 0, 0, 1, 1 + 1e-12, 1, 1, 1) on dx = 1.  At node 4 the
    left-biased ENO2 value compares D2_3 = 1/2 with D2_4 = -(1 - 1e-12)/2:
    in double the right candidate is smaller, 0.5 + O(1e-12); rounded to
    binary32 the data hold the exact tie 1/2 = |-1/2|, which goes left:
    D1_{3.5} + D2_3 = 1.5."""
    f = np.array([0, 0, 0, 0, 1, 1 + 1e-12, 1, 1, 1], dtype=np.float64)
    pm_d, _ = O.deriv_axis(_line_problem(9, "eno2", "f64"), f, 0)
    pm_f, _ = O.deriv_axis(_line_problem(9, "eno2", "f32"), f, 0)
    assert abs(pm_d[4] - 0.5) < 1e-9
    assert pm_f[4] == 1.5


def test_binary32_mode_changes_only_eno():
    """The mode decides stencils only: first order and WENO5 have no choice
    and give the same bits in both modes, on a 3-D grid."""
    rng = np.random.default_rng(5)
    f = rng.normal(size=(7, 9, 11)).astype(np.float32).astype(np.float64)
    for scheme in ("first", "weno5"):
        a = O.rhs(O.make_problem([0, 0, 0], [1, 1, 1], f.shape, periodic=(1,), scheme=scheme, decide="f64"), f)
        b = O.rhs(O.make_problem([0, 0, 0], [1, 1, 1], f.shape, periodic=(1,), scheme=scheme, decide="f32"), f)
        assert np.array_equal(a, b), scheme


def test_binary32_ghost_cells_on_both_ends():
    """Linear data stay exactly linear through the linearly extrapolated
    ghosts in binary32 too: every ENO choice of exactly linear data is a tie
    (all higher differences vanish) and the derivative is the slope."""
    f = (0.25 * np.arange(12) - 1.0).astype(np.float64)
    for scheme in ("eno2", "eno3"):
        pm, pp = O.deriv_axis(_line_problem(12, scheme, "f32"), f, 0)
        assert np.all(pm == 0.25) and np.all(pp == 0.25), scheme
