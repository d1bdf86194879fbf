"""Pins of the oracle's implicit surfaces and shape operations (Sec. III):
the ball is a signed distance (zero on the sphere, unit gradient away from the
centre, the exact distance along rays), the cylinder ignores the axes it
leaves out, Listing 2's ellipsoid matches its printed terms, and the
operations obey the set algebra they stand for (De Morgan, subtraction as
intersection with the complement, idempotence)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import shapes as S


def _grid(n, lo=-1.0, hi=1.0, periodic=()):
    d = len(n)
    return O.make_problem([lo] * d, [hi] * d, n, periodic=list(periodic), ham="normal", params=(1.0,))


def test_ball_is_the_signed_distance_to_a_sphere():
    P = _grid((41, 37, 33))
    c = [0.1, -0.2, 0.05]
    phi = S.shape(P, "ball", (0, 1, 2), c, 0.5)
    X = S.node_coords(P)
    r = np.sqrt(sum((X[d] - c[d]) ** 2 for d in range(3)))
    # exact distance along rays: |phi| = |r - 0.5|, sign negative inside
    np.testing.assert_allclose(phi, r - 0.5, rtol=0, atol=1e-15)
    assert (phi[r < 0.5] < 0).all() and (phi[r > 0.5] > 0).all()
    # unit gradient (central differences) away from the centre
    g = np.gradient(phi, *[O.grid(P, d)[0] for d in range(3)])
    norm = np.sqrt(sum(x ** 2 for x in g))
    mask = (r > 0.3)[1:-1, 1:-1, 1:-1]
    assert np.abs(norm[1:-1, 1:-1, 1:-1][mask] - 1).max() < 0.02


def test_cylinder_ignores_the_axes_it_leaves_out():
    P = _grid((21, 19, 7))
    phi = S.shape(P, "ball", (0, 1), [0.0, 0.3, 99.0], 0.4)
    assert np.array_equal(phi[:, :, 0:1].repeat(7, axis=2), phi)
    X = S.node_coords(P)
    np.testing.assert_allclose(phi[:, :, 3], np.hypot(X[0][:, :, 3], X[1][:, :, 3] - 0.3) - 0.4, atol=1e-15)


def test_ellipsoid_is_listing_2():
    """e = x^2 + 4 y^2 + 9 z^2 - radius (Listing 2, centred at 0)."""
    P = _grid((11, 12, 13))
    X = S.node_coords(P)
    e = S.shape(P, "ellipsoid", (0, 1, 2), [0, 0, 0], 0.8, weights=[1.0, 4.0, 9.0])
    np.testing.assert_allclose(e, X[0] ** 2 + 4.0 * X[1] ** 2 + 9.0 * X[2] ** 2 - 0.8, rtol=0, atol=1e-15)


def test_operations_obey_the_set_algebra():
    P = _grid((25, 23))
    a = S.shape(P, "ball", (0, 1), [-0.2, 0.0], 0.5)
    b = S.shape(P, "ball", (0, 1), [0.3, 0.1], 0.4)
    u, i = S.op("union", a, b), S.op("intersection", a, b)
    # interiors: union and intersection of the sets {phi < 0}
    assert np.array_equal(u < 0, (a < 0) | (b < 0))
    assert np.array_equal(i < 0, (a < 0) & (b < 0))
    # De Morgan, exactly
    assert np.array_equal(S.op("complement", u), S.op("intersection", -a, -b))
    assert np.array_equal(S.op("complement", i), S.op("union", -a, -b))
    # subtraction is the intersection with the complement
    assert np.array_equal(S.op("subtraction", a, b), S.op("intersection", a, S.op("complement", b)))
    assert np.array_equal(S.op("subtraction", a, b) < 0, (a < 0) & ~(b <= 0))
    # idempotence and the double complement
    assert np.array_equal(S.op("union", a, a), a) and np.array_equal(S.op("complement", S.op("complement", a)), a)
    with pytest.raises(ValueError):
        S.op("xor", a, b)
