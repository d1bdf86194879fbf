"""The two-rocket game (Sec. VI) on the GPU through the C ABI, against the
oracle element by element: every derivative scheme and RK order, both
precisions, ragged sizes, with and without the listing's positive restricted
update and a target, every launch shape, and one step of the full 100^3
workload at every node.  Its adjoint and its place in a batch are tested in
test_adjoint_gpu.py and test_batch_gpu.py."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_03501_amd import inputs
from helpers import assert_close, gpu_problem, oracle_problem, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_03501_amd import hjx  # noqa: E402

TDT = {"f32": torch.float32, "f64": torch.float64}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small(n=(21, 19, 17), **kw):
    """The rockets workload on a coarse ragged grid, with a capture radius
    a few cells wide."""
    return inputs.ROCKETS.with_(n=n, radius=20.0, **kw)


def field(w, seed):
    return inputs.initial_surface(w) + 4.0 * inputs.smooth_field(w.n, seed)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme,rk", [("first", 1), ("eno2", 2), ("eno3", 3), ("weno5", 3)])
@pytest.mark.parametrize("restrict", ["none", "positive"])
def test_rockets_solve_matches_the_oracle(restrict, scheme, rk, dtype):
    w = small(scheme=scheme, rk=rk, restrict=restrict)
    say(f"rockets {scheme} rk{rk} {dtype} {restrict} n={w.n}")
    phi0 = field(w, 13)
    Po = oracle_problem(w)
    t1 = 6.5 * O.cfl_dt(Po)
    target = phi0 + 1.0 if restrict == "none" else None
    ref, n_ref, _ = O.solve(Po, phi0, t1, target=target)
    P = gpu_problem(w, dtype)
    got, st = P.solve(to_dev(phi0, TDT[dtype]), t1, target=None if target is None else to_dev(target, TDT[dtype]))
    assert st["steps"] == n_ref == 7
    assert_close(to_host(got), ref, dtype, w.periodic, f"rockets {scheme} rk{rk} {restrict}")
    assert np.abs(ref - phi0).max() > 0.1       # it moved
    P.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rockets_dissipation_matches_the_oracle(dtype):
    w = inputs.ROCKETS
    alpha, dt = gpu_problem(w, dtype).dissipation()
    Po = oracle_problem(w)
    tol = 1e-12 if dtype == "f64" else 1e-5
    np.testing.assert_allclose(alpha, O.alpha(Po), rtol=tol)
    assert dt == pytest.approx(O.cfl_dt(Po), rel=tol)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["eno2", "weno5"])
def test_rockets_launch_shape_does_not_change_results(scheme, dtype):
    w = small(n=(23, 18, 20), scheme=scheme, rk=2, restrict="positive")
    phi0 = to_dev(field(w, 4), TDT[dtype])
    P = gpu_problem(w, dtype)
    t1 = 4.5 * P.dissipation()[1]
    P.tile = (1, 256, 1, 1)
    ref, _ = P.solve(phi0, t1)
    ref = ref.clone()
    for tile in [(0, 11, 3, 2), (0, 20, 12, 1), (0, 32, 8, 4)]:
        P.tile = tile
        got, _ = P.solve(phi0, t1)
        assert torch.equal(got, ref), tile
    P.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_size_rockets_step(dtype):
    """The 100^3 workload as the benchmark runs it (ENO2, RK2, the positive
    restricted update): one step from the capture cylinder against the
    oracle at every node."""
    w = inputs.ROCKETS
    phi0 = inputs.initial_surface(w)
    Po = oracle_problem(w)
    dt = O.cfl_dt(Po)
    say(f"full-size rockets {dtype}: oracle step")
    ref = O.step(Po, phi0, dt)
    P = gpu_problem(w, dtype)
    got = P.step(to_dev(phi0, TDT[dtype]), dt)
    assert_close(to_host(got), ref, dtype, w.periodic, f"rockets 100^3 {dtype}")
    assert (ref >= phi0 - 1e-12).all() and (ref > phi0 + 1e-6).any()
    P.close()
