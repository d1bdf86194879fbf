"""Scalar conservation laws on the GPU (Sec. IV-D, the Lax-Friedrichs
scheme; hjx_claw_* through the C ABI) against the oracle element by element:
linear and Burgers fluxes, 1-D to 4-D, periodic and edge-value axes, ragged
sizes, both precisions; the 4096^2 Burgers workload of the benchmark one
step at every node; conservation, the maximum principle and the error
paths."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_03501_amd import inputs
from helpers import assert_close, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_03501_amd import hjx  # noqa: E402

TDT = {"f32": torch.float32, "f64": torch.float64}

CASES = [
    ((1000,), (0,)),
    ((301,), ()),
    ((67, 45), (0, 1)),
    ((67, 45), (1,)),
    ((19, 23, 17), (0, 2)),
    ((9, 11, 8, 7), (0, 1, 2, 3)),
    ((9, 11, 8, 7), ()),
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def data(shape, seed):
    """Smooth bumps plus a jump and some noise: both fluxes move it and the
    Burgers flux steepens it."""
    v = 1.0 + 0.6 * inputs.smooth_field(shape, seed) + 0.1 * inputs.rough_field(shape, seed + 1)
    v[tuple(slice(0, n // 3) for n in shape)] += 0.8
    return v


def pair(shape, periodic, flux, dtype, cfl=0.9):
    d = len(shape)
    c = [1.0, -0.7, 0.5, 1.3][:d]
    lo, hi = [-1.0] * d, [1.0 + 0.5 * k for k in range(d)]
    C = O.make_claw(lo, hi, shape, periodic=list(periodic), flux=flux, c=c, cfl=cfl)
    G = hjx.Claw(lo, hi, shape, periodic=periodic, flux=flux, c=c, cfl=cfl, dtype=dtype)
    return C, G


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("flux", ["linear", "burgers"])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_claw_solve_matches_the_oracle(ci, flux, dtype):
    shape, periodic = CASES[ci]
    say(f"claw {shape} periodic={periodic} {flux} {dtype}")
    C, G = pair(shape, periodic, flux, dtype)
    v0d = to_dev(data(shape, 5 + ci), TDT[dtype])
    v0 = to_host(v0d)                     # the oracle starts from the same (rounded) values
    dt = O.claw_dt(C, v0)
    assert G.dt(v0d) == pytest.approx(dt, rel=1e-12 if dtype == "f64" else 1e-6)
    t1 = 9.5 * dt
    ref, n_ref, _ = O.claw_solve(C, v0, t1)
    got, st = G.solve(v0d, t1)
    assert st["steps"] == n_ref == 10
    assert_close(to_host(got), ref, dtype, periodic, f"claw {shape} {flux}")
    assert np.abs(ref - v0).max() > 1e-2
    G.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("flux", ["linear", "burgers"])
def test_claw_step_matches_the_oracle_and_conserves(flux, dtype):
    shape, periodic = (40, 33, 21), (0, 1, 2)
    C, G = pair(shape, periodic, flux, dtype)
    v = to_dev(data(shape, 17), TDT[dtype])
    dt = G.dt(v)
    out = G.step(v, dt)
    ref = O.claw_step(C, to_host(v), dt)
    assert_close(to_host(out), ref, dtype, periodic, f"claw step {flux}")
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert abs(float(out.double().sum() - v.double().sum())) <= tol * float(v.double().abs().sum())
    G.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_full_size_burgers_4096(dtype):
    """The benchmark's workload, 4096^2 periodic Burgers: one step against
    the oracle at every node, then steps that keep the range (the maximum
    principle)."""
    w = inputs.BURGERS2D
    v0 = inputs.burgers_initial(w)
    G = hjx.Claw(w.gmin, w.gmax, w.n, periodic=w.periodic, flux="burgers", c=w.params, cfl=w.cfl, dtype=dtype)
    C = O.make_claw(w.gmin, w.gmax, w.n, periodic=list(w.periodic), flux="burgers", c=w.params, cfl=w.cfl)
    vd = to_dev(v0, TDT[dtype])
    dt = G.dt(vd)
    say(f"burgers 4096^2 {dtype}: oracle step")
    ref = O.claw_step(C, to_host(vd), dt)
    out = G.step(vd, dt)
    assert_close(to_host(out), ref, dtype, w.periodic, "burgers 4096^2")
    lo, hi = float(vd.min()), float(vd.max())
    cur = out
    for _ in range(5):
        cur = G.step(cur, dt)
    slack = 1e-12 if dtype == "f64" else 1e-6
    assert float(cur.min()) >= lo - slack * abs(lo) and float(cur.max()) <= hi + slack * abs(hi)
    G.close()


def test_claw_errors():
    C, G = pair((30, 20), (0,), "burgers", "f64")
    v = to_dev(data((30, 20), 1), torch.float64)
    with pytest.raises(hjx.HjxError, match="aliases"):
        G.solve(v, 0.1, out=v)
    with pytest.raises(hjx.HjxError, match="aliases"):
        G.step(v, 0.01, out=v)
    with pytest.raises(hjx.HjxError, match="t1"):
        G.solve(v, -1.0)
    bad = v.clone()
    bad[3, 4] = float("nan")
    with pytest.raises(hjx.HjxError) as e:
        G.solve(bad, 0.1)
    assert e.value.status == hjx.HJX_ERR_NONFINITE
    # t1 = 0: a copy; still usable after the errors
    out, st = G.solve(v, 0.0)
    assert st["steps"] == 0 and torch.equal(out, v)
    out, st = G.solve(v, 0.05)
    ref, n, _ = O.claw_solve(C, to_host(v), 0.05)
    assert st["steps"] == n
    assert_close(to_host(out), ref, "f64", (0,), "after errors")
    G.close()
