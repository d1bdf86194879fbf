"""The steps variant of 1-D and 2-D grids (several whole RK steps per
launch, the halo evaluated again by neighbouring blocks): every solve gives
the bits of the direct variant's solve, which takes one launch per stage.
Covered: all four schemes, RK1/2/3, periodic and non-periodic axes in every
combination, min-with-target, both restricted updates, local Lax-Friedrichs
and Godunov's Hamiltonian, FP32 and FP64, tiles that do not divide the
grid or exceed it, launches of fewer steps than the tile's own (the solve's
step count not a multiple of it, and its clamped last step), in place and
out of place, graph replays; and the oracle's result."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2411_03501_amd import inputs
from helpers import assert_close, gpu_problem, oracle_problem, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - only on a GPU machine
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_03501_amd import hjx  # noqa: E402

TDT = {"f32": torch.float32, "f64": torch.float64}
RADIUS = {"first": 1, "eno2": 2, "eno3": 3, "weno5": 3}
DIRECT = (hjx.TILE_DIRECT, 256, 1, 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _w(name, gmin, gmax, n, periodic=(), params=(1.3,), scheme="first", rk=1, **kw):
    w = inputs.Workload(name, tuple(gmin), tuple(gmax), tuple(n), tuple(periodic), "normal", tuple(params), scheme,
                        rk)
    return w.with_(**kw) if kw else w


GRIDS = {
    "1d": _w("1d", [-1], [2], [37]),
    "1d_per": _w("1d_per", [0], [1], [41], periodic=(0,), params=(-0.7,)),
    "2d": _w("2d", [-1, -2], [1, 1], [29, 23], params=(0.9,)),
    "2d_per0": _w("2d_per0", [0, -1], [1, 1], [26, 19], periodic=(0,), params=(1.1,)),
    "2d_per1": _w("2d_per1", [-1, 0], [1, 1], [17, 31], periodic=(1,), params=(-0.8,)),
    "2d_per01": _w("2d_per01", [0, 0], [1, 1], [24, 27], periodic=(0, 1), params=(0.7,)),
}
TILES_2D = [(16, 16), (8, 8), (5, 7), (32, 32), (64, 4), (1, 1)]
TILES_1D = [(256, 1), (16, 1), (7, 1), (1, 1)]


def _ok_tile(w, tile, k):
    """Whether the steps variant takes this shape: a halo of k * rk * radius
    nodes no deeper than a periodic axis and at most 64 KiB of LDS."""
    H = k * w.rk * RADIUS[w.scheme]
    return all(H <= w.n[d] for d in w.periodic)


def _solve(P, phi, t1, tgt, dtype, inplace=False):
    d0 = to_dev(phi, TDT[dtype])
    target = to_dev(tgt, TDT[dtype]) if tgt is not None else None
    if inplace:
        out, st = P.solve(d0, t1, target=target, out=d0)
    else:
        out, st = P.solve(d0, t1, target=target)
    return out.cpu(), st


@pytest.mark.parametrize("grid", sorted(GRIDS))
@pytest.mark.parametrize("scheme,rk", [("first", 1), ("first", 3), ("eno2", 2), ("eno3", 3), ("weno5", 1),
                                       ("weno5", 3)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_steps_variant_gives_the_direct_bits(grid, scheme, rk, dtype):
    w = GRIDS[grid].with_(scheme=scheme, rk=rk)
    phi = inputs.rough_field(w.n, 31)
    tgt = inputs.rough_field(w.n, 32)
    P = gpu_problem(w, dtype)
    t1 = 6.5 * P.dissipation()[1]  # 7 steps, the last clamped
    P.tile = DIRECT
    ref, st = _solve(P, phi, t1, tgt, dtype)
    assert st["steps"] == 7
    ref_nt, _ = _solve(P, phi, t1, None, dtype)
    tiles = TILES_1D if w.dim == 1 else TILES_2D
    checked = 0
    for tx, ty in tiles:
        for k in (1, 2, 3, 4, 8):
            if not _ok_tile(w, (tx, ty), k):
                continue
            try:
                P.tile = (hjx.TILE_STEPS, tx, ty, k)
            except hjx.HjxError as e:  # more LDS than a block may take
                assert e.status == hjx.HJX_ERR_INVALID_ARG
                continue
            say(grid, scheme, rk, dtype, "tile", tx, ty, "steps", k)
            got, st = _solve(P, phi, t1, tgt, dtype)
            assert st["steps"] == 7
            assert torch.equal(got, ref), (grid, scheme, rk, dtype, tx, ty, k, "target")
            got, _ = _solve(P, phi, t1, None, dtype)
            assert torch.equal(got, ref_nt), (grid, scheme, rk, dtype, tx, ty, k, "no target")
            checked += 1
    assert checked >= 4


@pytest.mark.parametrize("over", [dict(restrict="nonpositive"), dict(restrict="positive"),
                                  dict(dissipation="local"), dict(dissipation="local", restrict="nonpositive"),
                                  dict(dissipation="godunov"), dict(dissipation="godunov", restrict="positive")])
@pytest.mark.parametrize("grid", ["1d_per", "2d", "2d_per01"])
def test_steps_variant_node_modes(grid, over):
    """The restricted updates, local dissipation and Godunov's Hamiltonian
    in the steps variant: the direct variant's bits, FP64 and FP32."""
    w = GRIDS[grid].with_(scheme="eno2", rk=2, **over)
    phi = inputs.rough_field(w.n, 41)
    tgt = inputs.rough_field(w.n, 42)
    for dtype in ("f64", "f32"):
        P = gpu_problem(w, dtype)
        t1 = 4.5 * P.dissipation()[1]
        P.tile = DIRECT
        ref, _ = _solve(P, phi, t1, tgt, dtype)
        for tile in ([(hjx.TILE_STEPS, 16, 1, 2), (hjx.TILE_STEPS, 5, 1, 3)] if w.dim == 1 else
                     [(hjx.TILE_STEPS, 16, 16, 2), (hjx.TILE_STEPS, 7, 3, 1)]):
            P.tile = tile
            got, _ = _solve(P, phi, t1, tgt, dtype)
            assert torch.equal(got, ref), (grid, over, dtype, tile)


def test_steps_variant_in_place_graphs_and_the_oracle(monkeypatch):
    """In place and out of place, direct launches, graph capture and replays,
    a single launch (the whole solve within one tile's steps, read and
    written in place), and the oracle within the FP64 bound."""
    w = GRIDS["2d_per1"].with_(scheme="weno5", rk=3)
    phi = inputs.smooth_field(w.n, 51, amplitude=1.5)
    P = gpu_problem(w, "f64")
    t1 = 4.5 * P.dissipation()[1]
    P.tile = DIRECT
    ref, st = _solve(P, phi, t1, phi, "f64")
    assert st["steps"] == 5
    for tile in [(hjx.TILE_STEPS, 8, 8, 1), (hjx.TILE_STEPS, 16, 16, 1)]:
        P.tile = tile
        d0 = to_dev(phi, torch.float64)
        tg = d0.clone()
        out = torch.empty_like(d0)
        for rep in range(4):  # direct launches, capture, replays
            got, _ = P.solve(d0, t1, target=tg, out=out)
            assert torch.equal(got.cpu(), ref), (tile, rep)
        monkeypatch.setenv("HJX_SOLVE_GRAPH", "0")
        x = d0.clone()
        P.solve(x, t1, target=tg, out=x)
        assert torch.equal(x.cpu(), ref), (tile, "in place")
        monkeypatch.delenv("HJX_SOLVE_GRAPH")
    # every step in one launch: 5 steps of first order RK1 on a grid whose
    # periodic axis holds the halo
    w1 = GRIDS["2d_per01"]
    phi1 = inputs.rough_field(w1.n, 52)
    P1 = gpu_problem(w1, "f64")
    t11 = 4.5 * P1.dissipation()[1]
    P1.tile = DIRECT
    r1, _ = _solve(P1, phi1, t11, None, "f64")
    P1.tile = (hjx.TILE_STEPS, 32, 32, 8)
    for inplace in (False, True):
        got, st = _solve(P1, phi1, t11, None, "f64", inplace=inplace)
        assert st["steps"] == 5 and torch.equal(got, r1), inplace
    oref, steps, _ = O.solve(oracle_problem(w), phi, t1, target=phi)
    assert steps == 5
    assert_close(to_host(ref), oref, "f64", w.periodic, what="steps variant against the oracle")


def test_steps_tile_validation():
    w = GRIDS["2d_per01"].with_(scheme="weno5", rk=3)
    P = gpu_problem(w, "f64")
    with pytest.raises(hjx.HjxError):  # a halo of 3 * 3 * 3 = 27 nodes, deeper than the 24-node periodic axis
        P.tile = (hjx.TILE_STEPS, 8, 8, 3)
    with pytest.raises(hjx.HjxError):  # 3 buffers of (64 + 18)^2 doubles: more than 64 KiB
        P.tile = (hjx.TILE_STEPS, 64, 64, 2)
    with pytest.raises(hjx.HjxError):
        P.tile = (hjx.TILE_STEPS, 8, 0, 1)
    with pytest.raises(hjx.HjxError):
        P.tile = (hjx.TILE_STEPS, 8, 8, 0)
    P.tile = (hjx.TILE_STEPS, 8, 8, 2)
    assert P.tile == (hjx.TILE_STEPS, 8, 8, 2)
    w1 = GRIDS["1d"]
    P1 = gpu_problem(w1, "f64")
    with pytest.raises(hjx.HjxError):  # 1-D tiles have ty = 1
        P1.tile = (hjx.TILE_STEPS, 8, 2, 1)
    w3 = _w("3d", [0, 0, 0], [1, 1, 1], [5, 6, 7])
    P3 = gpu_problem(w3, "f64")
    with pytest.raises(hjx.HjxError) as e:
        P3.tile = (hjx.TILE_STEPS, 8, 8, 1)
    assert e.value.status == hjx.HJX_ERR_UNSUPPORTED
    # the default for a small 2-D grid is the steps variant
    assert gpu_problem(GRIDS["2d"], "f64").tile[0] == hjx.TILE_STEPS


@pytest.mark.parametrize("tile", [(hjx.TILE_STEPS, 8, 8, 4), (hjx.TILE_STEPS, 16, 16, 1), DIRECT])
def test_nonfinite_checks(tile):
    """hjx_solve reports NaN/Inf in phi0 and in its result, whether the checks
    are separate launches (direct) or run inside the first and last launches
    of the steps variant; the result is written either way.  A finite spike
    of +-1e308 overflows the differences of the first step."""
    w = GRIDS["2d"]
    P = gpu_problem(w, "f64")
    P.tile = tile
    t1 = 3.5 * P.dissipation()[1]
    phi = inputs.smooth_field(w.n, 61)
    bad_in = phi.copy()
    bad_in[5, 7] = np.nan
    with pytest.raises(hjx.HjxError) as e:
        P.solve(to_dev(bad_in, torch.float64), t1)
    assert e.value.status == hjx.HJX_ERR_NONFINITE and "phi0" in str(e.value)
    spike = phi.copy()
    spike[10, 10], spike[10, 11] = 1e308, -1e308
    out = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    with pytest.raises(hjx.HjxError) as e:
        P.solve(to_dev(spike, torch.float64), t1, out=out)
    assert e.value.status == hjx.HJX_ERR_NONFINITE and "solution" in str(e.value)
    assert not torch.isfinite(out).all() and torch.isfinite(out).any()
    ok, st = P.solve(to_dev(phi, torch.float64), t1)   # a clean solve after the errors
    assert st["steps"] == 4 and torch.isfinite(ok).all()
