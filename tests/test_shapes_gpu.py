"""Implicit surfaces and shape operations on the device (hjx_shape,
hjx_shape_op) against the oracle's definitions: balls (spheres and
cylinders) and Listing 2's ellipsoid on ragged 1-D to 4-D grids with periodic
axes, both precisions; the four operations bit for bit, in place too; and
every member of the uneven 256-member batch built on the device against the
host recipe."""
import numpy as np
import pytest

import oracle as O
from oracle import shapes as S
from paper_2411_03501_amd import inputs
from helpers import assert_close, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_03501_amd import hjx  # noqa: E402

GRIDS = [((91,), ()), ((37, 29), (1,)), ((19, 23, 17), (2,)), ((9, 11, 8, 7), (0, 3))]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind,axes", [("ball", None), ("ball", (0, 1)), ("ellipsoid", None), ("ellipsoid", (0,))])
@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_shape_matches_the_oracle(gi, kind, axes, dtype):
    n, periodic = GRIDS[gi]
    d = len(n)
    axes = tuple(range(d)) if axes is None else tuple(a for a in axes if a < d)
    gmin, gmax = [-1.0 - 0.1 * k for k in range(d)], [1.0 + 0.2 * k for k in range(d)]
    c, w = [0.1, -0.2, 0.3, 0.0][:d], [1.0, 4.0, 9.0, 2.0][:d]
    got = hjx.shape(gmin, gmax, n, kind=kind, axes=axes, center=c, radius=0.6, weights=w, periodic=periodic,
                    dtype=dtype)
    P = O.make_problem(gmin, gmax, n, periodic=list(periodic), ham="normal", params=(1.0,))
    ref = S.shape(P, kind, axes, c, 0.6, weights=w)
    if dtype == "f64":
        np.testing.assert_allclose(to_host(got), ref, rtol=0, atol=1e-13)
    else:
        assert_close(to_host(got), ref, "f32", periodic, f"{kind} {n}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operations_match_the_oracle_bit_for_bit(dtype):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    n = (40, 33, 12)
    a = hjx.shape([-1] * 3, [1] * 3, n, axes=(0, 1), center=[-0.2, 0, 0], radius=0.5, dtype=dtype)
    b = hjx.shape([-1] * 3, [1] * 3, n, center=[0.3, 0.1, 0.0], radius=0.4, dtype=dtype)
    ah, bh = to_host(a), to_host(b)
    for op in ("union", "intersection", "complement", "subtraction"):
        got = hjx.shape_op(op, a, None if op == "complement" else b)
        want = torch.from_numpy(S.op(op, ah, bh)).to("cuda", dtype=tdt)
        assert torch.equal(got, want), op
    # in place: out aliases a
    c = a.clone()
    hjx.shape_op("subtraction", c, b, out=c)
    assert torch.equal(c, torch.from_numpy(S.op("subtraction", ah, bh)).to("cuda", dtype=tdt))


def test_batch256_initial_data_built_on_the_device():
    """Every eighth member's phi0 (a sphere over every axis or a cylinder over
    the first two, minus the member's radius) built by hjx_shape equals the
    host recipe, to rounding."""
    for k, w in list(enumerate(inputs.batch256()))[::8]:
        axes = None if w.surface == "sphere" else (0, 1)
        got = hjx.shape(w.gmin, w.gmax, w.n, axes=axes, radius=w.radius, periodic=w.periodic, dtype="f64")
        ref = inputs.initial_surface(w)
        np.testing.assert_allclose(to_host(got), ref, rtol=0, atol=1e-13, err_msg=f"member {k}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_construction_equals_one_launch_per_member(dtype):
    """hjx_shape_batch over all 256 members, one launch: every member equals
    hjx_shape on its own grid bit for bit (the same arithmetic), and a sample
    equals the host recipe."""
    ws = inputs.batch256()
    specs = [dict(gmin=w.gmin, gmax=w.gmax, n=w.n, periodic=w.periodic, radius=w.radius,
                  axes=None if w.surface == "sphere" else (0, 1)) for w in ws]
    outs = hjx.shape_batch(specs, dtype=dtype)
    for k in range(0, len(ws), 5):
        one = hjx.shape(dtype=dtype, **specs[k])
        assert torch.equal(outs[k], one), k
    for k in range(0, len(ws), 37):
        ref = inputs.initial_surface(ws[k])
        if dtype == "f64":
            np.testing.assert_allclose(to_host(outs[k]), ref, rtol=0, atol=1e-13)
        else:
            assert_close(to_host(outs[k]), ref, "f32", ws[k].periodic, f"member {k}")
    # mixed kinds and dimensions in one batch, ellipsoids too
    mixed = [dict(gmin=[-1], gmax=[1], n=[50], kind="ellipsoid", weights=[3.0], radius=0.2),
             dict(gmin=[-1, -2], gmax=[1, 2], n=[17, 33], periodic=(1,), center=[0.2, -0.1], radius=0.5),
             dict(gmin=[-1] * 4, gmax=[1] * 4, n=[5, 6, 7, 8], axes=(1, 3), radius=0.3)]
    outs = hjx.shape_batch(mixed, dtype=dtype)
    for o, sp in zip(outs, mixed):
        assert torch.equal(o, hjx.shape(dtype=dtype, **sp))


def test_shape_errors():
    g, _, _ = hjx.descriptors([0, 0], [1, 1], [5, 5])
    d = hjx.ShapeDesc()
    d.kind, d.axis_mask, d.radius = 0, 0b100, 0.5
    out = torch.empty((5, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(hjx.HjxError, match="axis_mask"):
        hjx.hjx_shape(g, d, hjx.HJX_F64, ctypes_ptr(out))
    d.axis_mask, d.kind = 0b11, 5
    with pytest.raises(hjx.HjxError, match="shape kind"):
        hjx.hjx_shape(g, d, hjx.HJX_F64, ctypes_ptr(out))
    with pytest.raises(hjx.HjxError, match="NULL"):
        hjx.hjx_shape_op(0, hjx.HJX_F64, ctypes_ptr(out), None, ctypes_ptr(out), 25)
    with pytest.raises(hjx.HjxError, match="shape op"):
        hjx.hjx_shape_op(9, hjx.HJX_F64, ctypes_ptr(out), ctypes_ptr(out), ctypes_ptr(out), 25)
    with pytest.raises(hjx.HjxError, match="member 1"):
        hjx.shape_batch([dict(gmin=[0, 0], gmax=[1, 1], n=[5, 5]), dict(gmin=[0, 0], gmax=[1, 1], n=[2, 5])])


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())
