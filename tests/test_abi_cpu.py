"""The C-ABI library: builds, loads, exports what include/hjx.h declares, and
rejects bad arguments before touching the device (runs without a GPU)."""
import ctypes
import math
import os
import re

import pytest

from paper_2411_03501_amd import hjx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hjx.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hjx_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("hjx_problem_create", "hjx_problem_destroy", "hjx_dissipation", "hjx_rhs", "hjx_step",
              "hjx_solve", "hjx_last_error", "hjx_version"):
        assert n in names


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(hjx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding knows each of them
    assert set(declared_functions()) <= set(hjx.SIGNATURES)


def test_struct_layouts_match_the_header():
    # field offsets of the descriptors, as laid out by the C compiler for the header
    assert ctypes.sizeof(hjx.GridDesc) == 8 + 3 * 8 * hjx.MAX_DIM
    assert hjx.GridDesc.n.offset == 8 + 2 * 8 * hjx.MAX_DIM
    assert ctypes.sizeof(hjx.HamDesc) == 8 + 64
    assert ctypes.sizeof(hjx.SchemeDesc) == 24
    assert hjx.SchemeDesc.restrict_update.offset == 20
    assert ctypes.sizeof(hjx.Stats) == 8 * (4 + hjx.MAX_DIM + 2)


def test_version_and_empty_error():
    assert re.match(r"\d+\.\d+\.\d+", hjx.hjx_version())


def _create(**kw):
    args = dict(gmin=[0, 0], gmax=[1, 1], n=[5, 5])
    args.update(kw)
    return hjx.hjx_problem_create(*hjx.descriptors(**args))


@pytest.mark.parametrize("kw,msg", [
    (dict(n=[2, 5]), "n\\[0\\]"),
    (dict(gmin=[0, 1], gmax=[1, 1]), "extent"),
    (dict(gmin=[0, float("nan")]), "extent"),
    (dict(periodic=(3,)), "periodic_mask"),
    (dict(ham="dubins3_pe", params=[1, 1, 1, 1]), "dim 3"),
    (dict(gmin=[0] * 3, gmax=[1] * 3, n=[5] * 3, ham="dubins3_pe", params=[1, 1, -1, 1]), "turn-rate"),
    (dict(gmin=[0] * 4, gmax=[1] * 4, n=[5] * 4, ham="dubins4", params=[1, -1]), "control bounds"),
    (dict(ham=7), "Hamiltonian kind"),
    (dict(params=[math.inf]), "not finite"),
    (dict(scheme=4), "derivative scheme"),
    (dict(rk=4), "rk order"),
    (dict(cfl=0.0), "cfl"),
    (dict(cfl=1.5), "cfl"),
    (dict(restrict=3), "restrict_update"),
    (dict(dissipation=3), "unknown dissipation"),
    (dict(gmin=[0] * 3, gmax=[1] * 3, n=[5] * 3, ham="dubins3_pe", params=[1, 1, 1, 1], dissipation=2), "Godunov"),
    (dict(ham="rockets", params=[1, 32, 1, 1]), "ROCKETS needs dim 3"),
    (dict(gmin=[0] * 3, gmax=[1] * 3, n=[5] * 3, ham="rockets", params=[1, 32, -1, 1]), "control bounds"),
    (dict(restrict=-1), "restrict_update"),
    (dict(gmin=[0] * 4, gmax=[1] * 4, n=[300, 300, 300, 300]), "2\\^31"),
])
def test_invalid_descriptors_are_rejected(kw, msg):
    with pytest.raises(hjx.HjxError) as e:
        _create(**kw)
    assert e.value.status == hjx.HJX_ERR_INVALID_ARG
    assert re.search(msg, str(e.value)), str(e.value)
    assert re.search(msg, hjx.hjx_last_error())


def test_bad_dim_and_dtype():
    g, h, s = hjx.descriptors([0], [1], [5])
    g.dim = 5
    with pytest.raises(hjx.HjxError, match="dim 5"):
        hjx.hjx_problem_create(g, h, s)
    g.dim = 1
    s.dtype = 9
    with pytest.raises(hjx.HjxError, match="dtype"):
        hjx.hjx_problem_create(g, h, s)


def test_null_arguments():
    L = hjx.lib()
    out = ctypes.c_void_p()
    assert L.hjx_problem_create(None, None, None, ctypes.byref(out)) == hjx.HJX_ERR_INVALID_ARG
    g, h, s = hjx.descriptors([0], [1], [5])
    assert L.hjx_problem_create(ctypes.byref(g), ctypes.byref(h), ctypes.byref(s), None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_solve(None, None, None, None, 0.0, 1.0, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_step(None, None, None, 0.1, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_rhs(None, None, None, None) == hjx.HJX_ERR_INVALID_ARG
    a = (ctypes.c_double * 4)()
    d = ctypes.c_double()
    assert L.hjx_dissipation(None, a, ctypes.byref(d), None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_problem_destroy(None) == hjx.HJX_OK


def test_batch_rejects_bad_arguments_before_the_device():
    L = hjx.lib()
    out = ctypes.c_void_p()
    assert L.hjx_batch_create(0, None, None, ctypes.byref(out)) == hjx.HJX_ERR_INVALID_ARG
    assert "n >= 1" in hjx.hjx_last_error()
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.hjx_batch_create(2, arr, None, ctypes.byref(out)) == hjx.HJX_ERR_INVALID_ARG
    assert "problems[0]" in hjx.hjx_last_error()
    assert L.hjx_batch_create(1, arr, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_batch_set_shape(None, 256, 1) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_batch_get_shape(None, None, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_batch_solve(None, None, None, None, None, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_batch_tune(None, None, None, None, None, 1, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_batch_destroy(None) == hjx.HJX_OK


@pytest.mark.parametrize("kw,msg", [
    (dict(flux=5), "unknown flux"),
    (dict(c=[1.0, math.nan]), "not finite"),
    (dict(cfl=0.0), "cfl"),
    (dict(dtype=7), "dtype"),
    (dict(n=[2, 5]), "n\\[0\\]"),
])
def test_claw_rejects_bad_arguments_before_the_device(kw, msg):
    args = dict(n=[5, 5], flux=hjx.FLUX["burgers"], c=[1.0, 1.0], dtype=hjx.HJX_F64, cfl=0.9)
    args.update(kw)
    g, _, _ = hjx.descriptors([0, 0], [1, 1], args["n"])
    with pytest.raises(hjx.HjxError) as e:
        hjx.hjx_claw_create(g, args["flux"], args["c"], args["dtype"], args["cfl"])
    assert e.value.status == hjx.HJX_ERR_INVALID_ARG
    assert re.search(msg, str(e.value)), str(e.value)


def test_claw_null_arguments():
    L = hjx.lib()
    out = ctypes.c_void_p()
    assert L.hjx_claw_create(None, 0, None, 1, 0.9, ctypes.byref(out)) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_claw_step(None, None, None, 0.1, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_claw_solve(None, None, None, 1.0, None, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_claw_dt(None, None, None, None) == hjx.HJX_ERR_INVALID_ARG
    assert L.hjx_claw_destroy(None) == hjx.HJX_OK


def test_shape_rejects_bad_arguments_before_the_device():
    g, _, _ = hjx.descriptors([0, 0], [1, 1], [5, 5])
    d = hjx.ShapeDesc()
    d.kind, d.axis_mask, d.radius = 0, 0, 0.5
    with pytest.raises(hjx.HjxError, match="axis_mask"):
        hjx.hjx_shape(g, d, hjx.HJX_F64, ctypes.c_void_p(8), stream=0)
    d.axis_mask, d.radius = 0b11, math.inf
    with pytest.raises(hjx.HjxError, match="radius"):
        hjx.hjx_shape(g, d, hjx.HJX_F64, ctypes.c_void_p(8), stream=0)
    with pytest.raises(hjx.HjxError, match="n = -1"):
        hjx.hjx_shape_op(0, hjx.HJX_F64, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), -1, stream=0)
