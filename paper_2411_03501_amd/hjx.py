"""ctypes binding of libhjx (include/hjx.h): argument marshalling only.

Every step of the solver runs in the HIP library.  The functions below carry
the C entry points' names and arguments; `Problem` wraps a handle for
convenience.  Arrays are torch tensors on the GPU, contiguous, of the
problem's dtype; the stream defaults to torch's current stream.  If the
library is not built this module raises: there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhjx.so")

HJX_OK, HJX_ERR_INVALID_ARG, HJX_ERR_UNSUPPORTED, HJX_ERR_DEVICE, HJX_ERR_NONFINITE, HJX_ERR_OOM = range(6)
HJX_F32, HJX_F64 = 0, 1
DERIV = {"first": 1, "eno2": 2, "eno3": 3, "weno5": 5}
HAM = {"normal": 0, "dubins3_pe": 1, "dubins4": 2, "rockets": 3}
RESTRICT = {"none": 0, "nonpositive": 1, "positive": 2}
FLUX = {"linear": 0, "burgers": 1}
DISSIPATION = {"global": 0, "local": 1, "godunov": 2}
SHAPES = {"ball": 0, "ellipsoid": 1}
SHAPE_OPS = {"union": 0, "intersection": 1, "complement": 2, "subtraction": 3}
MAX_DIM = 4


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("periodic_mask", ctypes.c_uint32),
                ("gmin", ctypes.c_double * MAX_DIM), ("gmax", ctypes.c_double * MAX_DIM),
                ("n", ctypes.c_int64 * MAX_DIM)]


class HamDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dissipation", ctypes.c_int32), ("p", ctypes.c_double * 8)]


class SchemeDesc(ctypes.Structure):
    _fields_ = [("deriv", ctypes.c_int32), ("rk", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("restrict_update", ctypes.c_int32)]


class ShapeDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("axis_mask", ctypes.c_uint32), ("center", ctypes.c_double * 4),
                ("weights", ctypes.c_double * 4), ("radius", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("dt", ctypes.c_double), ("dt_last", ctypes.c_double),
                ("t_final", ctypes.c_double), ("alpha", ctypes.c_double * MAX_DIM),
                ("elapsed_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]

    def as_dict(self):
        return {k: (list(getattr(self, k)) if k == "alpha" else getattr(self, k)) for k, _ in self._fields_}


class HjxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hjx status {status}: {msg}")
        self.status = status


_lib = None

# exported symbols and their signatures (kept in step with include/hjx.h)
_P = ctypes.c_void_p
SIGNATURES = {
    "hjx_version": ([], ctypes.c_char_p),
    "hjx_last_error": ([], ctypes.c_char_p),
    "hjx_problem_create": ([ctypes.POINTER(GridDesc), ctypes.POINTER(HamDesc), ctypes.POINTER(SchemeDesc),
                            ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hjx_problem_destroy": ([_P], ctypes.c_int),
    "hjx_dissipation": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "hjx_rhs": ([_P, _P, _P, _P], ctypes.c_int),
    "hjx_step": ([_P, _P, _P, ctypes.c_double, _P], ctypes.c_int),
    "hjx_problem_set_tile": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "hjx_problem_get_tile": ([_P] + [ctypes.POINTER(ctypes.c_int32)] * 4, ctypes.c_int),
    "hjx_tune": ([_P, _P, ctypes.c_int32, ctypes.c_char_p, _P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hjx_problem_set_params": ([_P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hjx_solve": ([_P, _P, _P, _P, ctypes.c_double, ctypes.c_double, _P, ctypes.POINTER(Stats)], ctypes.c_int),
    "hjx_tape_create": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_void_p)],
                        ctypes.c_int),
    "hjx_tape_destroy": ([_P], ctypes.c_int),
    "hjx_tape_set_mode": ([_P, ctypes.c_int32], ctypes.c_int),
    "hjx_tape_get_mode": ([_P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "hjx_solve_taped": ([_P, _P, _P, _P, _P, _P, ctypes.POINTER(Stats)], ctypes.c_int),
    "hjx_adjoint": ([_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "hjx_loss_volume": ([_P, _P, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _P, _P], ctypes.c_int),
    "hjx_batch_create": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), _P, ctypes.POINTER(ctypes.c_void_p)],
                         ctypes.c_int),
    "hjx_batch_destroy": ([_P], ctypes.c_int),
    "hjx_batch_set_shape": ([_P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "hjx_batch_get_shape": ([_P] + [ctypes.POINTER(ctypes.c_int32)] * 3, ctypes.c_int),
    "hjx_batch_solve": ([_P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double), _P,
                         ctypes.POINTER(Stats)], ctypes.c_int),
    "hjx_batch_tune": ([_P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _P,
                        ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "hjx_shape": ([ctypes.POINTER(GridDesc), ctypes.POINTER(ShapeDesc), ctypes.c_int32, _P, _P], ctypes.c_int),
    "hjx_shape_op": ([ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_int64, _P], ctypes.c_int),
    "hjx_shape_batch": ([ctypes.c_int32, ctypes.POINTER(GridDesc), ctypes.POINTER(ShapeDesc), ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_void_p), _P], ctypes.c_int),
    "hjx_shape_batch_noalloc": ([ctypes.c_int32, ctypes.POINTER(GridDesc), ctypes.POINTER(ShapeDesc), ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_void_p), _P], ctypes.c_int),
    "hjx_claw_create": ([ctypes.POINTER(GridDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                         ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "hjx_claw_destroy": ([_P], ctypes.c_int),
    "hjx_claw_dt": ([_P, _P, ctypes.POINTER(ctypes.c_double), _P], ctypes.c_int),
    "hjx_claw_step": ([_P, _P, _P, ctypes.c_double, _P], ctypes.c_int),
    "hjx_claw_solve": ([_P, _P, _P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
}


def lib():
    """Load libhjx.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status):
    if status != HJX_OK:
        raise HjxError(status, lib().hjx_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, numel, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name}: need a contiguous {dtype} tensor of {numel} elements, "
                         f"got {t.dtype} {tuple(t.shape)} contiguous={t.is_contiguous()}")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C names

def hjx_version():
    return lib().hjx_version().decode()


def hjx_last_error():
    return lib().hjx_last_error().decode()


def hjx_problem_create(grid, ham, scheme):
    h = ctypes.c_void_p()
    _check(lib().hjx_problem_create(ctypes.byref(grid), ctypes.byref(ham), ctypes.byref(scheme),
                                    ctypes.byref(h)))
    return h


def hjx_problem_destroy(handle):
    _check(lib().hjx_problem_destroy(handle))


TILE_PLANE_MARCH, TILE_DIRECT, TILE_STEPS = 0, 1, 2


def hjx_problem_set_tile(handle, variant, tx, ty, march):
    _check(lib().hjx_problem_set_tile(handle, int(variant), int(tx), int(ty), int(march)))


def hjx_problem_get_tile(handle):
    """(variant, tx, ty, march)"""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().hjx_problem_get_tile(handle, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def hjx_tune(handle, phi_ptr, reps=5, stream=None, cache_path=None):
    us = ctypes.c_double()
    cp = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().hjx_tune(handle, phi_ptr, int(reps), cp, _stream(stream), ctypes.byref(us)))
    return us.value


def hjx_problem_set_params(handle, params):
    v = (ctypes.c_double * 8)(*[float(x) for x in params][:8])
    _check(lib().hjx_problem_set_params(handle, v))


def hjx_dissipation(handle, dim, stream=None):
    a = (ctypes.c_double * MAX_DIM)()
    dt = ctypes.c_double()
    _check(lib().hjx_dissipation(handle, a, ctypes.byref(dt), _stream(stream)))
    return [a[d] for d in range(dim)], dt.value


def hjx_rhs(handle, phi_ptr, L_ptr, stream=None):
    _check(lib().hjx_rhs(handle, phi_ptr, L_ptr, _stream(stream)))


def hjx_step(handle, phi_ptr, target_ptr, dt, stream=None):
    _check(lib().hjx_step(handle, phi_ptr, target_ptr, float(dt), _stream(stream)))


def hjx_solve(handle, phi0_ptr, target_ptr, out_ptr, t0, t1, stream=None, stats=True):
    st = Stats() if stats else None
    _check(lib().hjx_solve(handle, phi0_ptr, target_ptr, out_ptr, float(t0), float(t1), _stream(stream),
                           ctypes.byref(st) if st is not None else None))
    return st


def hjx_tape_create(handle, t0, t1, ckpt_every, stream=None):
    t = ctypes.c_void_p()
    _check(lib().hjx_tape_create(handle, float(t0), float(t1), int(ckpt_every), _stream(stream), ctypes.byref(t)))
    return t


def hjx_tape_destroy(tape):
    _check(lib().hjx_tape_destroy(tape))


TAPE_RECOMPUTE, TAPE_STORE_DERIVS = 0, 1


def hjx_tape_set_mode(tape, mode):
    _check(lib().hjx_tape_set_mode(tape, int(mode)))


def hjx_tape_get_mode(tape):
    m = ctypes.c_int32()
    _check(lib().hjx_tape_get_mode(tape, ctypes.byref(m)))
    return m.value


def hjx_solve_taped(handle, tape, phi0_ptr, target_ptr, out_ptr, stream=None):
    st = Stats()
    _check(lib().hjx_solve_taped(handle, tape, phi0_ptr, target_ptr, out_ptr, _stream(stream), ctypes.byref(st)))
    return st


def hjx_adjoint(handle, tape, g_ptr, dphi0_ptr, dtarget_ptr, stream=None):
    dp = (ctypes.c_double * 8)()
    _check(lib().hjx_adjoint(handle, tape, g_ptr, dphi0_ptr, dtarget_ptr, dp, _stream(stream)))
    return [dp[k] for k in range(8)]


def hjx_loss_volume(handle, phi_ptr, eps, grad_ptr, stream=None):
    v = ctypes.c_double()
    _check(lib().hjx_loss_volume(handle, phi_ptr, float(eps), ctypes.byref(v), grad_ptr, _stream(stream)))
    return v.value


def _ptrs(ptrs):
    """A host array of device pointers (entries may be None)."""
    if ptrs is None:
        return None
    arr = (ctypes.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = None if p is None else (p.value if isinstance(p, ctypes.c_void_p) else int(p))
    return arr


def hjx_batch_create(handles, stream=None):
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    b = ctypes.c_void_p()
    _check(lib().hjx_batch_create(len(handles), arr, _stream(stream), ctypes.byref(b)))
    return b


def hjx_batch_destroy(batch):
    _check(lib().hjx_batch_destroy(batch))


def hjx_batch_set_shape(batch, item_nodes, blocks):
    _check(lib().hjx_batch_set_shape(batch, int(item_nodes), int(blocks)))


def hjx_batch_get_shape(batch):
    v = [ctypes.c_int32() for _ in range(3)]
    _check(lib().hjx_batch_get_shape(batch, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def hjx_batch_solve(batch, phi0_ptrs, target_ptrs, out_ptrs, t1, stream=None, stats=True):
    n = len(phi0_ptrs)
    st = (Stats * n)() if stats else None
    _check(lib().hjx_batch_solve(batch, _ptrs(phi0_ptrs), _ptrs(target_ptrs), _ptrs(out_ptrs),
                                 (ctypes.c_double * n)(*[float(v) for v in t1]), _stream(stream), st))
    return st


def hjx_batch_tune(batch, phi0_ptrs, target_ptrs, out_ptrs, t1, reps=2, stream=None):
    n = len(phi0_ptrs)
    ms = ctypes.c_double()
    _check(lib().hjx_batch_tune(batch, _ptrs(phi0_ptrs), _ptrs(target_ptrs), _ptrs(out_ptrs),
                                (ctypes.c_double * n)(*[float(v) for v in t1]), int(reps), _stream(stream),
                                ctypes.byref(ms)))
    return ms.value


# ------------------------------------------------------------------ handle wrapper

def descriptors(gmin, gmax, n, periodic=(), ham="normal", params=(1.0,), scheme="weno5", rk=3, cfl=0.75,
                dtype="f64", restrict="none", dissipation="global"):
    g = GridDesc()
    g.dim = len(n)
    g.periodic_mask = sum(1 << d for d in periodic)
    for d in range(len(n)):
        g.gmin[d], g.gmax[d], g.n[d] = float(gmin[d]), float(gmax[d]), int(n[d])
    h = HamDesc()
    h.kind = HAM[ham] if isinstance(ham, str) else int(ham)
    h.dissipation = DISSIPATION[dissipation] if isinstance(dissipation, str) else int(dissipation)
    for k, v in enumerate(params):
        h.p[k] = float(v)
    s = SchemeDesc()
    s.deriv = DERIV[scheme] if isinstance(scheme, str) else int(scheme)
    s.rk = int(rk)
    s.cfl = float(cfl)
    s.dtype = HJX_F32 if dtype in ("f32", torch.float32) else HJX_F64
    s.restrict_update = RESTRICT[restrict] if isinstance(restrict, str) else int(restrict)
    return g, h, s


class Problem:
    """A problem handle: grid, Hamiltonian and scheme (see include/hjx.h)."""

    def __init__(self, gmin, gmax, n, periodic=(), ham="normal", params=(1.0,), scheme="weno5", rk=3,
                 cfl=0.75, dtype="f64", restrict="none", dissipation="global"):
        self.shape = tuple(int(v) for v in n)
        self.dim = len(self.shape)
        self.numel = 1
        for v in self.shape:
            self.numel *= v
        self.dtype = torch.float32 if dtype in ("f32", torch.float32) else torch.float64
        self.handle = None
        self.handle = hjx_problem_create(*descriptors(gmin, gmax, n, periodic, ham, params, scheme, rk, cfl,
                                                      dtype, restrict, dissipation))
        self._params = tuple(float(v) for v in params)

    @classmethod
    def from_workload(cls, w, dtype=None):
        return cls(w.gmin, w.gmax, w.n, w.periodic, w.ham, w.params, w.scheme, w.rk, w.cfl, dtype or w.dtype,
                   w.restrict, w.dissipation)

    def close(self):
        if self.handle is not None:
            hjx_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, t, name):
        return _dev(t, self.dtype, self.numel, name)

    @property
    def tile(self):
        """(variant, tx, ty, march); variant 0 = plane-march, 1 = direct, 2 = steps
        (march whole RK steps per launch)."""
        return hjx_problem_get_tile(self.handle)

    @tile.setter
    def tile(self, shape):
        """(variant, tx, ty, march), or (tx, ty, march) for the plane-march variant."""
        if len(shape) == 3:
            shape = (TILE_PLANE_MARCH,) + tuple(shape)
        hjx_problem_set_tile(self.handle, *shape)

    def tune(self, phi, reps=5, stream=None, cache=None):
        """Pick the fastest stage-kernel launch shape for this problem; returns
        (tile, mean launch time in us).  cache: a tuning-cache file (None: the
        HJX_TUNE_CACHE environment variable, "": none)."""
        us = hjx_tune(self.handle, self._t(phi, "phi"), reps, stream, cache)
        return self.tile, us

    @property
    def params(self):
        """The Hamiltonian's parameters (a tuple of the kind's count)."""
        return self._params

    @params.setter
    def params(self, values):
        hjx_problem_set_params(self.handle, values)
        self._params = tuple(float(v) for v in values)

    def dissipation(self, stream=None):
        return hjx_dissipation(self.handle, self.dim, stream)

    def rhs(self, phi, out=None, stream=None):
        if out is None:
            out = torch.empty_like(phi)
        hjx_rhs(self.handle, self._t(phi, "phi"), self._t(out, "L_out"), stream)
        return out

    def step(self, phi, dt, target=None, stream=None):
        """One RK step in place on phi."""
        hjx_step(self.handle, self._t(phi, "phi"), self._t(target, "target"), dt, stream)
        return phi

    def tape(self, t1, t0=0.0, ckpt_every=8, stream=None):
        return Tape(self, t0, t1, ckpt_every, stream)

    def loss_volume(self, phi, eps, grad=True, stream=None):
        """Smoothed volume of {phi <= 0} and (optionally) its gradient."""
        g = torch.empty_like(phi) if grad else None
        v = hjx_loss_volume(self.handle, self._t(phi, "phi"), eps, self._t(g, "grad"), stream)
        return (v, g) if grad else v

    def solve(self, phi0, t1, t0=0.0, target=None, out=None, stream=None):
        """Returns (phi(t1), stats dict)."""
        if out is None:
            out = torch.empty_like(phi0)
        st = hjx_solve(self.handle, self._t(phi0, "phi0"), self._t(target, "target"), self._t(out, "phi_out"),
                       t0, t1, stream)
        return out, st.as_dict()


class Tape:
    """Checkpoints of one solve, for hjx_adjoint."""

    def __init__(self, problem, t0, t1, ckpt_every=8, stream=None):
        self.problem = problem
        self.handle = None
        self.handle = hjx_tape_create(problem.handle, t0, t1, ckpt_every, stream)
        self.has_target = False

    def close(self):
        if self.handle is not None:
            hjx_tape_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def mode(self):
        """TAPE_STORE_DERIVS (the replay keeps p-, p+) or TAPE_RECOMPUTE."""
        return hjx_tape_get_mode(self.handle)

    @mode.setter
    def mode(self, m):
        hjx_tape_set_mode(self.handle, m)

    def solve(self, phi0, target=None, out=None, stream=None):
        P = self.problem
        if out is None:
            out = torch.empty_like(phi0)
        st = hjx_solve_taped(P.handle, self.handle, P._t(phi0, "phi0"), P._t(target, "target"),
                             P._t(out, "phi_out"), stream)
        self.has_target = target is not None
        return out, st.as_dict()

    def adjoint(self, dL_dphiT, stream=None, sum_target=False):
        """Returns (dL/dphi0, dL/dtarget or None, dL/dparams list of 8).  With
        sum_target (the solve's target was phi0 itself) the library writes
        dL/dphi0 + dL/dtarget into the first array and the second is None."""
        P = self.problem
        g0 = torch.empty_like(dL_dphiT)
        if sum_target and not self.has_target:
            raise ValueError("sum_target: the solve had no target")
        gt = g0 if sum_target else (torch.empty_like(dL_dphiT) if self.has_target else None)
        dp = hjx_adjoint(P.handle, self.handle, P._t(dL_dphiT, "dL_dphiT"), P._t(g0, "dL_dphi0"),
                         P._t(gt, "dL_dtarget"), stream)
        return g0, (None if sum_target else gt), dp


class Batch:
    """Many problems solved together (hjx_batch_*).  The batch borrows each
    member's workspace; keep the members alive while it exists."""

    def __init__(self, problems, stream=None):
        self.problems = list(problems)
        self.handle = None
        self.handle = hjx_batch_create([p.handle for p in self.problems], stream)

    def close(self):
        if self.handle is not None:
            hjx_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        """(item_nodes, blocks, blocks_max)."""
        return hjx_batch_get_shape(self.handle)

    @shape.setter
    def shape(self, v):
        hjx_batch_set_shape(self.handle, *v[:2])

    def _args(self, phi0, target, out):
        n = len(self.problems)
        if len(phi0) != n or (target is not None and len(target) != n) or (out is not None and len(out) != n):
            raise ValueError(f"need {n} arrays per argument")
        if out is None:
            out = [torch.empty_like(x) for x in phi0]
        p0 = [P._t(x, f"phi0[{i}]") for i, (P, x) in enumerate(zip(self.problems, phi0))]
        tg = None if target is None else [P._t(x, f"target[{i}]") for i, (P, x) in
                                          enumerate(zip(self.problems, target))]
        po = [P._t(x, f"phi_out[{i}]") for i, (P, x) in enumerate(zip(self.problems, out))]
        return p0, tg, po, out

    def solve(self, phi0, t1, target=None, out=None, stream=None):
        """Returns (list of phi(t1[i]), list of stats dicts)."""
        p0, tg, po, out = self._args(phi0, target, out)
        st = hjx_batch_solve(self.handle, p0, tg, po, t1, stream)
        return out, [s.as_dict() for s in st]

    def tune(self, phi0, t1, target=None, out=None, reps=2, stream=None):
        """Pick the fastest launch shape; returns (shape, mean replay ms)."""
        p0, tg, po, out = self._args(phi0, target, out)
        ms = hjx_batch_tune(self.handle, p0, tg, po, t1, reps, stream)
        return self.shape, ms


# ------------------------------------------------------------------ shapes

def hjx_shape(grid, desc, dtype, out_ptr, stream=None):
    _check(lib().hjx_shape(ctypes.byref(grid), ctypes.byref(desc), int(dtype), out_ptr, _stream(stream)))


def hjx_shape_op(op, dtype, a_ptr, b_ptr, out_ptr, n, stream=None):
    _check(lib().hjx_shape_op(int(op), int(dtype), a_ptr, b_ptr, out_ptr, int(n), _stream(stream)))


def shape(gmin, gmax, n, kind="ball", axes=None, center=None, radius=1.0, weights=None, periodic=(), dtype="f64",
          out=None, stream=None):
    """An implicit surface on the grid (hjx_shape): kind "ball" (sphere over
    every axis in `axes`, cylinder over some) or "ellipsoid" (Listing 2)."""
    g, _, _ = descriptors(gmin, gmax, n, periodic)
    d = _shape_desc(len(n), kind, axes, center, radius, weights)
    tdt = torch.float32 if dtype in ("f32", torch.float32) else torch.float64
    if out is None:
        out = torch.empty(tuple(int(v) for v in n), dtype=tdt, device="cuda")
    numel = 1
    for v in n:
        numel *= int(v)
    hjx_shape(g, d, HJX_F32 if tdt == torch.float32 else HJX_F64, _dev(out, tdt, numel, "phi_out"), stream)
    return out


def _shape_desc(ndim, kind, axes, center, radius, weights):
    d = ShapeDesc()
    d.kind = SHAPES[kind] if isinstance(kind, str) else int(kind)
    d.axis_mask = sum(1 << a for a in (range(ndim) if axes is None else axes))
    for k in range(ndim):
        d.center[k] = float(center[k]) if center is not None else 0.0
        d.weights[k] = float(weights[k]) if weights is not None else 1.0
    d.radius = float(radius)
    return d


SHAPE_NOALLOC_MAX = 1024


def shape_batch(specs, dtype="f64", outs=None, stream=None, noalloc=False):
    """Shapes of many grids in one launch (hjx_shape_batch).  specs: dicts
    with gmin, gmax, n and optional periodic, kind, axes, center, radius,
    weights (as for shape()).  Returns the list of output tensors.
    noalloc: through hjx_shape_batch_noalloc (at most SHAPE_NOALLOC_MAX
    members; the library allocates nothing)."""
    tdt = torch.float32 if dtype in ("f32", torch.float32) else torch.float64
    k = len(specs)
    grids = (GridDesc * k)()
    descs = (ShapeDesc * k)()
    if outs is None:
        outs = [torch.empty(tuple(int(v) for v in sp["n"]), dtype=tdt, device="cuda") for sp in specs]
    ptrs = (ctypes.c_void_p * k)()
    for i, sp in enumerate(specs):
        g, _, _ = descriptors(sp["gmin"], sp["gmax"], sp["n"], sp.get("periodic", ()))
        grids[i] = g
        descs[i] = _shape_desc(len(sp["n"]), sp.get("kind", "ball"), sp.get("axes"), sp.get("center"),
                               sp.get("radius", 1.0), sp.get("weights"))
        numel = 1
        for v in sp["n"]:
            numel *= int(v)
        ptrs[i] = _dev(outs[i], tdt, numel, f"outs[{i}]")
    fn = lib().hjx_shape_batch_noalloc if noalloc else lib().hjx_shape_batch
    _check(fn(k, grids, descs, HJX_F32 if tdt == torch.float32 else HJX_F64, ptrs, _stream(stream)))
    return outs


def shape_op(op, a, b=None, out=None, stream=None):
    """Union min(a, b), intersection max(a, b), complement -a or subtraction
    max(a, -b), elementwise on the device (hjx_shape_op)."""
    if out is None:
        out = torch.empty_like(a)
    dt = HJX_F32 if a.dtype == torch.float32 else HJX_F64
    hjx_shape_op(SHAPE_OPS[op] if isinstance(op, str) else int(op), dt, _dev(a, a.dtype, a.numel(), "a"),
                 _dev(b, a.dtype, a.numel(), "b"), _dev(out, a.dtype, a.numel(), "out"), a.numel(), stream)
    return out


# ------------------------------------------------------------------ conservation laws

def hjx_claw_create(grid, flux, c, dtype, cfl):
    h = ctypes.c_void_p()
    arr = (ctypes.c_double * MAX_DIM)(*[float(x) for x in c][:MAX_DIM])
    _check(lib().hjx_claw_create(ctypes.byref(grid), int(flux), arr, int(dtype), float(cfl), ctypes.byref(h)))
    return h


def hjx_claw_destroy(handle):
    _check(lib().hjx_claw_destroy(handle))


def hjx_claw_dt(handle, v_ptr, stream=None):
    dt = ctypes.c_double()
    _check(lib().hjx_claw_dt(handle, v_ptr, ctypes.byref(dt), _stream(stream)))
    return dt.value


def hjx_claw_step(handle, v_ptr, out_ptr, dt, stream=None):
    _check(lib().hjx_claw_step(handle, v_ptr, out_ptr, float(dt), _stream(stream)))


def hjx_claw_solve(handle, v0_ptr, out_ptr, t1, stream=None):
    steps, dt = ctypes.c_int64(), ctypes.c_double()
    _check(lib().hjx_claw_solve(handle, v0_ptr, out_ptr, float(t1), _stream(stream), ctypes.byref(steps),
                                ctypes.byref(dt)))
    return steps.value, dt.value


class Claw:
    """A scalar conservation law v_t + sum_d f_d(v)_{x_d} = 0 solved by the
    Lax-Friedrichs scheme (hjx_claw_*, see include/hjx.h)."""

    def __init__(self, gmin, gmax, n, periodic=(), flux="burgers", c=(1.0,), cfl=0.9, dtype="f64"):
        self.shape = tuple(int(v) for v in n)
        self.dim = len(self.shape)
        self.numel = 1
        for v in self.shape:
            self.numel *= v
        self.dtype = torch.float32 if dtype in ("f32", torch.float32) else torch.float64
        cc = [float(c[d] if d < len(c) else c[-1]) for d in range(self.dim)]
        g, _, _ = descriptors(gmin, gmax, n, periodic)
        self.handle = None
        self.handle = hjx_claw_create(g, FLUX[flux] if isinstance(flux, str) else int(flux), cc,
                                      HJX_F32 if self.dtype == torch.float32 else HJX_F64, cfl)

    def close(self):
        if self.handle is not None:
            hjx_claw_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, t, name):
        return _dev(t, self.dtype, self.numel, name)

    def dt(self, v, stream=None):
        return hjx_claw_dt(self.handle, self._t(v, "v"), stream)

    def step(self, v, dt, out=None, stream=None):
        if out is None:
            out = torch.empty_like(v)
        hjx_claw_step(self.handle, self._t(v, "v"), self._t(out, "v_out"), dt, stream)
        return out

    def solve(self, v0, t1, out=None, stream=None):
        """Returns (v(t1), {"steps", "dt"})."""
        if out is None:
            out = torch.empty_like(v0)
        steps, dt = hjx_claw_solve(self.handle, self._t(v0, "v0"), self._t(out, "v_out"), t1, stream)
        return out, {"steps": steps, "dt": dt}


class HjxSolve(torch.autograd.Function):
    """phi(t1) = solve(phi0; params) from 0 to t1, with min-with-target
    against phi0 itself (the reachable-tube setting) or no target, as a
    differentiable function of phi0 and of the Hamiltonian's parameters.

    Usage: HjxSolve.apply(phi0, params, problem, t1, with_target=True, ckpt_every=8)
      phi0    tensor of the problem's shape and dtype on the device;
      params  1-D tensor of the kind's parameter count (any device and
              float dtype): the problem's parameters are set to it for the
              solve (hjx_problem_set_params);
      problem a Problem; returns phi(t1).
    backward runs hjx_adjoint on the tape of the forward solve (checkpoints
    every ckpt_every steps) and returns dL/dphi0 (through both the initial
    value and the target when phi0 is the target; the library adds the two)
    and dL/dparams (float64 from the library, cast to params' dtype and
    device).  The tape lives as long as the graph node, so backward may run
    again with retain_graph; phi0 is saved for backward, so changing it in
    place before backward raises."""

    @staticmethod
    def forward(ctx, phi0, params, problem, t1, with_target=True, ckpt_every=8):
        values = [float(v) for v in params.detach().to("cpu", torch.float64).reshape(-1)]
        problem.params = values
        tape = problem.tape(t1, 0.0, ckpt_every)
        x = phi0.detach()
        if not x.is_contiguous():
            x = x.contiguous()
        out, _ = tape.solve(x, target=x if with_target else None)
        ctx.save_for_backward(x)     # the target the reverse sweep replays
        ctx.tape = tape
        ctx.values = values
        ctx.params_like = (params.dtype, params.device, params.shape)
        ctx.with_target = with_target
        return out

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors      # raises if phi0 changed in place since forward
        tape = ctx.tape
        tape.problem.params = ctx.values  # the parameters the tape was made with
        g0, _, dp = tape.adjoint(g.contiguous(), sum_target=ctx.with_target)
        dtype, device, shape = ctx.params_like
        n = 1
        for v in shape:
            n *= v
        gp = torch.tensor(dp[:n], dtype=torch.float64).to(device=device, dtype=dtype).reshape(shape)
        return g0, gp, None, None, None, None
