"""FP64 CPU oracle for explicit Hamilton-Jacobi level-set time stepping.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports it.

A thin ctypes wrapper over oracle/libhjxo.so (plain C99, built by
oracle/build.py).  Arrays are numpy float64, C-contiguous, row-major with the
last axis fastest.  The C source states, function by function, which passage
of the paper (LevelSetPy, arXiv 2411.03501) it follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhjxo.so")

MAXD = 4
SCHEME = {"first": 1, "eno2": 2, "eno3": 3, "weno5": 5}
HAM = {"normal": 0, "dubins3_pe": 1, "dubins4": 2, "rockets": 3}
# restricted update (see restricted_rate in hjxo.c)
RESTRICT = {"none": 0, "nonpositive": 1, "positive": 2}
# numerical Hamiltonian: Lax-Friedrichs with alpha_d as the grid maximum
# (global) or at the node (local), or Godunov's (normal motion only)
DISSIPATION = {"global": 0, "local": 1, "godunov": 2}


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("gmin", ctypes.c_double * MAXD),
        ("gmax", ctypes.c_double * MAXD),
        ("n", ctypes.c_long * MAXD),
        ("periodic_mask", ctypes.c_uint),
        ("ham_kind", ctypes.c_int),
        ("hp", ctypes.c_double * 8),
        ("scheme", ctypes.c_int),
        ("rk", ctypes.c_int),
        ("cfl", ctypes.c_double),
        ("restrict_update", ctypes.c_int),
        ("dissipation", ctypes.c_int),
        ("decide_f32", ctypes.c_int),
    ]


def make_problem(gmin, gmax, n, periodic=(), ham="normal", params=(1.0,), scheme="weno5", rk=3,
                 cfl=0.75, restrict="none", dissipation="global", decide="f64"):
    """Build an oracle problem.  `periodic` lists periodic axes.  `decide`
    is the precision of the ENO stencil choices ("f64", or "f32" for the
    binary32 choices of eno_choice in hjxo.c); the arithmetic is FP64."""
    P = Problem()
    P.dim = len(n)
    for d in range(len(n)):
        P.gmin[d] = float(gmin[d])
        P.gmax[d] = float(gmax[d])
        P.n[d] = int(n[d])
    P.periodic_mask = sum(1 << d for d in periodic)
    P.ham_kind = HAM[ham] if isinstance(ham, str) else int(ham)
    for k, v in enumerate(params):
        P.hp[k] = float(v)
    P.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    P.rk = int(rk)
    P.cfl = float(cfl)
    P.restrict_update = RESTRICT[restrict] if isinstance(restrict, str) else int(restrict)
    P.dissipation = DISSIPATION[dissipation] if isinstance(dissipation, str) else int(dissipation)
    P.decide_f32 = {"f64": 0, "f32": 1}[decide]
    return P


class Claw(ctypes.Structure):
    """A scalar conservation law v_t + sum_d f_d(v)_{x_d} = 0 on a grid."""
    _fields_ = [
        ("dim", ctypes.c_int),
        ("gmin", ctypes.c_double * MAXD),
        ("gmax", ctypes.c_double * MAXD),
        ("n", ctypes.c_long * MAXD),
        ("periodic_mask", ctypes.c_uint),
        ("flux", ctypes.c_int),
        ("c", ctypes.c_double * MAXD),
        ("cfl", ctypes.c_double),
    ]


FLUX = {"linear": 0, "burgers": 1}


def make_claw(gmin, gmax, n, periodic=(), flux="burgers", c=(1.0,), cfl=0.9):
    C = Claw()
    C.dim = len(n)
    for d in range(len(n)):
        C.gmin[d], C.gmax[d], C.n[d] = float(gmin[d]), float(gmax[d]), int(n[d])
        C.c[d] = float(c[d] if d < len(c) else c[-1])
    C.periodic_mask = sum(1 << d for d in periodic)
    C.flux = FLUX[flux] if isinstance(flux, str) else int(flux)
    C.cfl = float(cfl)
    return C


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        PP = ctypes.POINTER(Problem)
        L.hjxo_set_threads.argtypes = [ctypes.c_int]
        L.hjxo_max_threads.restype = ctypes.c_int
        L.hjxo_grid.argtypes = [PP, ctypes.c_int, dp, dp]
        L.hjxo_deriv_line.argtypes = [ctypes.c_int, dp, ctypes.c_long, ctypes.c_int,
                                      ctypes.c_double, dp, dp]
        L.hjxo_weno5.argtypes = [ctypes.c_double] * 5
        L.hjxo_weno5.restype = ctypes.c_double
        L.hjxo_deriv_axis.argtypes = [PP, dp, ctypes.c_int, dp, dp]
        L.hjxo_ham.argtypes = [PP, ctypes.c_long, dp]
        L.hjxo_ham.restype = ctypes.c_double
        L.hjxo_alpha.argtypes = [PP, dp]
        L.hjxo_cfl_dt.argtypes = [PP]
        L.hjxo_cfl_dt.restype = ctypes.c_double
        L.hjxo_rhs.argtypes = [PP, dp, dp]
        L.hjxo_step.argtypes = [PP, dp, dp, ctypes.c_double]
        L.hjxo_solve.argtypes = [PP, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.hjxo_solve.restype = ctypes.c_long
        L.hjxo_solve_part.argtypes = [PP, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_long, dp]
        L.hjxo_solve_part.restype = ctypes.c_long
        L.hjxo_cs_solve_loss.argtypes = [PP, dp, dp, dp, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         dp, dp, dp, dp]
        L.hjxo_cs_solve_loss.restype = ctypes.c_long
        CP = ctypes.POINTER(Claw)
        L.hjxo_claw_dt.argtypes = [CP, dp]
        L.hjxo_claw_dt.restype = ctypes.c_double
        L.hjxo_claw_step.argtypes = [CP, dp, dp, ctypes.c_double]
        L.hjxo_claw_solve.argtypes = [CP, dp, ctypes.c_double, dp, dp]
        L.hjxo_claw_solve.restype = ctypes.c_long
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")
    return rc


def set_threads(n):
    lib().hjxo_set_threads(int(n))


def max_threads():
    return lib().hjxo_max_threads()


def shape(P):
    return tuple(P.n[d] for d in range(P.dim))


def grid(P, d):
    """(dx, coordinates) of axis d."""
    dx = ctypes.c_double()
    xs = np.empty(P.n[d], np.float64)
    _check(lib().hjxo_grid(ctypes.byref(P), d, ctypes.byref(dx), _ptr(xs)), "grid")
    return dx.value, xs


def deriv_line(scheme, phi, dx, periodic=False):
    """(p-, p+) along a 1-D line, with ghost cells."""
    phi = _f64(phi)
    pm = np.empty_like(phi)
    pp = np.empty_like(phi)
    s = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    _check(lib().hjxo_deriv_line(s, _ptr(phi), phi.size, int(bool(periodic)), float(dx),
                                 _ptr(pm), _ptr(pp)), "deriv_line")
    return pm, pp


def weno5(v1, v2, v3, v4, v5):
    return lib().hjxo_weno5(v1, v2, v3, v4, v5)


def deriv_axis(P, phi, d):
    phi = _f64(phi)
    pm = np.empty_like(phi)
    pp = np.empty_like(phi)
    _check(lib().hjxo_deriv_axis(ctypes.byref(P), _ptr(phi), d, _ptr(pm), _ptr(pp)), "deriv")
    return pm, pp


def ham(P, flat_index, p):
    p = _f64(p)
    return lib().hjxo_ham(ctypes.byref(P), int(flat_index), _ptr(p))


def alpha(P):
    a = np.zeros(MAXD, np.float64)
    _check(lib().hjxo_alpha(ctypes.byref(P), _ptr(a)), "alpha")
    return a[:P.dim].copy()


def cfl_dt(P):
    return lib().hjxo_cfl_dt(ctypes.byref(P))


def rhs(P, phi):
    phi = _f64(phi)
    L = np.empty_like(phi)
    _check(lib().hjxo_rhs(ctypes.byref(P), _ptr(phi), _ptr(L)), "rhs")
    return L


def step(P, phi, dt, target=None):
    out = _f64(phi).copy()
    tgt = None if target is None else _f64(target)
    _check(lib().hjxo_step(ctypes.byref(P), _ptr(out), _ptr(tgt), float(dt)), "step")
    return out


def solve(P, phi0, t1, t0=0.0, target=None):
    """Returns (phi(t1), number of steps, first dt)."""
    phi0 = _f64(phi0)
    out = np.empty_like(phi0)
    tgt = None if target is None else _f64(target)
    dt0 = ctypes.c_double(0.0)
    n = _check(lib().hjxo_solve(ctypes.byref(P), _ptr(phi0), _ptr(tgt), float(t0), float(t1),
                                _ptr(out), ctypes.byref(dt0)), "solve")
    return out, n, dt0.value


def solve_part(P, phi, t0, t1, max_steps, target=None):
    """At most max_steps steps of solve() from t0 towards t1, in place on phi
    (float64, C-contiguous).  Returns (steps taken, t reached); continuing
    from there takes exactly the steps of one solve()."""
    assert phi.dtype == np.float64 and phi.flags.c_contiguous
    tgt = None if target is None else _f64(target)
    reached = ctypes.c_double(t0)
    n = _check(lib().hjxo_solve_part(ctypes.byref(P), _ptr(phi), _ptr(tgt), float(t0), float(t1), int(max_steps),
                                     ctypes.byref(reached)), "solve_part")
    return n, reached.value


def solve_in_parts(P, phi0, t1, t0=0.0, target=None, part=100, report=None):
    """solve() taken `part` steps at a time (the same steps, the same bits),
    calling report(steps_so_far, t) after each part.  Returns (phi(t1),
    number of steps)."""
    phi = _f64(phi0).copy()
    tgt = None if target is None else _f64(target)
    t, steps = float(t0), 0
    reached = ctypes.c_double(t)
    while t < t1:
        n = _check(lib().hjxo_solve_part(ctypes.byref(P), _ptr(phi), _ptr(tgt), t, float(t1), int(part),
                                         ctypes.byref(reached)), "solve_part")
        steps += n
        t = reached.value
        if report:
            report(steps, t)
        if n == 0:
            break
    return phi, steps


def cs_solve_loss(P, phi0, t1, dphi0=None, dparams=None, with_target=True, t0=0.0, eps_h=None,
                  h=1e-20, want_state=False):
    """Complex-step directional derivative of the smoothed-Heaviside volume
    loss after a solve.  Returns (loss, dloss, steps[, phi_T, dphi_T])."""
    phi0 = _f64(phi0)
    if eps_h is None:
        eps_h = 1.5 * max(grid(P, 0)[0], grid(P, 1)[0])
    d0 = None if dphi0 is None else _f64(dphi0)
    dh = None
    if dparams is not None:
        dh = np.zeros(8, np.float64)
        dh[:len(dparams)] = dparams
    loss = ctypes.c_double()
    dloss = ctypes.c_double()
    phT = np.empty_like(phi0) if want_state else None
    tan = np.empty_like(phi0) if want_state else None
    n = _check(lib().hjxo_cs_solve_loss(ctypes.byref(P), _ptr(phi0), _ptr(d0), _ptr(dh),
                                        int(bool(with_target)), float(t0), float(t1),
                                        float(eps_h), float(h), ctypes.byref(loss),
                                        ctypes.byref(dloss), _ptr(phT), _ptr(tan)), "cs_solve")
    if want_state:
        return loss.value, dloss.value, n, phT, tan
    return loss.value, dloss.value, n


def claw_dt(C, v):
    dt = lib().hjxo_claw_dt(ctypes.byref(C), _ptr(_f64(v)))
    if dt < 0:
        raise ValueError("oracle claw_dt rejected its arguments")
    return dt


def claw_step(C, v, dt):
    v = _f64(v)
    out = np.empty_like(v)
    _check(lib().hjxo_claw_step(ctypes.byref(C), _ptr(v), _ptr(out), float(dt)), "claw_step")
    return out


def claw_solve(C, v0, t1):
    """Returns (v(t1), number of steps, dt)."""
    v0 = _f64(v0)
    out = np.empty_like(v0)
    dt = ctypes.c_double(0.0)
    n = _check(lib().hjxo_claw_solve(ctypes.byref(C), _ptr(v0), float(t1), _ptr(out), ctypes.byref(dt)),
               "claw_solve")
    return out, n, dt.value
