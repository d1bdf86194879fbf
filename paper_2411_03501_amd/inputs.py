"""Seeded synthetic inputs for the level-set workloads.

This module only describes problems and builds input arrays: grid extents,
Hamiltonian parameters, scheme choices, initial implicit surfaces and random
test fields.  It holds none of the solver's arithmetic (no stencils,
Hamiltonians, dissipation, time step or integrator), imports nothing from the
rest of the package, and is the only code that the HIP library's callers and
the CPU oracle's callers have in common.

Workloads (all synthetic; the paper measures on no dataset):
  normal2d   2-D motion in the normal direction, H = a|grad phi|, a = 1,
             phi0 = |x| - 0.5 on 101 x 101 nodes over [-1, 1]^2,
             first-order upwind + forward Euler, CFL 0.75, horizon 0.3, FP64.
  dubins3d   3-D pursuit-evasion of two unicycles in relative coordinates
             (x, y, theta), v_e = v_p = 5, |w_e|, |w_p| <= 1, 101^3 nodes over
             [-6, 20] x [-10, 10] x [0, 2 pi) periodic in theta,
             phi0 = cylinder of radius 5, WENO5 + LF + TVD-RK3,
             backward reachable tube (min with target) to horizon 2.8.
  dubins3d_81  the same at 81^3 (gradient workload), FP32.
  car4d      4-D car with speed state (x, y, theta, v), |w| <= 1, |a| <= 1,
             81^4 nodes over [-5, 5]^2 x [0, 2 pi) x [0, 2], theta periodic,
             phi0 = cylinder of radius 1 in (x, y), WENO5 + LF + RK3 to 1.5.
  batch256   256 seeded instances of the 2-D and 3-D kinds above with uneven
             grids (64..161 nodes per axis), radii in [0.3, 5], speeds in
             [0.5, 5] and 16..64 steps each (numpy default_rng(2411)).
"""
from dataclasses import dataclass, field, replace
import math

import numpy as np


@dataclass
class Workload:
    name: str
    gmin: tuple
    gmax: tuple
    n: tuple
    periodic: tuple = ()
    ham: str = "normal"           # normal | dubins3_pe | dubins4
    params: tuple = (1.0,)
    scheme: str = "weno5"         # first | eno2 | eno3 | weno5
    rk: int = 3
    cfl: float = 0.75
    t1: float = 1.0
    with_target: bool = False
    radius: float = 0.5           # of the initial implicit surface
    surface: str = "sphere"       # sphere: |x| - r over all axes; cylinder: |(x0, x1)| - r
    dtype: str = "f64"
    steps: int = 0                # batch instances: number of full steps
    extra: dict = field(default_factory=dict)
    restrict: str = "none"        # restricted update: none | nonpositive | positive
    dissipation: str = "global"   # Lax-Friedrichs alpha: global | local

    @property
    def dim(self):
        return len(self.n)

    @property
    def points(self):
        return int(np.prod(self.n))

    def with_(self, **kw):
        return replace(self, **kw)


NORMAL2D = Workload("normal2d", (-1.0, -1.0), (1.0, 1.0), (101, 101), (), "normal", (1.0,),
                    "first", 1, 0.75, 0.3, False, 0.5, "sphere", "f64")
DUBINS3D = Workload("dubins3d", (-6.0, -10.0, 0.0), (20.0, 10.0, 2 * math.pi), (101, 101, 101), (2,),
                    "dubins3_pe", (5.0, 5.0, 1.0, 1.0), "weno5", 3, 0.75, 2.8, True, 5.0,
                    "cylinder", "f64")
DUBINS3D_81 = DUBINS3D.with_(name="dubins3d_81", n=(81, 81, 81), dtype="f32")
CAR4D = Workload("car4d", (-5.0, -5.0, 0.0, 0.0), (5.0, 5.0, 2 * math.pi, 2.0), (81, 81, 81, 81), (2,),
                 "dubins4", (1.0, 1.0), "weno5", 3, 0.75, 1.5, False, 1.0, "cylinder", "f32")

# The two-rocket game (Sec. VI): 100 nodes per axis, x and z over [-64, 64],
# the angle over [-pi/2, pi/2]; a = 1, g = 32, unit control bounds; ENO2 with
# second-order TVD-RK over 2.5 s; capture radius 1.5 (a cylinder along the
# angle); the listing's 'positive' restricted update.
ROCKETS = Workload("rockets", (-64.0, -64.0, -math.pi / 2), (64.0, 64.0, math.pi / 2), (100, 100, 100), (),
                   "rockets", (1.0, 32.0, 1.0, 1.0), "eno2", 2, 0.75, 2.5, False, 1.5, "cylinder", "f32",
                   restrict="positive")

WORKLOADS = {w.name: w for w in (NORMAL2D, DUBINS3D, DUBINS3D_81, CAR4D, ROCKETS)}

# A scalar conservation law (Sec. IV-D) at a size that fills the GPU:
# Burgers' equation v_t + (c0 v^2/2)_x + (c1 v^2/2)_y = 0 on the periodic unit
# square, 4096^2 nodes, c = (1, 0.5), CFL 0.9; params holds c.
BURGERS2D = Workload("burgers2d", (0.0, 0.0), (1.0, 1.0), (4096, 4096), (0, 1), "burgers", (1.0, 0.5),
                     "lf", 1, 0.9, 0.0, False, 0.0, "none", "f32")


def burgers_initial(w, seed=2411):
    """Smooth data for the Burgers workload: 1 plus a seeded low-mode
    Fourier sum of amplitude 0.5 (shocks form as it steepens)."""
    return 1.0 + 0.5 * smooth_field(w.n, seed)


def node_axes(w):
    """Node positions per axis: non-periodic axes include both ends,
    periodic axes are the half-open [gmin, gmax)."""
    axes = []
    for d in range(w.dim):
        n = w.n[d]
        span = w.gmax[d] - w.gmin[d]
        h = span / n if d in w.periodic else span / (n - 1)
        axes.append(w.gmin[d] + np.arange(n, dtype=np.float64) * h)
    return axes


def initial_surface(w):
    """Signed distance to a sphere (all axes) or to a cylinder along the
    first two axes, minus the radius: phi0 < 0 inside.  float64."""
    axes = node_axes(w)
    if w.surface == "sphere":
        r2 = 0.0
        for d in range(w.dim):
            shp = [1] * w.dim
            shp[d] = w.n[d]
            r2 = r2 + axes[d].reshape(shp) ** 2
        phi = np.sqrt(r2) - w.radius
    elif w.surface == "cylinder":
        shp0 = [1] * w.dim
        shp0[0] = w.n[0]
        shp1 = [1] * w.dim
        shp1[1] = w.n[1]
        phi = np.sqrt(axes[0].reshape(shp0) ** 2 + axes[1].reshape(shp1) ** 2) - w.radius
    else:
        raise ValueError(w.surface)
    return np.array(np.broadcast_to(phi, w.n), dtype=np.float64, order="C", copy=True)


def smooth_field(shape, seed, modes=4, amplitude=1.0):
    """A smooth random field on the unit box (periodic in every axis):
    a seeded sum of a few low Fourier modes."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    out = np.zeros(shape, np.float64)
    for _ in range(modes):
        k = rng.integers(-2, 3, size=len(shape))
        ph = rng.uniform(0, 2 * np.pi)
        a = rng.normal()
        arg = sum(2 * np.pi * k[d] * grids[d] for d in range(len(shape))) + ph
        out += a * np.cos(arg)
    return amplitude * out


def rough_field(shape, seed, amplitude=1.0):
    """Seeded uniform noise in [-amplitude, amplitude]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=shape)


def batch256(count=256, seed=2411):
    """The uneven batched workload.  Draw order per instance: kind, radius,
    speed, nodes per axis, steps."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        kind = int(rng.integers(0, 2))
        r = float(rng.uniform(0.3, 5.0))
        s = float(rng.uniform(0.5, 5.0))
        dim = 2 if kind == 0 else 3
        n = tuple(int(v) for v in rng.integers(64, 162, size=dim))
        steps = int(rng.integers(16, 65))
        if kind == 0:
            w = Workload(f"batch{k}_normal2d", (-2 * r, -2 * r), (2 * r, 2 * r), n, (), "normal", (s,),
                         "weno5", 3, 0.75, 0.0, False, r, "sphere", "f32", steps)
        else:
            w = Workload(f"batch{k}_dubins3d", (-1.2 * r, -2 * r, 0.0), (4 * r, 2 * r, 2 * math.pi), n,
                         (2,), "dubins3_pe", (s, s, 1.0, 1.0), "weno5", 3, 0.75, 0.0, True, r,
                         "cylinder", "f32", steps)
        out.append(w)
    return out
