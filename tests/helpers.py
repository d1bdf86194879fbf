"""Shared test helpers: problem construction on both sides from one seeded
workload description, and the comparison rules."""
import numpy as np

import oracle as O
from paper_2411_03501_amd import inputs

# FP64: max-abs difference to the oracle; FP32: relative to the oracle's range
TOL_F64 = 1e-10
TOL_F32_REL = 1e-4


def oracle_problem(w, **over):
    """The oracle's problem for workload w; decide="f32" takes the ENO
    stencil choices in binary32, as an FP32 solver takes them."""
    kw = dict(gmin=w.gmin, gmax=w.gmax, n=w.n, periodic=w.periodic, ham=w.ham, params=w.params,
              scheme=w.scheme, rk=w.rk, cfl=w.cfl, restrict=w.restrict,
              dissipation=w.dissipation)
    kw.update(over)
    return O.make_problem(**kw)


def gpu_problem(w, dtype=None, **over):
    from paper_2411_03501_amd import hjx
    kw = dict(gmin=w.gmin, gmax=w.gmax, n=w.n, periodic=w.periodic, ham=w.ham, params=w.params,
              scheme=w.scheme, rk=w.rk, cfl=w.cfl, dtype=dtype or w.dtype, restrict=w.restrict,
              dissipation=w.dissipation)
    kw.update(over)
    return hjx.Problem(**kw)


def as_input(a, dtype):
    """The values a solver in `dtype` actually receives: `a` rounded to
    binary32 for "f32" (returned as float64, exactly), unchanged for "f64".
    Parity is taken on the same inputs on both sides."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if dtype == "f32" else a


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def to_host(t):
    return t.detach().to("cpu", dtype=__import__("torch").float64).numpy()


def near_zero_mask(ref, periodic=(), width=2):
    """Nodes with a node of the opposite sign (or a zero) of `ref` within
    `width` cells in the max-norm: separable min/max filters, wrapping on
    periodic axes and clipping elsewhere."""
    lo = ref.copy()
    hi = ref.copy()
    for d in range(ref.ndim):
        n = ref.shape[d]
        new_lo = lo.copy()
        new_hi = hi.copy()
        for k in range(-width, width + 1):
            if k == 0:
                continue
            if d in periodic:
                sl = np.roll(lo, -k, axis=d), np.roll(hi, -k, axis=d)
            else:
                idx = np.clip(np.arange(n) + k, 0, n - 1)
                sl = np.take(lo, idx, axis=d), np.take(hi, idx, axis=d)
            new_lo = np.minimum(new_lo, sl[0])
            new_hi = np.maximum(new_hi, sl[1])
        lo, hi = new_lo, new_hi
    # some neighbour has the other sign (or is zero)
    return ((ref > 0) & (lo <= 0)) | ((ref < 0) & (hi >= 0)) | (ref == 0)


def oracle_binary32_state(Po, phi0, t1, target=None):
    """The oracle's solve from phi0 with its state rounded to binary32 after
    every step (the same schedule: one step per part of the oracle's own
    time loop).  Every value is still computed in FP64; only the storage
    between steps is binary32, as an FP32 solver's is at the least."""
    phi = np.ascontiguousarray(phi0, dtype=np.float64).copy()
    t, steps = 0.0, 0
    while t < t1:
        n, t = O.solve_part(Po, phi, t, t1, 1, target)
        phi[...] = phi.astype(np.float32)
        steps += n
        if n == 0:
            break
    return phi, steps


def assert_close(got, ref, dtype, periodic=(), what="", f32_floor=0.0):
    """FP64: |got - ref| <= 1e-10.  FP32: |got - ref| <= max(1e-4 * range(ref),
    f32_floor) and sign(got) == sign(ref) beyond two cells from the zero
    level set.  f32_floor: how far the oracle itself moves with a binary32
    state (oracle_binary32_state), for whole solves."""
    err = np.abs(got - ref).max()
    if dtype == "f64":
        assert err <= TOL_F64, f"{what}: max |gpu - oracle| = {err:.3e} > {TOL_F64}"
        return err
    rng = ref.max() - ref.min()
    tol = max(TOL_F32_REL * rng, f32_floor)
    assert err <= tol, (f"{what}: max |gpu - oracle| = {err:.3e} > max(1e-4 * range {rng:.3e}, "
                        f"binary32-state floor {f32_floor:.3e})")
    far = ~near_zero_mask(ref, periodic)
    bad = far & (np.sign(got) != np.sign(ref))
    assert not bad.any(), f"{what}: {bad.sum()} sign disagreements beyond two cells of the zero set"
    return err


def workload_phi0(w):
    return inputs.initial_surface(w)
