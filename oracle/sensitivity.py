"""How far the FP64 oracle moves from itself under rounding-sized changes
(test infrastructure, like the rest of this package; nothing in the HIP path
uses it).

Two experiments on a workload of paper_2411_03501_amd.inputs, each a whole
solve with min-with-target:

  perturb   solve from phi0 and from phi0 * (1 + rel * U(-1, 1)) (seeded)
            and compare: max |diff|, share of nodes above 1e-10 and above
            1e-4 of the range, sign flips beyond two cells of the zero set;
  reflect   for the pursuit-evasion game, compare the solution with its
            image under (x, y, theta) -> (x, -y, -theta), a symmetry of the
            problem that its coordinate tables satisfy only to rounding.

Usage: python -m oracle.sensitivity perturb dubins3d --rel 6e-8 [--n 41 41 40] [--t1 2.8]
       python -m oracle.sensitivity reflect dubins3d --n 41 41 40 --t1 2.8
"""
import argparse
import os
import sys
import time

import numpy as np

import oracle as O

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2411_03501_amd import inputs  # noqa: E402


def _problem(w):
    return O.make_problem(gmin=w.gmin, gmax=w.gmax, n=w.n, periodic=w.periodic, ham=w.ham, params=w.params,
                          scheme=w.scheme, rk=w.rk, cfl=w.cfl)


def _near_zero(ref, periodic, width=2):
    lo, hi = ref.copy(), ref.copy()
    for d in range(ref.ndim):
        n = ref.shape[d]
        nlo, nhi = lo.copy(), hi.copy()
        for k in range(-width, width + 1):
            if k:
                if d in periodic:
                    a, b = np.roll(lo, -k, axis=d), np.roll(hi, -k, axis=d)
                else:
                    idx = np.clip(np.arange(n) + k, 0, n - 1)
                    a, b = np.take(lo, idx, axis=d), np.take(hi, idx, axis=d)
                nlo, nhi = np.minimum(nlo, a), np.maximum(nhi, b)
        lo, hi = nlo, nhi
    return ((ref > 0) & (lo <= 0)) | ((ref < 0) & (hi >= 0)) | (ref == 0)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["perturb", "reflect"])
    ap.add_argument("workload")
    ap.add_argument("--n", type=int, nargs="+")
    ap.add_argument("--t1", type=float)
    ap.add_argument("--rel", type=float, default=6e-8)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    a = ap.parse_args(argv)
    w = inputs.WORKLOADS[a.workload]
    if a.n:
        w = w.with_(n=tuple(a.n))
    if a.t1 is not None:
        w = w.with_(t1=a.t1)
    O.set_threads(min(a.threads, O.max_threads()))
    P = _problem(w)
    phi0 = inputs.initial_surface(w)
    tgt = w.with_target
    t = time.time()
    ref, steps, _ = O.solve(P, phi0, w.t1, target=phi0 if tgt else None)
    rng = ref.max() - ref.min()
    if a.what == "reflect":
        b = np.flip(ref, axis=1)
        nth = ref.shape[2]
        b = np.take(b, (nth - np.arange(nth)) % nth, axis=2)
        d = np.abs(ref - b)
        print(f"{w.name} n={w.n} t1={w.t1} steps {steps}: reflection asymmetry {d.max():.3e} "
              f"({time.time() - t:.0f} s)")
        return
    pert = phi0 * (1 + a.rel * np.random.default_rng(a.seed).uniform(-1, 1, size=phi0.shape))
    other, _, _ = O.solve(P, pert, w.t1, target=pert if tgt else None)
    d = np.abs(ref - other)
    far = ~_near_zero(ref, w.periodic)
    i = np.unravel_index(np.argmax(d), d.shape)
    print(f"{w.name} n={w.n} t1={w.t1} steps {steps}, phi0 perturbed by {a.rel:.0e} relative: "
          f"max |diff| {d.max():.3e} ({d.max() / rng:.1e} of the range) at {tuple(int(v) for v in i)}, "
          f"nodes above 1e-10: {(d > 1e-10).mean():.2%}, above 1e-4 of the range: {(d > 1e-4 * rng).mean():.2%}, "
          f"sign flips beyond two cells: {int((far & (np.sign(ref) != np.sign(other))).sum())} "
          f"({time.time() - t:.0f} s)")


if __name__ == "__main__":
    main()
