"""Throughput of the level-set hot path on one MI355X.

A bench step is one whole solve of the workload: the dissipation reduction,
the CFL step and every WENO5 + Lax-Friedrichs + TVD-RK3 step to the horizon,
on synthetic inputs already resident in HBM.  Default workload (the largest
one GPU holds): the 4-D Dubins car with a speed state (x, y, theta, v),
|w| <= 1, |a| <= 1, 81^4 = 43,046,721 nodes over [-5,5]^2 x [0,2pi) x [0,2],
phi0 = a cylinder of radius 1 in (x, y), horizon 1.5 (170 RK3 steps), FP32.
The 3-D pursuit-evasion game (101^3, 874 steps with min-with-target) runs
as a secondary leg in FP32 and FP64.

Prints ONE JSON line.  value = grid-point updates/s, a grid-point update
being one node advanced by one full RK3 step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one FP32 or FP64 operation, FMA counted once, per lane per clock; packed
# FP32 is not used)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_ops_per_point(scheme, ham, dim, dtype="f32"):
    """Algorithmic VALU operations per node per RK stage (FMA = 1).

    WENO5 follows the scope table's estimate of the method's arithmetic,
    with every interval's WENO5 window shared by the two nodes it serves:
    per node per RK3 step about 900 operations in 3-D and 1150 in 4-D in
    FP32, and 100 per axis plus 40 for H, LF and RK per stage in FP64
    (division and reciprocals take several instructions there).  First
    order: two differences and two scalings per axis plus H, LF and RK."""
    if scheme == "weno5":
        if dtype == "f64":
            return 100 * dim + 40
        return {1: 115.0, 2: 190.0, 3: 900.0 / 3, 4: 1150.0 / 3}[dim]
    ham_lf = {"normal": 2 * dim + 2 + 2 * dim, "dubins3_pe": 27, "dubins4": 26, "rockets": 27}[ham]
    return 4 * dim + ham_lf + 4


def stage_bytes_per_point(rk, with_target, elem):
    reads_writes = {1: 2, 2: 5, 3: 8}[rk] + (1 if with_target else 0)
    return reads_writes * elem / rk


def describe(w, rk_steps):
    """The workload in words: problem, grid, scheme, horizon."""
    what = {"normal": f"{w.dim}-D motion in the normal direction",
            "dubins3_pe": "3-D pursuit-evasion game of two Dubins cars",
            "dubins4": "4-D Dubins car with a speed state",
            "rockets": "3-D game of two rockets"}[w.ham]
    scheme = {"first": "first-order upwind", "eno2": "ENO2", "eno3": "ENO3", "weno5": "WENO5"}[w.scheme]
    rk = {1: "forward Euler", 2: "TVD-RK2", 3: "TVD-RK3"}[w.rk]
    tube = ", min-with-target (BRT)" if w.with_target else ""
    return (f"{w.name}: {what}, {'x'.join(map(str, w.n))} nodes, {scheme}+LF+{rk}{tube}, horizon {w.t1} "
            f"({rk_steps} RK steps per solve)")


# the sources that define the stage kernels (their per-node arithmetic and launch)
KERNEL_SOURCES = ["paper_2411_03501_amd/csrc/hjx_device.h", "paper_2411_03501_amd/csrc/hjx_tile.h",
                  "paper_2411_03501_amd/csrc/hjx_kernels.hip"]


def strip_comments(src):
    """C++ source without its comments and with runs of whitespace made one
    space: what the compiler sees, as far as a kernel's code goes.  String
    and character literals are kept as they are."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_sources_sha256():
    """sha256 of the stage-kernel sources without comments or layout, so
    that the counters taken for a kernel stay attached to it until its code
    changes."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()


def measured_traffic(w, dtype, tile):
    """HBM bytes per stage launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings), or None
    when there is none for this workload and tile or the kernel sources have
    changed since the counters were taken."""
    import re
    name = f"traffic_{w.name}_{dtype}.md"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    src = re.search(r"kernel sources sha256: ([0-9a-f]{64})", text)
    tl = re.search(r"tile: \(([\d, ]+)\)", text)
    val = re.search(r"HBM bytes per launch: ([0-9.e+]+)", text)
    if not (src and tl and val) or src.group(1) != kernel_sources_sha256():
        return None
    if tuple(int(v) for v in tl.group(1).split(",")) != tuple(tile):
        return None
    return float(val.group(1))


def run_gpu(w, dtype, steps, warmup, tile=None):
    import torch

    from paper_2411_03501_amd import hjx, inputs

    tdt = torch.float32 if dtype == "f32" else torch.float64
    P = hjx.Problem.from_workload(w, dtype)
    phi0 = torch.from_numpy(inputs.initial_surface(w)).to("cuda", dtype=tdt)
    target = phi0 if w.with_target else None
    out = torch.empty_like(phi0)
    if tile is None:
        tile, us = P.tune(phi0, reps=8)   # launch-shape autotuner (outside the timed region)
        log(f"  tuned tile {tile}: {us:.2f} us per stage launch")
    else:
        P.tile = tile
        tile = P.tile
        log(f"  fixed tile {tile}")
    for i in range(warmup):
        P.solve(phi0, w.t1, target=target, out=out)
        log(f"  warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    loop_ms = []
    t0 = time.perf_counter()
    for i in range(steps):
        _, st = P.solve(phi0, w.t1, target=target, out=out)
        loop_ms.append(st["elapsed_ms"])
        log(f"  step {i + 1}/{steps}: {st['steps']} RK steps, loop {st['elapsed_ms']:.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    P.close()
    st["tile"] = list(tile)
    return elapsed, st, loop_ms


def run_adjoint(w, reps=2):
    """Gradient workload: forward solve (plain) vs backward (segment replay +
    reverse sweep, checkpoint every 8 steps) of the smoothed-volume loss,
    and central differences (FP64 solves on the same GPU) of dL/dtheta for
    every Hamiltonian parameter and of dL/dphi0 along three smooth
    directions."""
    import numpy as np
    import torch

    from paper_2411_03501_amd import hjx, inputs

    P = hjx.Problem.from_workload(w, "f32")
    phi0 = torch.from_numpy(inputs.initial_surface(w)).to("cuda", dtype=torch.float32)
    tile, tile_us = P.tune(phi0, reps=8)   # the forward at its fastest launch shape
    log(f"  adjoint forward: tuned tile {tile}: {tile_us:.2f} us per stage launch")
    dx = [(w.gmax[d] - w.gmin[d]) / (w.n[d] if d in w.periodic else w.n[d] - 1) for d in range(w.dim)]
    eps = 1.5 * max(dx[0], dx[1])
    out = torch.empty_like(phi0)
    P.solve(phi0, w.t1, target=phi0, out=out)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.solve(phi0, w.t1, target=phi0, out=out)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / reps
    tape = P.tape(w.t1, ckpt_every=8)
    tape.solve(phi0, target=phi0, out=out)
    loss, g = P.loss_volume(out, eps)
    tape.adjoint(g, sum_target=True)  # warm-up
    torch.cuda.synchronize()
    bwd_times = []
    for _ in range(reps):
        tape.solve(phi0, target=phi0, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, g = P.loss_volume(out, eps)
        g0, _, dp = tape.adjoint(g, sum_target=True)   # dL/dphi0 through the initial value and the target
        torch.cuda.synchronize()
        bwd_times.append(time.perf_counter() - t0)
    bwd = min(bwd_times)
    log(f"  adjoint: forward {fwd * 1e3:.1f} ms, backward {bwd * 1e3:.1f} ms")
    grad_phi0 = g0.double()

    # central differences of FP64 solves with small steps (the loss is only
    # piecewise smooth: a large step crosses changes of the step count, and
    # the theta-independent surface sits on a kink of WENO5 for directions
    # that vary with theta, so the phi0 direction here does not)
    phi64 = phi0.double()

    def loss_at(params, f0):
        Q = hjx.Problem(w.gmin, w.gmax, w.n, w.periodic, w.ham, params, w.scheme, w.rk, w.cfl, "f64")
        o, _ = Q.solve(f0, w.t1, target=f0)
        v = Q.loss_volume(o, eps, grad=False)
        Q.close()
        return v

    # every Hamiltonian parameter (relative steps) and three smooth
    # directions of phi0 that do not vary with theta
    fd_params, rel_params = [], []
    for m in range(len(w.params)):
        h = 1e-5 * w.params[m]
        pp = list(w.params)
        pm = list(w.params)
        pp[m] += h
        pm[m] -= h
        fd = (loss_at(pp, phi64) - loss_at(pm, phi64)) / (2 * h)
        fd_params.append(fd)
        rel_params.append(abs(dp[m] - fd) / max(abs(fd), 1e-12))
    fd_dirs, adj_dirs, rel_dirs = [], [], []
    for seed in (5, 6, 7):
        d2 = inputs.smooth_field(w.n[:2], seed)
        delta = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(d2[:, :, None], w.n))).to("cuda")
        hd = 1e-5
        fd = (loss_at(w.params, phi64 + hd * delta) - loss_at(w.params, phi64 - hd * delta)) / (2 * hd)
        adj = float((grad_phi0 * delta).sum())
        fd_dirs.append(fd)
        adj_dirs.append(adj)
        rel_dirs.append(abs(adj - fd) / abs(fd))
    tape.close()
    P.close()
    log(f"  central differences: params rel err {max(rel_params):.1e}, phi0 directions rel err {max(rel_dirs):.1e}")
    return {"workload": f"{w.name}: {'x'.join(map(str, w.n))} FP32, horizon {w.t1}, checkpoint every 8 steps",
            "forward_tile": list(tile), "forward_stage_us": tile_us,
            "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3, "adjoint_over_forward": bwd / fwd,
            "loss": loss, "dL_dparams_adjoint": list(dp[:len(w.params)]), "dL_dparams_central_diff": fd_params,
            "dL_dphi0_dirs_adjoint": adj_dirs, "dL_dphi0_dirs_central_diff": fd_dirs,
            "max_rel_err_params": max(rel_params), "max_rel_err_phi0_dirs": max(rel_dirs),
            "central_diff": "FP64 solves, steps 1e-5 (relative for the parameters), phi0 directions independent "
                            "of theta; parameters (v_e, v_p, wbar_e, wbar_p)"}


def run_batch(reps=2):
    """The uneven 256-member batch (2-D level sets moving in the normal
    direction and 3-D pursuit-evasion games, 64..161 nodes per axis, 16..64
    RK3 steps each, FP32): one batched solve (persistent stage launches
    replayed from a hipGraph) against a loop of per-member hjx_solve calls
    over the same members, inputs and horizons."""
    import torch

    from paper_2411_03501_amd import hjx, inputs

    ws = inputs.batch256()
    probs = [hjx.Problem.from_workload(w, "f32") for w in ws]
    phi0 = [torch.from_numpy(inputs.initial_surface(w)).to("cuda", dtype=torch.float32) for w in ws]
    t1 = [w.steps * P.dissipation()[1] for w, P in zip(ws, probs)]
    target = [x if w.with_target else None for x, w in zip(phi0, ws)]
    out = [torch.empty_like(x) for x in phi0]
    updates = sum(w.points * w.steps for w in ws)
    log(f"  batch256: {sum(w.points for w in ws) / 1e6:.1f} M nodes, {updates / 1e9:.2f} G updates per solve")

    def singles():
        for P, x, t, g, o in zip(probs, phi0, t1, target, out):
            P.solve(x, t, target=g, out=o)

    singles()   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        singles()
    torch.cuda.synchronize()
    single_s = (time.perf_counter() - t0) / reps

    B = hjx.Batch(probs)
    shape, tuned_ms = B.tune(phi0, t1, target=target, out=out, reps=1)
    log(f"  tuned batch shape {shape}: {tuned_ms:.1f} ms per horizon")
    B.solve(phi0, t1, target=target, out=out)   # warm-up
    torch.cuda.synchronize()
    graph_ms = []
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = B.solve(phi0, t1, target=target, out=out)
        graph_ms.append(st[0]["elapsed_ms"])
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / reps
    log(f"  per-member solves {single_s * 1e3:.1f} ms, batched {batch_s * 1e3:.1f} ms "
        f"(graph {min(graph_ms):.1f} ms)")
    B.close()
    for P in probs:
        P.close()
    return {"members": len(ws), "nodes": sum(w.points for w in ws), "updates_per_solve": updates,
            "batched_updates_per_s": updates / batch_s, "per_member_updates_per_s": updates / single_s,
            "batched_ms": batch_s * 1e3, "per_member_ms": single_s * 1e3, "graph_replay_ms": min(graph_ms),
            "speedup": single_s / batch_s, "shape": {"item_nodes": shape[0], "blocks": shape[1]}}


def run_first_order_large(n=4096, steps=2, warmup=1, dissipation="global"):
    """The HBM-bound path at a size that fills the GPU: normal2d's scheme
    (FP64, first-order upwind + forward Euler, CFL 0.75, no target) on
    n x n nodes to the same horizon.  Algorithmic bytes per launch: phi read
    once and the result written once (the neighbours' re-reads are halo)."""
    from paper_2411_03501_amd import inputs

    w = inputs.NORMAL2D.with_(name=f"normal2d_{n}", n=(n, n), dissipation=dissipation)
    elapsed, st, loop_ms = run_gpu(w, "f64", steps, warmup)
    launches = st["steps"] * w.rk
    kern_s = (sum(loop_ms) / len(loop_ms)) / 1e3 / launches
    bytes_launch = stage_bytes_per_point(w.rk, w.with_target, 8) * w.points
    gbs = bytes_launch / kern_s / 1e9
    log(f"  {w.name}: {st['steps']} steps, {kern_s * 1e6:.1f} us per launch, {gbs:.0f} GB/s algorithmic")
    flux = "Lax-Friedrichs" if dissipation == "global" else f"{dissipation} numerical Hamiltonian"
    return {"workload": f"{w.name}: {n}x{n} FP64, first-order upwind + forward Euler, {flux}, {st['steps']} steps",
            "updates_per_s": w.points * st["steps"] * steps / elapsed, "stage_kernel_us": kern_s * 1e6,
            "tile": st["tile"], "bytes_per_launch": bytes_launch, "hbm_alg_gbs": gbs,
            "hbm_frac": gbs / PEAK_HBM_GBS}


def run_variant(w, what, dtype="f32", steps=2, warmup=1, plain_us=None, **change):
    """A scheme variant on the headline workload (the same grid, scheme,
    horizon and target), through the stage kernels compiled for it."""
    wt = w.with_(**change)
    elapsed, st, loop_ms = run_gpu(wt, dtype, steps, warmup)
    kern_s = (sum(loop_ms) / len(loop_ms)) / 1e3 / (st["steps"] * wt.rk)
    ops = alg_ops_per_point(wt.scheme, wt.ham, wt.dim) * wt.points
    res = {"workload": f"{w.name} {dtype} with {what}, {st['steps']} RK steps",
           "updates_per_s": wt.points * st["steps"] * steps / elapsed, "stage_kernel_us": kern_s * 1e6,
           "tile": st["tile"], "alu_frac": ops / kern_s / 1e12 / PEAK_VALU_TOPS}
    if plain_us:
        res["stage_us_over_plain"] = kern_s * 1e6 / plain_us
    log(f"  {what}: {kern_s * 1e6:.2f} us per stage launch")
    return res


def run_tube(w, dtype="f32", steps=2, warmup=1, plain_us=None):
    """The restricted update (tube form: every stage's rate clipped to
    min(L, 0)) on the headline workload."""
    return run_variant(w, "the tube form's clip min(L, 0)", dtype, steps, warmup, plain_us, restrict="nonpositive")


def run_local(w, dtype="f32", steps=2, warmup=1, plain_us=None):
    """Local Lax-Friedrichs dissipation (alpha_d at the node) on the headline
    workload."""
    return run_variant(w, "local Lax-Friedrichs dissipation", dtype, steps, warmup, plain_us, dissipation="local")


def run_rockets(steps=2, warmup=1):
    """The paper's own workload, the two-rocket game: 100^3 nodes, ENO2 +
    LF + TVD-RK2 over 2.5 s with the positive restricted update, FP32."""
    from paper_2411_03501_amd import inputs

    w = inputs.ROCKETS
    elapsed, st, loop_ms = run_gpu(w, "f32", steps, warmup)
    kern_s = (sum(loop_ms) / len(loop_ms)) / 1e3 / (st["steps"] * w.rk)
    bytes_launch = stage_bytes_per_point(w.rk, w.with_target, 4) * w.points
    log(f"  rockets: {st['steps']} RK steps, {kern_s * 1e6:.2f} us per stage launch")
    return {"workload": describe(w, st["steps"]) + ", positive restricted update, FP32",
            "updates_per_s": w.points * st["steps"] * steps / elapsed, "stage_kernel_us": kern_s * 1e6,
            "tile": st["tile"], "hbm_alg_gbs": bytes_launch / kern_s / 1e9,
            "hbm_alg_frac": bytes_launch / kern_s / 1e9 / PEAK_HBM_GBS}


def run_claw(steps=400, warmup=20):
    """Scalar conservation law (Sec. IV-D, Lax-Friedrichs): periodic 2-D
    Burgers at 4096^2, FP32.  Algorithmic bytes per step: the old values
    read once and the new ones written once (the neighbours' re-reads are
    halo), 8 bytes per node."""
    import torch

    from paper_2411_03501_amd import hjx, inputs

    w = inputs.BURGERS2D
    G = hjx.Claw(w.gmin, w.gmax, w.n, periodic=w.periodic, flux="burgers", c=w.params, cfl=w.cfl, dtype="f32")
    a = torch.from_numpy(inputs.burgers_initial(w)).to("cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    dt = G.dt(a)
    for _ in range(warmup):
        G.step(a, dt, out=b)
        a, b = b, a
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        G.step(a, dt, out=b)
        a, b = b, a
    e1.record()
    torch.cuda.synchronize()
    kern_s = e0.elapsed_time(e1) / 1e3 / steps
    # a whole solve (input check, CFL reduction, the steps, output check)
    v0 = torch.from_numpy(inputs.burgers_initial(w)).to("cuda", dtype=torch.float32)
    t0 = time.perf_counter()
    _, st = G.solve(v0, (steps - 0.5) * G.dt(v0), out=b)
    solve_s = time.perf_counter() - t0
    G.close()
    bytes_step = 2 * 4 * w.points
    gbs = bytes_step / kern_s / 1e9
    log(f"  burgers2d: {kern_s * 1e6:.2f} us per step, {gbs:.0f} GB/s algorithmic")
    return {"workload": "burgers2d: 2-D Burgers, 4096x4096 periodic, Lax-Friedrichs, CFL 0.9, FP32",
            "step_kernel_us": kern_s * 1e6, "updates_per_s": w.points / kern_s,
            "solve_updates_per_s": w.points * st["steps"] / solve_s, "solve_steps": st["steps"],
            "bytes_per_step": bytes_step, "hbm_alg_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}


def run_shapes():
    """Initial data of the 256-member batch (a sphere or a cylinder per
    member, 186.9 M nodes, FP32) built on the device by hjx_shape, against
    the host recipe that the batched benchmark otherwise uses."""
    import torch

    from paper_2411_03501_amd import hjx, inputs

    ws = inputs.batch256()
    outs = [torch.empty(w.n, dtype=torch.float32, device="cuda") for w in ws]
    specs = [dict(gmin=w.gmin, gmax=w.gmax, n=w.n, periodic=w.periodic, radius=w.radius,
                  axes=None if w.surface == "sphere" else (0, 1)) for w in ws]

    def per_member():
        for sp, o in zip(specs, outs):
            hjx.shape(dtype="f32", out=o, **sp)

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    one_ms = timed(per_member)
    dev_ms = timed(lambda: hjx.shape_batch(specs, dtype="f32", outs=outs))
    t0 = time.perf_counter()
    for w in ws[:32]:
        inputs.initial_surface(w)
    host_ms = (time.perf_counter() - t0) * 1e3 * len(ws) / 32
    nodes = sum(w.points for w in ws)
    log(f"  batch256 initial data: one launch {dev_ms:.2f} ms, a launch per member {one_ms:.2f} ms, "
        f"host recipe about {host_ms:.0f} ms")
    return {"workload": f"initial data of batch256: {len(ws)} spheres and cylinders, {nodes / 1e6:.1f} M nodes, FP32",
            "device_ms": dev_ms, "per_member_launches_ms": one_ms, "host_recipe_ms_est": host_ms,
            "write_gbs": nodes * 4 / dev_ms / 1e6, "hbm_frac": nodes * 4 / dev_ms / 1e6 / PEAK_HBM_GBS,
            "host_sample": "the host recipe (float64 numpy) timed on the first 32 members, scaled to 256"}


def run_small(reps=20):
    """The launch-bound workload: normal2d (101^2, FP64, first-order upwind +
    forward Euler, 40 steps).  Per solve: hjx_solve repeated with the same
    arguments (its stepping launches captured on the second call and
    replayed, plus the non-finite checks and one synchronisation), hjx_solve
    with graphs off (HJX_SOLVE_GRAPH=0: direct launches), and the same solve
    as a batch of one member (the batch's own horizon graph)."""
    import torch

    from paper_2411_03501_amd import hjx, inputs

    w = inputs.NORMAL2D
    P = hjx.Problem.from_workload(w, "f64")
    phi0 = torch.from_numpy(inputs.initial_surface(w)).to("cuda", dtype=torch.float64)
    out = torch.empty_like(phi0)
    _, st = P.solve(phi0, w.t1, out=out)   # direct launches
    P.solve(phi0, w.t1, out=out)           # the same solve again: captured into a graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        P.solve(phi0, w.t1, out=out)       # replays
    torch.cuda.synchronize()
    single = (time.perf_counter() - t0) / reps
    os.environ["HJX_SOLVE_GRAPH"] = "0"
    try:
        P.solve(phi0, w.t1, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            P.solve(phi0, w.t1, out=out)   # direct launches every time
        torch.cuda.synchronize()
        direct = (time.perf_counter() - t0) / reps
    finally:
        del os.environ["HJX_SOLVE_GRAPH"]
    B = hjx.Batch([P])
    shape, _ = B.tune([phi0], [w.t1], out=[out], reps=3)
    B.solve([phi0], [w.t1], out=[out])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph_ms = []
    for _ in range(reps):
        _, bst = B.solve([phi0], [w.t1], out=[out])
        graph_ms.append(bst[0]["elapsed_ms"])
    torch.cuda.synchronize()
    batched = (time.perf_counter() - t0) / reps
    B.close()
    P.close()
    n = st["steps"]
    upd = w.points * n
    log(f"  normal2d: {n} steps, hjx_solve {single * 1e6:.0f} us (direct launches {direct * 1e6:.0f} us), "
        f"batch of one {batched * 1e6:.0f} us (graph {min(graph_ms) * 1e3:.0f} us, shape {shape})")
    return {"workload": f"normal2d: 101x101 FP64, first-order + forward Euler, {n} steps",
            "steps": n, "solve_us": single * 1e6, "solve_direct_us": direct * 1e6, "graph_solve_us": batched * 1e6,
            "graph_replay_us": min(graph_ms) * 1e3, "us_per_step_graph": min(graph_ms) * 1e3 / n,
            "updates_per_s": upd / single, "graph_updates_per_s": upd / batched,
            "graph_shape": {"item_nodes": shape[0], "blocks": shape[1]}}


def run_copy(nbytes=1 << 30, reps=4):
    """A plain device-to-device copy of nbytes (torch's copy kernel): HBM
    counters of this kernel give the scale between counter readings and
    bytes moved."""
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"bytes_read": nbytes, "bytes_written": nbytes, "reps": reps, "gbs": 2 * nbytes / dt / 1e9}


def cpu_model():
    """The host CPU's model name: lscpu's "Model name", else /proc/cpuinfo's
    "model name", else None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def run_cpu_baseline(w, budget_s=12.0, max_steps=4, single_budget_s=10.0):
    """The oracle as it stands, on the host's cores: full-grid RK steps of
    the same workload from phi0, first on min(cores, 16) threads (up to
    max_steps steps or budget_s seconds), then on one thread (steps until
    single_budget_s seconds have passed, at least one)."""
    import numpy as np

    import oracle as O
    from paper_2411_03501_amd import inputs

    Po = O.make_problem(w.gmin, w.gmax, w.n, w.periodic, w.ham, w.params, w.scheme, w.rk, w.cfl)
    phi0 = inputs.initial_surface(w)
    dt = O.cfl_dt(Po)
    tgt = phi0.copy() if w.with_target else None

    def timed(threads, steps_max, budget):
        O.set_threads(threads)
        phi, done = phi0, 0
        t0 = time.perf_counter()
        while True:
            phi = O.step(Po, phi, dt, target=tgt)
            done += 1
            el = time.perf_counter() - t0
            log(f"  oracle on {threads} thread(s), step {done}: {el:.1f} s")
            if el > budget or done >= steps_max:
                break
        assert np.isfinite(phi).all()
        return done, el

    threads = min(os.cpu_count() or 1, 16)
    done, el = timed(threads, max_steps, budget_s)
    done1, el1 = timed(1, max_steps, single_budget_s)
    return {"value": w.points * done / el, "unit": "grid-point updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} RK3 steps of the full {w.name} grid ({w.points} nodes) from phi0, FP64, "
                      f"{threads} threads",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "s_per_rk_step": el / done,
            "single_thread": {"value": w.points * done1 / el1, "unit": "grid-point updates/s", "cores": 1,
                              "s_per_rk_step": el1 / done1,
                              "sample": f"{done1} RK3 step(s) of the full {w.name} grid, FP64, one thread"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="car4d")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--tile", default=None,
                    help="variant,tx,ty,march of the stage kernel instead of the autotuner's choice "
                         "(counter runs: the tuner's timings are distorted under counter collection)")
    ap.add_argument("--only", choices=["batch256", "adjoint", "copy", "normal2d", "first_order_large", "tube",
                                       "rockets", "claw", "local", "godunov_large", "shapes"],
                    help="run one secondary measurement alone and print its JSON (for profiling); "
                         "copy: a plain 1 GiB device copy, the reference for HBM counter calibration")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the solver would shard by slabs with halo exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    from paper_2411_03501_amd import inputs

    if args.only:
        if args.only == "batch256":
            res = run_batch()
        elif args.only == "adjoint":
            res = run_adjoint(inputs.DUBINS3D_81)
        elif args.only == "normal2d":
            res = run_small()
        elif args.only == "first_order_large":
            res = run_first_order_large()
        elif args.only == "shapes":
            res = run_shapes()
        elif args.only == "godunov_large":
            res = run_first_order_large(dissipation="godunov")
        elif args.only == "local":
            res = run_local(inputs.WORKLOADS[args.workload], args.dtype)
        elif args.only == "claw":
            res = run_claw()
        elif args.only == "rockets":
            res = run_rockets()
        elif args.only == "tube":
            res = run_tube(inputs.WORKLOADS[args.workload], args.dtype)
        else:
            res = run_copy()
        print(json.dumps({"only": args.only, **res}), flush=True)
        return

    w = inputs.WORKLOADS[args.workload]
    log(f"bench {w.name} {args.dtype}: {w.points} nodes, K={args.steps} W={args.warmup}")
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    elapsed, st, loop_ms = run_gpu(w, args.dtype, args.steps, args.warmup, tile)
    rk_steps = st["steps"]
    updates = w.points * rk_steps * args.steps
    value = updates / elapsed
    roof = roofline(w, args.dtype, st, loop_ms)

    extra = {}
    if not args.no_extra:
        wd = inputs.DUBINS3D
        for dt_ in ("f32", "f64"):
            if (wd.name, dt_) == (w.name, args.dtype):
                continue
            log(f"secondary: {wd.name} {dt_}")
            e2, st2, lm2 = run_gpu(wd, dt_, 2, 1)
            r2 = roofline(wd, dt_, st2, lm2)
            extra[f"{wd.name}_{dt_}"] = {
                "workload": describe(wd, st2["steps"]) + f", {dt_.upper()}",
                "updates_per_s": wd.points * st2["steps"] * 2 / e2, "stage_kernel_us": r2["kernel_us"],
                "tile": st2["tile"], "alu_frac": r2["frac"] if r2["bound"] == "alu" else None,
                "traffic": r2["traffic"], "hbm_alg_frac": r2.get("hbm_frac")}
            if dt_ == "f32":
                plain32 = r2["kernel_us"]
        if w.name != "car4d":
            w4 = inputs.CAR4D
            log(f"secondary: {w4.name} f32")
            e4, st4, lm4 = run_gpu(w4, "f32", 2, 1)
            r4 = roofline(w4, "f32", st4, lm4)
            extra["car4d_f32"] = {"updates_per_s": w4.points * st4["steps"] * 2 / e4, "rk_steps": st4["steps"],
                                  "stage_kernel_us": r4["kernel_us"], "alu_frac": r4["frac"],
                                  "hbm_alg_frac": r4["hbm_frac"]}
        if w.name == "dubins3d" and args.dtype == "f32":
            plain32 = roof["kernel_us"]

        log(f"tube form: {wd.name} f32 with the clip")
        extra[f"{wd.name}_tube_f32"] = run_tube(wd, "f32", plain_us=plain32)

        log(f"local LF: {wd.name} f32")
        extra[f"{wd.name}_local_lf_f32"] = run_local(wd, "f32", plain_us=plain32)

        log("rockets f32: the paper's own workload")
        extra["rockets_f32"] = run_rockets()

        log("burgers2d f32: the conservation-law scheme")
        extra["burgers2d_f32"] = run_claw()

        log("normal2d f64: launch-bound solve, host-driven vs graph replay")
        extra["normal2d_f64"] = run_small()

        log("first-order f64 at 4096^2: the HBM-bound path")
        extra["normal2d_4096_f64"] = run_first_order_large()

        log("first-order f64 at 4096^2 with Godunov's numerical Hamiltonian")
        extra["normal2d_4096_godunov_f64"] = run_first_order_large(dissipation="godunov")

        log("batch256 initial data on the device")
        extra["batch256_initial_data"] = run_shapes()

        log("batch256 f32: batched vs per-member")
        extra["batch256"] = run_batch()

        log("adjoint: dubins3d_81 f32")
        extra["adjoint"] = run_adjoint(inputs.DUBINS3D_81)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline: oracle")
        cpu = run_cpu_baseline(w)

    line = {
        "metric": "grid-point updates/s per WENO5-RK3 step",
        "adjoint_over_forward": extra.get("adjoint", {}).get("adjoint_over_forward"),
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": describe(w, rk_steps),
                   "nodes": w.points, "rk_steps_per_solve": rk_steps, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


def roofline(w, dtype, st, loop_ms):
    """The stage kernel's roofline record for one workload: its mean launch
    duration from the event-timed stepping loops (the solve's own stream,
    divided by the number of stage launches), the algorithmic operations or
    bytes per launch, and the HBM bytes of the committed counter summary."""
    elem = 4 if dtype == "f32" else 8
    kern_s = (sum(loop_ms) / len(loop_ms)) / 1e3 / (st["steps"] * w.rk)
    ops = alg_ops_per_point(w.scheme, w.ham, w.dim, dtype) * w.points
    achieved_tops = ops / kern_s / 1e12
    bytes_launch = stage_bytes_per_point(w.rk, w.with_target, elem) * w.points
    achieved_gbs = bytes_launch / kern_s / 1e9
    traffic = measured_traffic(w, dtype, st["tile"])
    kernel_name = {1: "stage_direct_kernel", 2: "steps_kernel"}.get(
        st["tile"][0], "stage_tile_kernel" if w.dim >= 3 else "stage_kernel (plane-march)")
    if w.scheme == "weno5":
        return {"bound": "alu", "achieved": achieved_tops, "peak": PEAK_VALU_TOPS, "unit": "Tops/s",
                "frac": achieved_tops / PEAK_VALU_TOPS, "traffic": traffic,
                "kernel": kernel_name, "kernel_us": kern_s * 1e6, "tile": st["tile"],
                "ops_per_launch": ops, "bytes_per_launch": bytes_launch,
                "hbm_alg_gbs": achieved_gbs, "hbm_frac": achieved_gbs / PEAK_HBM_GBS}
    return {"bound": "hbm", "achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved_gbs / PEAK_HBM_GBS, "traffic": traffic,
            "kernel": kernel_name, "kernel_us": kern_s * 1e6, "tile": st["tile"], "bytes_per_launch": bytes_launch}


if __name__ == "__main__":
    main()
