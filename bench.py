#!/usr/bin/env python3
"""Throughput of the fused unsplit acoustics step on one MI355X.

Workload (the bandwidth-roofline configuration): one 2048x2048 patch, rho=1,
K=4, radial ring pulse, extrapolation boundaries, MC limiter, FP64; every step
is one persistent level launch plus the device-side Courant-number reduction
and dt update (CFL 0.9), the whole step loop captured as one hipGraph.  A
"step" is one pass of that whole hot path over the grid.

Printed as ONE JSON line.  Extra objects: the FP32 variant of the same run,
the synthetic AMR level batch (batched persistent launch vs one launch per
patch, FP64 and FP32), the 64-instance ensemble (graph vs eager, default vs
autotuned tiling), the 512^2 adjoint run (forward, backward, adjoint step),
conservation sums, the roofline of the step kernel and the
oracle's throughput on the host cores (cpu_baseline).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# The paper's own headline (context only, not comparable: whole AMR runs of
# its acoustics benchmark on 2013-2016 NVIDIA GPUs against a 16-core CPU).
PAPER_CONTEXT = {
    "total_runtime_speedup": "2-3x (at most 2.7x), one GPU against 16 CPU cores running "
                             "the original Clawpack AMR code",
    "hardware": ["NVIDIA K20x against 16 AMD Opteron 6274 cores at 2.2 GHz",
                 "NVIDIA P100 (host Intel Xeon E5-2698, 16 threads) against 16 Intel Xeon "
                 "cores at 2.0 GHz"],
    "advance_step_speedup": "3.0x (K20x) and 3.8x (P100) for the advance-and-save-fluxes "
                            "section that holds this path",
    "precision": "FP64", "source": "abstract, Sec. 4.2, Sec. 5"}
METRIC = "Gcell-updates/s and % HBM peak, batched-AMR vs per-patch launch, FP64 1e-12"
RHO, K_BULK = 1.0, 4.0
C_SOUND = math.sqrt(K_BULK / RHO)


def algorithmic_bytes(shapes, elem_bytes, physical_bc):
    """Bytes one step must move: every padded cell read once, every interior
    cell written once, and on physical boundaries the ghost ring written."""
    total = 0
    for mx, my in shapes:
        padded = (mx + 4) * (my + 4)
        total += 3 * elem_bytes * (padded + mx * my)
        if physical_bc:
            total += 3 * elem_bytes * (padded - mx * my)
    return total


def device_finite(torch, lev):
    """Every cell of every patch of the level's current state is finite,
    checked on the device (ghost cells included, row padding excluded)."""
    pool = lev.pools[lev.current_pool()].view(lev.dtype)
    torch.cuda.synchronize()
    return all(bool(torch.isfinite(lev.patch_view(pool, k)).all()) for k in range(lev.n))


def rel_linf(q, ref):
    """Per component (p, u, v): max |q - ref| / max |ref| (a component whose
    reference is zero is divided by the largest magnitude of all three)."""
    import numpy as np

    q = np.asarray(q, np.float64)
    ref = np.asarray(ref, np.float64)
    allmax = float(np.abs(ref).max()) or 1.0
    out = []
    for m in range(3):
        s = float(np.abs(ref[m]).max())
        out.append(float(np.abs(q[m] - ref[m]).max()) / (s if s > 0 else allmax))
    return out


def run_uniform(ws, torch, n, steps, warmup, dtype, kernel_launches, tune=True, limiter="mc",
                transverse_corr=False, keep_state=False):
    import workloads

    dx = 1.0 / n
    q0 = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    lev = ws.Level([dict(mx=n, my=n, dx=dx, dy=dx, bc="extrap")], [(RHO, K_BULK)], dtype=dtype,
                   limiter=limiter, transverse_corr=transverse_corr)
    dt0 = 0.9 * dx / C_SOUND

    def reset():
        lev.upload(0, q0)
        lev.fill_ghosts()
        lev.set_dt([dt0])

    reset()
    if tune:
        # tile shapes picked by the library's autotuner (timing only; the
        # state is restored, and results do not depend on the tiling)
        from paper_1808_02638_amd.autotune import autotune
        autotune(lev)  # cached per GPU architecture, library build and shape
    var, tw, th, wg, grid = lev.get_tiling()
    tiling = {"variant": var[0], "tile_w": int(tw[0]), "tile_h": int(th[0]),
              "wg_per_cu": wg, "grid": grid}
    reset()
    for _ in range(warmup):
        lev.step_auto(0.9)
    torch.cuda.synchronize()
    reset()
    lev.capture(steps, 0.9)
    sums0 = lev.conservation_sums()[0]
    stream = lev.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    lev.graph_launch()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    sums1 = lev.conservation_sums()[0]
    _dt, cfl_last, cfl_max = lev.read_dt_cfl()
    q = lev.download(0)
    finite = bool(torch.isfinite(torch.from_numpy(q)).all())
    # each step launch bracketed by its own HIP event pair (reported for
    # reference; the pairs add their own overhead to every launch)
    kernel_ms = lev.time_step_kernel(kernel_launches)
    lev.close()
    return dict(ms=ms, wall_s=wall, sums0=sums0.tolist(), sums1=sums1.tolist(),
                cfl_last=float(cfl_last[0]), cfl_max=float(cfl_max[0]), finite=finite,
                kernel_ms=kernel_ms, tiling=tiling, q=q if keep_state else None)


def run_medium(ws, torch, n=2048, steps=200, warmup=10, tune=True):
    """The 2048^2 FP64 pulse in a heterogeneous medium (three layers, +-10%
    cell perturbation): DIRECT tiles of the variable-coefficient kernel,
    CFL 0.9 from the device reduction over the cells, steps in one hipGraph."""
    import numpy as np

    import workloads

    dx = 1.0 / n
    rho, K = workloads.layered_medium(n, n)
    lev = ws.Level([dict(mx=n, my=n, dx=dx, dy=dx, bc="extrap")], [(RHO, K_BULK)])
    lev.set_medium(0, rho, K)
    q0 = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    dt0 = 0.9 * dx / float(np.sqrt(K / rho).max())

    def reset():
        lev.upload(0, q0)
        lev.fill_ghosts()
        lev.set_dt([dt0])

    reset()
    if tune:
        from paper_1808_02638_amd.autotune import autotune
        autotune(lev)
    var, tw, th, wg, grid = lev.get_tiling()
    reset()
    for _ in range(warmup):
        lev.step_auto(0.9)
    reset()
    lev.capture(steps, 0.9)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(lev.stream)
    lev.graph_launch()
    e1.record(lev.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _dt, cfl_last, cfl_max = lev.read_dt_cfl()
    finite = bool(np.isfinite(lev.download(0)).all())
    lev.close()
    padded = (n + 4) * (n + 4)
    nbytes = algorithmic_bytes([(n, n)], 8, True) + 2 * 8 * padded  # plus c, Z read once
    kms = ms / steps
    return {"grid": f"{n}x{n}", "steps": steps, "value": round(n * n * steps / (ms / 1e3) / 1e9, 3),
            "kernel_ms": kms, "bytes_per_launch": nbytes,
            "kernel_GBs": round(nbytes / (kms / 1e3) / 1e9, 1),
            "frac": round(nbytes / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "tiling": {"variant": var[0], "tile_w": int(tw[0]), "tile_h": int(th[0]),
                       "wg_per_cu": wg},
            "cfl_max": float(cfl_max[0]), "finite": finite}


def run_tiled(ws, torch, n=2048, tiles=4, steps=200, warmup=10, tune=True):
    """The 2048^2 FP64 pulse with extrapolating sides cut into tiles x tiles
    patches that exchange ghosts after every step (a tiled coarsest level);
    CFL 0.9 from the device reduction, steps in one hipGraph.  Compared with
    the single-patch leg this prices the exchange."""
    import numpy as np

    import workloads

    dx = 1.0 / n
    w = n // tiles
    shapes = [(w, w)] * (tiles * tiles)
    origins = [(w * a, w * b) for b in range(tiles) for a in range(tiles)]
    lev = ws.Level([dict(mx=w, my=w, dx=dx, dy=dx) for _ in shapes], [(RHO, K_BULK)])
    lev.link(origins, (n, n), (False, False))
    q0 = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    parts = [np.ascontiguousarray(q0[:, y0:y0 + w + 4, x0:x0 + w + 4]) for (x0, y0) in origins]
    dt0 = 0.9 * dx / C_SOUND

    def reset():
        for k, q in enumerate(parts):
            lev.upload(k, q)
        lev.fill_ghosts()
        lev.set_dt([dt0])

    reset()
    if tune:
        from paper_1808_02638_amd.autotune import autotune
        autotune(lev)
    var, tw, th, wg, grid = lev.get_tiling()
    reset()
    for _ in range(warmup):
        lev.step_auto(0.9)
    reset()
    lev.capture(steps, 0.9)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(lev.stream)
    lev.graph_launch()
    e1.record(lev.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    _dt, _cl, cfl_max = lev.read_dt_cfl()
    finite = all(bool(np.isfinite(lev.download(k)).all()) for k in range(len(shapes)))
    lev.close()
    ghosts = len(shapes) * (4 * (w + 4) + 4 * w)
    return {"domain": f"{n}x{n}", "tiles": f"{tiles}x{tiles} of {w}x{w}", "steps": steps,
            "value": round(n * n * steps / (ms / 1e3) / 1e9, 3),
            "us_per_step": round(ms / steps * 1e3, 2),
            "exchange_bytes_per_step": ghosts * (2 * 3 * 8 + 16),
            "tiling": {"variant": var[0], "tile_w": int(tw[0]), "tile_h": int(th[0]),
                       "wg_per_cu": wg},
            "cfl_max": float(cfl_max[0]), "finite": finite}


def run_amr(ws, torch, dtype, level_steps, tune=True):
    import workloads

    levels = workloads.amr_level_batch()
    out = {"levels": [], "n_patches": sum(len(l) for l in levels)}
    tot_cells = tot_bytes = 0
    tb = tp = 0.0
    for specs in levels:
        lev = ws.Level([dict(mx=p.mx, my=p.my, dx=p.dx, dy=p.dy) for p in specs], [(RHO, K_BULK)],
                       dtype=dtype)
        for k, p in enumerate(specs):
            lev.upload(k, workloads.padded_state(p.mx, p.my, p.xlo, p.ylo, p.dx, p.dy))
        lev.set_dt([0.9 * specs[0].dx / C_SOUND])
        # the per-patch baseline: one launch per patch of the library's
        # default tiles (a PACKED tile holds several patches, so per-patch
        # launches take the default tiling)
        lev.time_step_kernel(2, per_patch=True)
        ms_p = lev.time_step_kernel(level_steps, per_patch=True)
        if tune:
            from paper_1808_02638_amd.autotune import autotune
            autotune(lev)
        lev.time_step_kernel(2)
        ms_br = lev.time_step_kernel(level_steps)
        tuned_vars = sorted(set(lev.get_tiling()[0]))
        # the batched level steps as one captured graph (level_steps launches,
        # the Courant number filed inside each), so no per-launch event pair
        # or host call enters the time; the per-patch baseline is one launch
        # per patch from the host, as such a code runs
        steps_g = level_steps + level_steps % 2
        lev.capture(steps_g, 0.9)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        lev.graph_launch()
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            e0.record(lev.stream)
            lev.graph_launch()
            e1.record(lev.stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / steps_g)
        ms_b = sorted(times)[len(times) // 2]
        cells = sum(p.mx * p.my for p in specs)
        nbytes = algorithmic_bytes([(p.mx, p.my) for p in specs], dtype.itemsize, False)
        tot_cells += cells
        tot_bytes += nbytes
        tb += ms_b
        tp += ms_p
        out["levels"].append(dict(patches=len(specs), cells=cells,
                                  batched_gcells=round(cells / ms_b / 1e6, 3),
                                  batched_us=round(ms_b * 1e3, 2),
                                  batched_bracketed_us=round(ms_br * 1e3, 2),
                                  frac=round(nbytes / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                  tile_variants=tuned_vars,
                                  per_patch_gcells=round(cells / ms_p / 1e6, 3)))
        lev.close()
    out["batched_gcells"] = tot_cells / tb / 1e6
    out["batched_frac"] = round(tot_bytes / (tb / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    out["per_patch_gcells"] = tot_cells / tp / 1e6
    out["speedup"] = tp / tb
    out["cells_per_level_step"] = tot_cells
    return out


def run_ensemble(ws, torch, steps, tune=True):
    """64 independent instances of uneven sizes in one level: default vs
    autotuned tiling (step kernel alone), then the steps eager (one launch per
    step from the host) and as one captured graph, FP64, per-instance dt."""
    import workloads

    insts = workloads.ensemble()
    lev = ws.Level([dict(mx=e.mx, my=e.my, dx=e.dx, dy=e.dy, instance=k, bc="extrap")
                    for k, e in enumerate(insts)], [(e.rho, e.K) for e in insts])
    dt0 = [0.9 * min(e.dx, e.dy) / math.sqrt(e.K / e.rho) for e in insts]
    cells = sum(e.mx * e.my for e in insts)

    def reset():
        for k, e in enumerate(insts):
            lev.upload(k, e.state())
        lev.fill_ghosts()
        lev.set_dt(dt0)

    reset()
    lev.time_step_kernel(2)
    default_ms = lev.time_step_kernel(20)
    if tune:
        from paper_1808_02638_amd.autotune import autotune
        autotune(lev)
    lev.time_step_kernel(2)
    tuned_ms = lev.time_step_kernel(20)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reset()
    torch.cuda.synchronize()
    e0.record(lev.stream)
    for _ in range(steps):
        lev.step_auto(0.9)
    e1.record(lev.stream)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1)
    reset()
    lev.capture(steps, 0.9)
    torch.cuda.synchronize()
    e0.record(lev.stream)
    lev.graph_launch()
    e1.record(lev.stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1)
    _dt, cfl_last, _ = lev.read_dt_cfl()
    var, _tw, _th, wg, grid = lev.get_tiling()
    lev.close()
    nbytes = algorithmic_bytes([(e.mx, e.my) for e in insts], 8, True)
    return {"instances": len(insts), "cells": cells, "steps": steps,
            "bytes_per_step": nbytes,
            "frac": round(nbytes / (graph_ms / steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "graph_gcells": round(cells * steps / graph_ms / 1e6, 3),
            "eager_gcells": round(cells * steps / eager_ms / 1e6, 3),
            "graph_us_per_step": round(graph_ms * 1e3 / steps, 2),
            "eager_us_per_step": round(eager_ms * 1e3 / steps, 2),
            "default_tiling_kernel_us": round(default_ms * 1e3, 2),
            "tuned_tiling_kernel_us": round(tuned_ms * 1e3, 2),
            "tuned_variants": {v: var.count(v) for v in sorted(set(var))},
            "cfl_last_min_max": [float(cfl_last.min()), float(cfl_last.max())]}


def run_adjoint(ws, torch):
    """The adjoint workload: 512^2 FP64, 200 fixed-dt steps at Courant 0.8, 16
    receivers, checkpoints every 20 steps: forward traces and the backward
    sweep (re-run forward segments recording the branches, then the adjoint
    steps), and the adjoint step kernel alone; then the same with every
    step's branches recorded in the forward pass (no re-run)."""
    import numpy as np

    import workloads

    setup = workloads.adjoint_setup()
    n, steps = setup.n, setup.steps
    run = ws.AcousticsAdjoint(n, n, setup.dx, setup.dx, RHO, K_BULK, setup.receivers, steps,
                              setup.dt, checkpoint_every=setup.checkpoint_every)
    target = torch.zeros((steps, len(setup.receivers)), dtype=torch.float64, device="cuda")
    p0 = torch.tensor(setup.p0(), device="cuda", requires_grad=True)
    for _ in range(2):  # warm
        p0.grad = None
        run.misfit(p0, target).backward()
    torch.cuda.synchronize()
    p0.grad = None
    t0 = time.perf_counter()
    loss = run.misfit(p0, target)  # the same torch ops as the warm-up runs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad_ok = bool(torch.isfinite(p0.grad).all())
    grad_ckpt = p0.grad.detach().clone()
    # the adjoint step alone: lam' -> S^T lam' on the recorded branches
    lev = run.level
    masks = lev.new_masks()
    lev.step_record_masks(setup.dt, masks)
    a, b = lev.new_buffer(), lev.new_buffer()
    lev.patch_view(a, 0)[:, 2:-2, 2:-2] = torch.from_numpy(
        np.random.default_rng(1).normal(size=(3, n, n))).cuda()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 100
    # captured as one graph, so the host's per-call cost stays out of the timing
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(lev.stream):
        lev.adjoint_step(setup.dt, masks, a, b)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=lev.stream):
            for r in range(reps):
                lev.adjoint_step(setup.dt, masks, a, b) if r % 2 == 0 else \
                    lev.adjoint_step(setup.dt, masks, b, a)
        graph.replay()
        e0.record(lev.stream)
        graph.replay()
        e1.record(lev.stream)
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / reps
    byts = n * n * (48 + 1)  # lam in, lam out (3 FP64 each), one mask byte per cell
    run.close()
    # every step's branches recorded in the forward pass instead of the
    # checkpoints: the backward pass runs only the adjoint steps
    runb = ws.AcousticsAdjoint(n, n, setup.dx, setup.dx, RHO, K_BULK, setup.receivers, steps,
                               setup.dt, checkpoint_every=setup.checkpoint_every,
                               store_branches=True)
    for _ in range(2):  # warm
        p0.grad = None
        runb.misfit(p0, target).backward()
    torch.cuda.synchronize()
    p0.grad = None
    t3 = time.perf_counter()
    loss = runb.misfit(p0, target)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    same = bool(torch.equal(p0.grad, grad_ckpt))
    runb.close()
    return {"grid": f"{n}x{n}", "steps": steps, "checkpoint_every": setup.checkpoint_every,
            "forward_ms": round((t1 - t0) * 1e3, 3), "backward_ms": round((t2 - t1) * 1e3, 3),
            "adjoint_step_us": round(adj_ms * 1e3, 2),
            "adjoint_step_gcells": round(n * n / adj_ms / 1e6, 2),
            "adjoint_step_GBs": round(byts / (adj_ms / 1e3) / 1e9, 1), "grad_finite": grad_ok,
            "stored_branches": {"forward_ms": round((t4 - t3) * 1e3, 3),
                                "backward_ms": round((t5 - t4) * 1e3, 3),
                                "branch_bytes": steps * n * n, "grad_equal": same}}


PROFILE = os.path.join(ROOT, "profiles", "step_kernel_march_f64_2048sq.md")


def run_two_level(ws, torch, steps=20, warmup=3, r=4, n=1024, tune=True):
    """Composite coarse steps of a 1024^2 coarse grid and 364 ratio-4 fine
    patches of 120^2 cells over the ring's annulus (coarse step, r fine steps
    with ghosts from the coarse level, updating, conservation fix), against
    the same level steps without the coupling kernels."""
    import numpy as np

    import workloads

    rects = workloads.two_level_layout(n)
    dx = 1.0 / n
    coarse = ws.Level([dict(mx=n, my=n, dx=dx, dy=dx, bc="extrap")], [(RHO, K_BULK)])
    fine = ws.Level([dict(mx=r * w, my=r * h, dx=dx / r, dy=dx / r) for (_, _, w, h) in rects],
                    [(RHO, K_BULK)], stream=coarse.stream)
    coarse.upload(0, workloads.padded_state(n, n, 0.0, 0.0, dx, dx))
    coarse.fill_ghosts()
    for k, (ci0, cj0, w, h) in enumerate(rects):
        fine.upload(k, workloads.padded_state(r * w, r * h, ci0 * dx, cj0 * dx, dx / r, dx / r))
    tl = ws.TwoLevel(coarse, fine, r, [(0, ci0, cj0) for (ci0, cj0, _, _) in rects])
    dt = 0.9 * dx / C_SOUND
    stream = coarse.stream
    if tune:
        from paper_1808_02638_amd.autotune import autotune
        for lev in (coarse, fine):
            autotune(lev)  # timing only: the state is restored and results do not change

    def timed(fn, count):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(count):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / count

    for _ in range(warmup):
        tl.step(dt)
    ms = timed(lambda: tl.step(dt), steps)
    # the composite result (before the uncoupled timing rounds below)
    finite = device_finite(torch, coarse) and device_finite(torch, fine)

    def levels_only():
        coarse.step(dt, read_cfl=False)
        for _ in range(r):
            fine.step(dt / r, read_cfl=False)

    ms_levels = timed(levels_only, steps)
    tilings = [lev.get_tiling() for lev in (coarse, fine)]
    fine_cells = sum(r * w * r * h for (_, _, w, h) in rects)
    updates = n * n + r * fine_cells
    nbytes = (algorithmic_bytes([(n, n)], 8, True)
              + r * algorithmic_bytes([(r * w, r * h) for (_, _, w, h) in rects], 8, False))
    tl.close()
    fine.close()
    coarse.close()
    return {"coarse": f"{n}x{n}", "ratio": r, "fine_patches": len(rects),
            "fine_cells": fine_cells, "cell_updates_per_step": updates, "steps": steps,
            "ms_per_composite_step": ms, "gcells": round(updates / (ms / 1e3) / 1e9, 3),
            "levels_only_ms": ms_levels,
            "coupling_overhead": round(ms / ms_levels - 1.0, 4),
            "tilings": [{"variant": t[0][0], "tile_w": int(t[1][0]), "tile_h": int(t[2][0]),
                         "wg_per_cu": t[3]} for t in tilings],
            "GBs": round(nbytes / (ms / 1e3) / 1e9, 1),
            "frac": round(nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "finite": finite}


def run_three_level(ws, torch, steps=10, warmup=2, r=4, n=512, tune=True):
    """Composite steps of three levels: 512^2, 103 ratio-4 level-1 patches of
    120^2 over the annulus, 409 ratio-4 level-2 patches of 120^2 inside them
    near the ring (level 2 takes 16 steps per level-0 step)."""
    import numpy as np

    import workloads

    l1, l2 = workloads.three_level_layout(n)
    dx0, dx1, dx2 = 1.0 / n, 1.0 / (n * r), 1.0 / (n * r * r)
    lev0 = ws.Level([dict(mx=n, my=n, dx=dx0, dy=dx0, bc="extrap")], [(RHO, K_BULK)])
    lev1 = ws.Level([dict(mx=r * w, my=r * h, dx=dx1, dy=dx1) for (_, _, w, h) in l1],
                    [(RHO, K_BULK)], stream=lev0.stream)
    lev2 = ws.Level([dict(mx=r * w, my=r * h, dx=dx2, dy=dx2) for (_, _, _, w, h) in l2],
                    [(RHO, K_BULK)], stream=lev0.stream)
    lev0.upload(0, workloads.padded_state(n, n, 0.0, 0.0, dx0, dx0))
    lev0.fill_ghosts()
    for k, (ci0, cj0, w, h) in enumerate(l1):
        lev1.upload(k, workloads.padded_state(r * w, r * h, ci0 * dx0, cj0 * dx0, dx1, dx1))
    for k, (p, a0, b0, w, h) in enumerate(l2):
        x0, y0 = l1[p][0] * dx0 + a0 * dx1, l1[p][1] * dx0 + b0 * dx1
        lev2.upload(k, workloads.padded_state(r * w, r * h, x0, y0, dx2, dx2))
    hier = ws.Hierarchy([lev0, lev1, lev2], r,
                        [[(0, ci0, cj0) for (ci0, cj0, _, _) in l1],
                         [(p, a0, b0) for (p, a0, b0, _, _) in l2]])
    dt = 0.9 * dx0 / C_SOUND
    stream = lev0.stream
    if tune:
        from paper_1808_02638_amd.autotune import autotune
        for lev in (lev0, lev1, lev2):
            autotune(lev)
    for _ in range(warmup):
        hier.step(dt)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        hier.step(dt)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    finite = all(device_finite(torch, L) for L in (lev0, lev1, lev2))
    c1 = sum(r * w * r * h for (_, _, w, h) in l1)
    c2 = sum(r * w * r * h for (_, _, _, w, h) in l2)
    updates = n * n + r * c1 + r * r * c2
    nbytes = (algorithmic_bytes([(n, n)], 8, True)
              + r * algorithmic_bytes([(r * w, r * h) for (_, _, w, h) in l1], 8, False)
              + r * r * algorithmic_bytes([(r * w, r * h) for (_, _, _, w, h) in l2], 8, False))
    hier.close()
    for lev in (lev2, lev1, lev0):
        lev.close()
    return {"levels": [f"{n}x{n}", f"{len(l1)} patches, {c1} cells",
                       f"{len(l2)} patches, {c2} cells"], "ratio": r, "steps": steps,
            "cell_updates_per_step": updates, "ms_per_composite_step": ms,
            "gcells": round(updates / (ms / 1e3) / 1e9, 3),
            "GBs": round(nbytes / (ms / 1e3) / 1e9, 1),
            "frac": round(nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "finite": finite}


STEP_KERNEL_SOURCES = ("ws_kernels.hip", "ws_device.h", "ws_internal.h", "ws_tables.h")


def step_kernel_sha1():
    """SHA-1 of the step kernel's sources (the kernel file and the three
    headers it includes from the library), in that order."""
    import hashlib

    h = hashlib.sha1()
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1808_02638_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(tiling, profile=PROFILE, n=2048):
    """HBM bytes per launch of the FP64 step kernel on the n x n grid (2048 or
    4096) from the committed counter summary, or None when the step kernel's
    sources have changed since the counters were taken or the tiling differs
    from the one they were taken with."""
    try:
        text = open(profile).read()
    except OSError:
        return None
    sfx = "" if n == 2048 else f"_{n}"
    keys = ("kernel_source_sha1", f"traffic{sfx}_bytes_per_launch", f"tiling{sfx}")
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.split(": ", 1)[0] in keys)
    if fields.get("kernel_source_sha1", "").strip() != step_kernel_sha1():
        return None
    if fields.get(keys[2], "").strip() != f"{tiling['variant']}/{tiling['tile_w']}/{tiling['tile_h']}":
        return None
    return int(fields[keys[1]]) if keys[1] in fields else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, target_s):
    """The oracle on the host cores: steps of the n x n FP64 grid for about
    target_s seconds with every thread the process may use, then a short
    single-threaded sample (the oracle's OpenMP loops over rows)."""
    import oracle
    import workloads

    dx = 1.0 / n
    q = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    oracle.fill_bc(q, "extrap")
    dt = 0.9 * dx / C_SOUND
    t = time.perf_counter()
    q1, _, _ = oracle.step(q, dx, dx, dt, RHO, K_BULK, "mc")
    one = time.perf_counter() - t
    steps = max(1, int(target_s / max(one, 1e-3)))
    t = time.perf_counter()
    for _ in range(steps):
        q1, _, _ = oracle.step(q1, dx, dx, dt, RHO, K_BULK, "mc")
        oracle.fill_bc(q1, "extrap")
    el = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    # one thread: a single step (the process-wide OpenMP setting is left alone)
    t = time.perf_counter()
    oracle.step(q1, dx, dx, dt, RHO, K_BULK, "mc", parallel=False)
    el1 = time.perf_counter() - t
    return {"value": n * n * steps / el / 1e9, "unit": "Gcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} oracle steps of the {n}x{n} FP64 grid ({el:.1f} s, OpenMP "
                      f"over {threads} threads)",
            "single_thread_value": n * n / el1 / 1e9, "cpu_model": cpu_model()}


def cpu_baseline_workloads():
    """The oracle on the host cores for the other workloads, each on a bounded
    sample (a few seconds): the 128^2 patch over its 100 steps, one level step
    of each level of the AMR level batch, one step of the 64-instance
    ensemble, and 20 forward plus 20 adjoint steps of the 512^2 adjoint run."""
    import math as _m

    import numpy as np

    import oracle
    import workloads

    out = {}
    n = 128
    dx = 1.0 / n
    q = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    oracle.fill_bc(q, "extrap")
    t = time.perf_counter()
    oracle.run(q, 100, dx, dx, RHO, K_BULK, limiter="mc", bc="extrap", cfl_desired=0.9)
    el = time.perf_counter() - t
    out["patch_128_fp64"] = {"value": n * n * 100 / el / 1e9, "sample": "all 100 steps",
                             "seconds": round(el, 3)}
    levels = workloads.amr_level_batch()
    cells, el = 0, 0.0
    for specs in levels:
        states = [workloads.padded_state(p.mx, p.my, p.xlo, p.ylo, p.dx, p.dy) for p in specs]
        t = time.perf_counter()
        oracle.step_patches(states, [p.dx for p in specs], [p.dy for p in specs],
                            [0.9 * specs[0].dx / C_SOUND] * len(specs), RHO, K_BULK)
        el += time.perf_counter() - t
        cells += sum(p.mx * p.my for p in specs)
    out["amr_level_batch_fp64"] = {"value": cells / el / 1e9,
                                   "sample": "one level step of each of the three levels",
                                   "seconds": round(el, 3)}
    insts = workloads.ensemble()
    states = [e.state() for e in insts]
    dts = [0.9 * min(e.dx, e.dy) / _m.sqrt(e.K / e.rho) for e in insts]
    t = time.perf_counter()
    oracle.step_patches(states, [e.dx for e in insts], [e.dy for e in insts], dts,
                        [e.rho for e in insts], [e.K for e in insts])
    el = time.perf_counter() - t
    out["ensemble_fp64"] = {"value": sum(e.mx * e.my for e in insts) / el / 1e9,
                            "sample": "one step of all 64 instances", "seconds": round(el, 3)}
    setup = workloads.adjoint_setup()
    ns, k = setup.n, 20
    t = time.perf_counter()
    _J, _tr, states, masks = oracle.forward_traces(setup.p0(), k, setup.dx, setup.dx, setup.dt,
                                                   RHO, K_BULK, setup.receivers)
    lam = np.zeros((3, ns, ns))
    lam[0, ns // 2, ns // 2] = 1.0
    for s in range(k - 1, -1, -1):
        lam = oracle.adjoint_step(lam, states[s], setup.dx, setup.dx, setup.dt, RHO, K_BULK,
                                  masks[s])
    el = time.perf_counter() - t
    out["adjoint_512_fp64"] = {"value": 2 * k * ns * ns / el / 1e9,
                               "sample": f"{k} forward steps recording the branches, then "
                                         f"{k} adjoint steps (cell updates of both)",
                               "seconds": round(el, 3)}
    for v in out.values():
        v["value"] = round(v["value"], 5)
        v["unit"] = "Gcell-updates/s"
    return out


def copy_bandwidth(torch, nbytes):
    """A plain device copy of nbytes (read + write), the practical reference
    for the step's traffic."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        dst.copy_(src)
    times = []
    for _ in range(10):
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    return {"bytes_each_way": nbytes, "GBs": round(2 * nbytes / (ms / 1e3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--kernel-launches", type=int, default=200)
    ap.add_argument("--amr-steps", type=int, default=10)
    ap.add_argument("--ensemble-steps", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true", help="skip FP32, AMR and CPU legs")
    ap.add_argument("--no-tune", action="store_true", help="time the default tiling")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--medium-only", action="store_true",
                    help="only run the heterogeneous-medium leg (for profiling)")
    ap.add_argument("--tiled-only", action="store_true",
                    help="only run the tiled-level leg (for profiling)")
    ap.add_argument("--levels-only", action="store_true",
                    help="only run the two- and three-level composite legs (for profiling)")
    ap.add_argument("--leg", choices=("fp32", "amr", "ensemble", "adjoint", "uniform_4096"),
                    help="only run this extra leg and print its object (for profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(the level step is benchmarked at its single-GPU shape)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1808_02638_amd as ws

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
        # calibrate the step kernel's counter readings
        src = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.medium_only:
        print(json.dumps({"medium_fp64": run_medium(ws, torch, tune=not args.no_tune)}),
              flush=True)
        return
    if args.tiled_only:
        print(json.dumps({"tiled_fp64": run_tiled(ws, torch, tune=not args.no_tune)}), flush=True)
        return
    if args.levels_only:
        print(json.dumps({"two_level_fp64": run_two_level(ws, torch, tune=not args.no_tune),
                          "three_level_fp64": run_three_level(ws, torch, tune=not args.no_tune)}),
              flush=True)
        return
    if args.leg:
        tune = not args.no_tune
        if args.leg in ("fp32", "uniform_4096"):
            big = args.leg == "uniform_4096"
            nn, kk = (4096, min(args.steps, 100)) if big else (args.n, args.steps)
            dt_ = torch.float64 if big else torch.float32
            r = run_uniform(ws, torch, nn, kk, args.warmup, dt_, 20, tune=tune)
            eb = 8 if big else 4
            out = {"n": nn, "steps": kk, "value": round(nn * nn * kk / (r["ms"] / 1e3) / 1e9, 3),
                   "kernel_ms": r["ms"] / kk, "tiling": r["tiling"], "finite": r["finite"],
                   "frac": round(algorithmic_bytes([(nn, nn)], eb, True) / (r["ms"] / kk / 1e3)
                                 / 1e9 / HBM_PEAK_GBS, 4)}
        elif args.leg == "amr":
            out = run_amr(ws, torch, torch.float64, args.amr_steps, tune=tune)
        elif args.leg == "ensemble":
            out = run_ensemble(ws, torch, args.ensemble_steps, tune=tune)
        else:
            out = run_adjoint(ws, torch)
        print(json.dumps({args.leg: out}), flush=True)
        return
    n, K = args.n, args.steps
    shapes = [(n, n)]
    r64 = run_uniform(ws, torch, n, K, args.warmup, torch.float64, args.kernel_launches,
                      tune=not args.no_tune, keep_state=not args.no_extras)
    value = n * n * K / (r64["ms"] / 1e3) / 1e9
    bytes64 = algorithmic_bytes(shapes, 8, True)
    # the timed region is K launches of the step kernel and nothing else (the
    # Courant-number reduction and dt update run inside it): its HIP-event
    # time over K is the kernel's average launch duration
    kernel_ms = r64["ms"] / K
    achieved = bytes64 / (kernel_ms / 1e3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"uniform {n}x{n} 2D acoustics, radial ring pulse, rho=1 K=4, "
                               f"extrapolation BCs, MC limiter, CFL 0.9 with the device "
                               f"max-speed reduction and dt update every step, {K} steps "
                               f"in one hipGraph",
                   "cells": n * n, "global_batch": 1, "parallelism": "single GPU",
                   "tiling": r64["tiling"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(r64["tiling"]) if n == 2048 else None,
                     "kernel": "step_kernel_march<double, MC>",
                     "bytes_per_launch": bytes64, "kernel_ms": kernel_ms,
                     "kernel_ms_bracketed": r64["kernel_ms"]},
        "pct_hbm_peak": round(100 * achieved / HBM_PEAK_GBS, 2),
        "conservation_fp64": {"start": r64["sums0"], "end": r64["sums1"]},
        "cfl_max": r64["cfl_max"],
        "finite": r64["finite"],
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_extras:
        r32 = run_uniform(ws, torch, n, K, args.warmup, torch.float32, args.kernel_launches,
                          tune=not args.no_tune, keep_state=True)
        b32 = algorithmic_bytes(shapes, 4, True)
        a32 = b32 / (r32["ms"] / K / 1e3) / 1e9
        # the FP32 result of the same K steps against the FP64 one (which the
        # tests hold to the FP64 oracle at 1e-12, so this is the FP32 error
        # against the oracle to that accuracy), per component p, u, v
        err32 = rel_linf(r32["q"], r64["q"])
        r64["q"] = r32["q"] = None
        line["fp32"] = {"value": round(n * n * K / (r32["ms"] / 1e3) / 1e9, 3),
                        "tiling": r32["tiling"],
                        "ms_per_step": r32["ms"] / K,
                        "kernel_GBs": round(a32, 1), "frac": round(a32 / HBM_PEAK_GBS, 4),
                        "rel_linf_vs_fp64": [float(f"{e:.3e}") for e in err32],
                        "within_1e-5": bool(max(err32) <= 1e-5), "finite": r32["finite"]}
        # the paper's own limiter, and the variant that also splits the limited
        # correction transversely, on the same workload
        for key, lim, tc in (("vanleer_fp64", "vanleer", False),
                             ("transverse_corr_fp64", "mc", True)):
            rv = run_uniform(ws, torch, n, K, args.warmup, torch.float64, 20,
                             tune=not args.no_tune, limiter=lim, transverse_corr=tc)
            av = bytes64 / (rv["ms"] / K / 1e3) / 1e9
            line[key] = {"value": round(n * n * K / (rv["ms"] / 1e3) / 1e9, 3),
                         "tiling": rv["tiling"], "kernel_ms": rv["ms"] / K,
                         "kernel_GBs": round(av, 1), "frac": round(av / HBM_PEAK_GBS, 4),
                         "cfl_max": rv["cfl_max"], "finite": rv["finite"]}
        line["amr_level_batch"] = {
            "fp64": run_amr(ws, torch, torch.float64, args.amr_steps, tune=not args.no_tune),
            "fp32": run_amr(ws, torch, torch.float32, args.amr_steps, tune=not args.no_tune)}
        # the same workload on a 4096^2 grid: its 806 MB ping-pong set does not
        # fit the 256 MB Infinity Cache (a cache-free check of the roofline)
        big = 4096
        rb = run_uniform(ws, torch, big, 100, 5, torch.float64, 20, tune=not args.no_tune)
        bb = algorithmic_bytes([(big, big)], 8, True)
        line["uniform_4096_fp64"] = {
            "value": round(big * big * 100 / (rb["ms"] / 1e3) / 1e9, 3), "steps": 100,
            "kernel_ms": rb["ms"] / 100,
            "frac": round(bb / (rb["ms"] / 100 / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_launch": bb, "traffic": measured_traffic(rb["tiling"], n=big),
            "tiling": rb["tiling"]}
        line["copy_reference"] = {"pool_size": copy_bandwidth(torch, bytes64 // 2),
                                  "cache_free": copy_bandwidth(torch, 4 * bytes64)}
        line["ensemble_fp64"] = run_ensemble(ws, torch, args.ensemble_steps, tune=not args.no_tune)
        line["adjoint_fp64"] = run_adjoint(ws, torch)
        line["medium_fp64"] = run_medium(ws, torch, tune=not args.no_tune)
        line["tiled_fp64"] = run_tiled(ws, torch, tune=not args.no_tune)
        line["two_level_fp64"] = run_two_level(ws, torch, tune=not args.no_tune)
        line["three_level_fp64"] = run_three_level(ws, torch, tune=not args.no_tune)
        line["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
        line["cpu_baseline"]["other_workloads"] = cpu_baseline_workloads()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
