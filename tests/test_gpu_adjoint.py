"""GPU adjoint: the branch-recording forward step and the frozen-branch
adjoint step of the HIP library (through its C ABI) against the oracle, the
receiver gather/scatter helpers, and the autograd wrapper's gradient against
the oracle's adjoint sweep and against central finite differences.

Masks are compared bitwise (both sides decide the branches in FP64); adjoint
results to a relative L-infinity of 1e-12 per component.
"""

import math

import numpy as np
import pytest
import torch

import workloads
from helpers import FP64_TOL, rel_linf

pytestmark = pytest.mark.gpu

RHO, KB, C0 = 1.0, 4.0, 2.0


@pytest.fixture(scope="module")
def ws():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_02638_amd as ws
    return ws


def recorded_state(oracle_lib, mx, my, steps=4, seed=0, noise=0.05):
    """A state a few oracle steps into the pulse run on an mx x my grid of the
    unit square, with velocity noise so every branch occurs; ghosts filled."""
    q = workloads.padded_state(mx, my, 0, 0, 1 / mx, 1 / my, 0.52, 0.47)
    rng = np.random.default_rng(seed)
    q[1:, 2:-2, 2:-2] += noise * rng.normal(size=(2, my, mx))
    oracle_lib.fill_bc(q, "extrap")
    dt = 0.8 / max(mx, my) / C0
    if steps:
        q = oracle_lib.run(q, steps, 1 / mx, 1 / my, RHO, KB, limiter="mc", bc="extrap",
                           dt=dt)["q"]
    return q, dt


def level_of(ws, shapes, bcs, tiling=None):
    lev = ws.Level([dict(mx=mx, my=my, dx=1 / mx, dy=1 / my, bc=bc)
                    for (mx, my), bc in zip(shapes, bcs)], [(RHO, KB)])
    if tiling is not None:
        lev.set_tiling(**tiling)
    return lev


def patch_masks(lev, masks, k):
    off = sum((mx + 1) * (my + 1) for mx, my in lev.shapes[:k])
    mx, my = lev.shapes[k]
    return masks[off:off + (mx + 1) * (my + 1)].cpu().numpy().reshape(my + 1, mx + 1)


CASES = [
    ("small", [(24, 16)], ["extrap"], None),
    ("march", [(200, 72)], ["extrap"], None),
    ("direct_wide", [(200, 72)], ["extrap"], dict(tile_w=64, tile_h=16, variant="direct")),
    ("frozen_ghosts", [(37, 23)], [None], None),
    ("degenerate", [(1, 1), (1, 7), (6, 1), (2, 2)], ["extrap", "extrap", "extrap", None], None),
    ("mixed_level", [(150, 40), (33, 17), (9, 30)], ["extrap", None, "extrap"], None),
]


def _setup(ws, oracle_lib, shapes, bcs, tiling):
    lev = level_of(ws, shapes, bcs, tiling)
    states, dts = [], []
    for k, (mx, my) in enumerate(shapes):
        q, dt = recorded_state(oracle_lib, mx, my, steps=3 if mx * my > 4 else 0, seed=k)
        states.append(q)
        dts.append(dt)
        lev.upload(k, q)
    dt = min(dts)
    return lev, states, dt


@pytest.mark.parametrize("name,shapes,bcs,tiling", CASES, ids=[c[0] for c in CASES])
def test_recorded_masks_match_oracle(ws, oracle_lib, name, shapes, bcs, tiling):
    lev, states, dt = _setup(ws, oracle_lib, shapes, bcs, tiling)
    masks = lev.new_masks()
    lev.step_record_masks(dt, masks)
    torch.cuda.synchronize()
    counts = np.zeros(4, np.int64)
    for k, (mx, my) in enumerate(shapes):
        ref_q, _cfl, ref_m = oracle_lib.step(states[k], 1 / mx, 1 / my, dt, RHO, KB, "mc",
                                             record_masks=True)
        got = patch_masks(lev, masks, k)
        bad = np.argwhere(got != ref_m)
        assert bad.size == 0, f"{name} patch {k}: {len(bad)} mask bytes differ, first {bad[:5]}"
        counts += np.bincount(np.concatenate([(ref_m >> s) & 3 for s in (0, 2, 4, 6)]).ravel(),
                              minlength=4)
        if bcs[k] == "extrap":
            oracle_lib.fill_bc(ref_q, "extrap")
            err = rel_linf(lev.download(k), ref_q)
        else:
            err = rel_linf(lev.download(k)[:, 2:-2, 2:-2], ref_q[:, 2:-2, 2:-2])
        assert err.max() <= FP64_TOL, (name, k, err)
    if name in ("small", "march"):
        assert (counts > 0).all(), counts  # every branch occurs


@pytest.mark.parametrize("name,shapes,bcs,tiling", CASES, ids=[c[0] for c in CASES])
def test_adjoint_step_matches_oracle(ws, oracle_lib, name, shapes, bcs, tiling):
    lev, states, dt = _setup(ws, oracle_lib, shapes, bcs, tiling)
    masks = lev.new_masks()
    lev.step_record_masks(dt, masks)
    lam_in, lam_out = lev.new_buffer(), lev.new_buffer()
    rng = np.random.default_rng(5)
    lams = []
    for k, (mx, my) in enumerate(shapes):
        lam = rng.normal(size=(3, my, mx))
        lams.append(lam)
        view = lev.patch_view(lam_in, k)
        view.copy_(torch.from_numpy(rng.normal(size=view.shape)))  # ghosts are not read
        view[:, 2:-2, 2:-2] = torch.from_numpy(lam)
    lam_out.fill_(np.nan)
    torch.cuda.synchronize()
    lev.adjoint_step(dt, masks, lam_in, lam_out)
    torch.cuda.synchronize()
    for k, (mx, my) in enumerate(shapes):
        ref_m = patch_masks(lev, masks, k)
        ref = oracle_lib.adjoint_step(lams[k], states[k], 1 / mx, 1 / my, dt, RHO, KB, ref_m,
                                      bc="extrap" if bcs[k] == "extrap" else None)
        out = lev.patch_view(lam_out, k).cpu().numpy()
        err = rel_linf(out[:, 2:-2, 2:-2], ref)
        print(f"{name} patch {k} ({mx}x{my}, {bcs[k]}): adjoint rel Linf {err.max():.2e}")
        assert err.max() <= FP64_TOL, (name, k, err)
        ghost = out.copy()
        ghost[:, 2:-2, 2:-2] = 0.0
        assert not ghost.any(), "lam_out ghosts must be 0"


def test_adjoint_is_transpose_of_gpu_step(ws, oracle_lib):
    """The limiter is positively homogeneous, so the step frozen at q maps q
    to step(q): <step(q), y> = <q, S^T y> over the interior, GPU only."""
    mx, my = 90, 64
    q, dt = recorded_state(oracle_lib, mx, my, steps=2)
    lev = level_of(ws, [(mx, my)], ["extrap"])
    lev.upload(0, q)
    lev.fill_ghosts()
    q = lev.download(0)
    masks = lev.new_masks()
    lev.step_record_masks(dt, masks)
    sq = lev.download(0)[:, 2:-2, 2:-2]
    rng = np.random.default_rng(9)
    y = rng.normal(size=(3, my, mx))
    lam_in, lam_out = lev.new_buffer(), lev.new_buffer()
    lev.patch_view(lam_in, 0)[:, 2:-2, 2:-2] = torch.from_numpy(y)
    lev.adjoint_step(dt, masks, lam_in, lam_out)
    sty = lev.patch_view(lam_out, 0)[:, 2:-2, 2:-2].cpu().numpy()
    lhs = float(np.vdot(sq, y))
    rhs = float(np.vdot(q[:, 2:-2, 2:-2], sty))
    scale = np.abs(sq).sum() * np.abs(y).max()
    assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


def test_gather_and_add_at(ws):
    lev = level_of(ws, [(40, 30), (17, 9)], ["extrap", None])
    buf = lev.new_buffer()
    rng = np.random.default_rng(2)
    for k in range(2):
        v = lev.patch_view(buf, k)
        v.copy_(torch.from_numpy(rng.normal(size=v.shape)))
    mx, my = lev.shapes[1]
    ij = np.array([[0, 0], [16, 8], [5, 3], [5, 3], [17, 0], [-1, 2], [3, 9]], np.int32)
    ij_d = torch.from_numpy(ij).cuda()
    out = torch.empty(len(ij), dtype=torch.float64, device="cuda")
    lev.gather(1, 2, ij_d, out, buf=buf)
    host = lev.patch_view(buf, 1).cpu().numpy()
    got = out.cpu().numpy()
    for n, (i, j) in enumerate(ij):
        if 0 <= i < mx and 0 <= j < my:
            assert got[n] == host[2, j + 2, i + 2]
        else:
            assert np.isnan(got[n])
    val = torch.arange(1, len(ij) + 1, dtype=torch.float64, device="cuda")
    before = lev.patch_view(buf, 1).cpu().numpy()
    lev.add_at(1, 0, ij_d, val, buf=buf)
    after = lev.patch_view(buf, 1).cpu().numpy()
    expect = before.copy()
    for n, (i, j) in enumerate(ij):
        if 0 <= i < mx and 0 <= j < my:
            expect[0, j + 2, i + 2] += n + 1
    assert np.allclose(after, expect, rtol=0, atol=1e-14)
    assert after[0, 3 + 2, 5 + 2] == before[0, 3 + 2, 5 + 2] + 3 + 4 or \
        after[0, 3 + 2, 5 + 2] == before[0, 3 + 2, 5 + 2] + 4 + 3


def _smooth_problem(n, seed=11):
    xs = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    rng = np.random.default_rng(seed)
    bg = sum(rng.uniform(0.05, 0.2) * np.sin(2 * np.pi * (rng.integers(1, 4) * X
                                                          + rng.integers(1, 4) * Y)
                                             + rng.uniform(0, 6)) for _ in range(4))
    p0 = 1.0 + np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.02) + bg
    vel = np.zeros((2, n, n))
    vel[0] = 0.1 * np.cos(2 * np.pi * Y)
    return p0, vel, rng


def test_gradient_matches_oracle_adjoint(ws, oracle_lib):
    """48^2, 30 steps, checkpoints every 7 steps (a ragged last segment):
    traces, misfit and gradient vs the oracle's forward and adjoint sweep."""
    n, steps = 48, 30
    setup = workloads.adjoint_setup(n=n, steps=steps)
    p0, vel, _ = _smooth_problem(n)
    state0 = np.concatenate([np.zeros((1, n, n)), vel])  # (p, u, v); p is replaced by p0
    target = oracle_lib.forward_traces(p0 * 0.9, steps, 1 / n, 1 / n, setup.dt, RHO, KB,
                                       setup.receivers, None, state0)[1]
    J_o, g_o, tr_o, _ = oracle_lib.adjoint_run(p0, steps, 1 / n, 1 / n, setup.dt, RHO, KB,
                                               setup.receivers, target, state0=state0)
    run = ws.AcousticsAdjoint(n, n, 1 / n, 1 / n, RHO, KB, setup.receivers, steps, setup.dt,
                              checkpoint_every=7, velocity0=vel)
    p = torch.tensor(p0, device="cuda", requires_grad=True)
    tr = run.traces(p)
    J = 0.5 * ((tr - torch.from_numpy(target).cuda()) ** 2).sum()
    J.backward()
    tr_g = tr.detach().cpu().numpy()
    g = p.grad.cpu().numpy()
    e_tr = np.abs(tr_g - tr_o).max() / np.abs(tr_o).max()
    e_g = np.abs(g - g_o).max() / np.abs(g_o).max()
    print(f"traces rel Linf {e_tr:.2e}, gradient rel Linf {e_g:.2e}, J {float(J):.6e} vs {J_o:.6e}")
    assert e_tr <= FP64_TOL
    assert e_g <= FP64_TOL
    assert abs(float(J) - J_o) <= 1e-10 * J_o
    run.close()


def test_gradient_independent_of_checkpoint_interval(ws):
    """Checkpoints every 1, 7, 25 or 40 steps, or every step's branches
    recorded in the forward pass (no re-run in the backward pass): the same
    traces and gradient, bit for bit."""
    n, steps = 40, 25
    setup = workloads.adjoint_setup(n=n, steps=steps)
    p0, vel, _ = _smooth_problem(n, seed=4)
    target = torch.zeros((steps, len(setup.receivers)), dtype=torch.float64, device="cuda")
    grads, traces = [], []
    for k, store in ((1, False), (7, False), (25, False), (40, False), (7, True)):
        run = ws.AcousticsAdjoint(n, n, 1 / n, 1 / n, RHO, KB, setup.receivers, steps, setup.dt,
                                  checkpoint_every=k, velocity0=vel, store_branches=store)
        p = torch.tensor(p0, device="cuda", requires_grad=True)
        tr = run.traces(p)
        (0.5 * ((tr - target) ** 2).sum()).backward()
        grads.append(p.grad.cpu().numpy())
        traces.append(tr.detach().cpu().numpy())
        run.close()
    for g, t in zip(grads[1:], traces[1:]):
        assert np.array_equal(g, grads[0])
        assert np.array_equal(t, traces[0])


def _gpu_forward(ws, n, p0, vel, steps, dt, receivers):
    """J-free forward on the GPU that also records every step's branches."""
    lev = level_of(ws, [(n, n)], ["extrap"])
    q = np.zeros((3, n + 4, n + 4))
    q[0, 2:-2, 2:-2] = p0
    q[1:, 2:-2, 2:-2] = vel
    lev.upload(0, q)
    lev.fill_ghosts()
    ij = torch.from_numpy(np.ascontiguousarray(receivers, np.int32)).cuda()
    tr = torch.empty((steps, len(receivers)), dtype=torch.float64, device="cuda")
    masks = []
    for s in range(steps):
        m = lev.new_masks()
        lev.step_record_masks(dt, m)
        lev.gather(0, 0, ij, tr[s])
        masks.append(m)
    torch.cuda.synchronize()
    out = tr.cpu().numpy(), [m.cpu().numpy() for m in masks]
    lev.close()
    return out


def _fd_probe(ws, n, steps, setup, p0, vel, tr_t, m0, g, v, h=1e-6):
    """(J(p0 + h v) - J(p0 - h v)) / 2h, with the difference of the two misfits
    formed term by term, 1/2 sum (r+ - r-)(r+ + r-), and summed compensated
    (the misfits themselves are large next to their difference)."""
    tp, mp = _gpu_forward(ws, n, p0 + h * v, vel, steps, setup.dt, setup.receivers)
    tm, mm = _gpu_forward(ws, n, p0 - h * v, vel, steps, setup.dt, setup.receivers)
    flips = sum(int((a != b).sum() + (a != c).sum()) for a, b, c in zip(m0, mp, mm))
    terms = 0.5 * (tp - tm) * ((tp - tr_t) + (tm - tr_t))
    return math.fsum(terms.ravel().tolist()) / (2 * h), float(np.vdot(g, v)), flips


def _gradient(ws, n, steps, setup, p0, vel):
    tr_t, _ = _gpu_forward(ws, n, 0.9 * p0, vel, steps, setup.dt, setup.receivers)
    run = ws.AcousticsAdjoint(n, n, 1 / n, 1 / n, RHO, KB, setup.receivers, steps, setup.dt,
                              checkpoint_every=setup.checkpoint_every, velocity0=vel)
    p = torch.tensor(p0, device="cuda", requires_grad=True)
    run.misfit(p, torch.from_numpy(tr_t).cuda()).backward()
    g = p.grad.cpu().numpy()
    run.close()
    _, m0 = _gpu_forward(ws, n, p0, vel, steps, setup.dt, setup.receivers)
    return tr_t, m0, g


def test_gradient_matches_central_differences(ws):
    """32^2, 12 steps: central differences (h = 1e-6) of the GPU misfit along
    seeded random directions vs <grad, v>, graded where no branch changes
    between p0 - h v, p0 and p0 + h v (J is piecewise quadratic in p0, so the
    difference is exact up to rounding inside one branch region)."""
    n, steps = 32, 12
    setup = workloads.adjoint_setup(n=n, steps=steps)
    p0, vel, rng = _smooth_problem(n)
    tr_t, m0, g = _gradient(ws, n, steps, setup, p0, vel)
    graded, flipped = [], 0
    for _ in range(8):
        fd, ad, flips = _fd_probe(ws, n, steps, setup, p0, vel, tr_t, m0, g,
                                  rng.normal(size=(n, n)))
        if flips:
            flipped += 1
        else:
            graded.append((fd, ad))
    print(f"32^2 x 12: graded {len(graded)}, flipped {flipped}: {graded}")
    assert len(graded) >= 4, flipped
    for fd, ad in graded:
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-8), (fd, ad)


def test_full_size_gradient_central_differences(ws):
    """The full adjoint workload: 512^2, 200 steps at Courant 0.8, 16
    receivers, checkpoints every 20 steps.  Probes along single seeded cells
    inside the pulse annulus; flip-free probes are graded at 1e-6, probes
    with branch changes are reported with their flip counts."""
    setup = workloads.adjoint_setup()
    n, steps = setup.n, setup.steps
    p0 = setup.p0()
    vel = np.zeros((2, n, n))
    tr_t = _gpu_forward(ws, n, setup.target_p0(), vel, steps, setup.dt, setup.receivers)[0]
    run = ws.AcousticsAdjoint(n, n, 1 / n, 1 / n, RHO, KB, setup.receivers, steps, setup.dt,
                              checkpoint_every=setup.checkpoint_every)
    p = torch.tensor(p0, device="cuda", requires_grad=True)
    run.misfit(p, torch.from_numpy(tr_t).cuda()).backward()
    g = p.grad.cpu().numpy()
    run.close()
    assert np.isfinite(g).all() and np.abs(g).max() > 0
    # the same gradient bits with every step's branches stored in the forward pass
    runb = ws.AcousticsAdjoint(n, n, 1 / n, 1 / n, RHO, KB, setup.receivers, steps, setup.dt,
                               store_branches=True)
    pb = torch.tensor(p0, device="cuda", requires_grad=True)
    runb.misfit(pb, torch.from_numpy(tr_t).cuda()).backward()
    assert np.array_equal(pb.grad.cpu().numpy(), g)
    runb.close()
    _, m0 = _gpu_forward(ws, n, p0, vel, steps, setup.dt, setup.receivers)
    rng = np.random.default_rng(20)
    xs = (np.arange(n) + 0.5) / n
    r = np.hypot(*np.meshgrid(xs - 0.5, xs - 0.5, indexing="xy"))
    cells = np.argwhere(np.abs(r - 0.25) < 0.09)
    picks = cells[rng.choice(len(cells), size=6, replace=False)]
    rows = []
    for j, i in picks:
        v = np.zeros((n, n))
        v[j, i] = 1.0
        fd, ad, flips = _fd_probe(ws, n, steps, setup, p0, vel, tr_t, m0, g, v)
        rows.append((int(i), int(j), fd, ad, flips))
    print("512^2 x 200 probes (i, j, fd, adjoint, branch flips):")
    for row in rows:
        print("  ", row)
    graded = [(fd, ad) for _i, _j, fd, ad, fl in rows if fl == 0]
    assert graded, "every probe changed branches"
    for fd, ad in graded:
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-8), (fd, ad)


def test_adjoint_invalid_use(ws):
    lev = level_of(ws, [(16, 16)], ["extrap"])
    masks = lev.new_masks()
    a, b = lev.new_buffer(), lev.new_buffer()
    with pytest.raises(ws.WaveStepError):
        lev.adjoint_step(0.001, masks, a, a)
    with pytest.raises(ws.WaveStepError):
        lev.adjoint_step(-1.0, masks, a, b)
    per = ws.Level([dict(mx=16, my=16, dx=1 / 16, dy=1 / 16, bc="periodic")], [(RHO, KB)])
    with pytest.raises(ws.WaveStepError):
        per.adjoint_step(0.001, per.new_masks(), per.new_buffer(), per.new_buffer())
    f32 = ws.Level([dict(mx=16, my=16, dx=1 / 16, dy=1 / 16, bc="extrap")], [(RHO, KB)],
                   dtype=torch.float32)
    with pytest.raises((ws.WaveStepError, ValueError)):
        f32.adjoint_step(0.001, f32.new_masks(), a, b)
    lw = ws.Level([dict(mx=16, my=16, dx=1 / 16, dy=1 / 16, bc="extrap")], [(RHO, KB)],
                  limiter="none")
    with pytest.raises(ws.WaveStepError):
        lw.step_record_masks(0.001, lw.new_masks())
    for l in (lev, per, f32, lw):
        l.close()
