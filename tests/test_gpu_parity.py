"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

FP64 must match to a relative L-infinity of 1e-12 per component, FP32 to 1e-5
(the error is printed for every FP32 result).  Batched vs per-patch launches,
tile shapes, and graph vs eager execution must agree bitwise.
"""

import math

import numpy as np
import pytest
import torch

import workloads
from helpers import FP32_TOL, FP64_TOL, rel_linf

pytestmark = pytest.mark.gpu

RHO, KB, C0 = 1.0, 4.0, 2.0


@pytest.fixture(scope="module")
def ws():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_02638_amd as ws
    return ws


def uniform_level(ws, n, dtype=torch.float64, bc="extrap", limiter="mc", xc=0.5, yc=0.5,
                  ny=None, state=None):
    ny = ny or n
    q = state if state is not None else workloads.padded_state(n, ny, 0.0, 0.0, 1 / n, 1 / ny, xc, yc)
    lev = ws.Level([dict(mx=n, my=ny, dx=1 / n, dy=1 / ny, bc=bc)], [(RHO, KB)], dtype=dtype,
                   limiter=limiter)
    lev.upload(0, q)
    lev.fill_ghosts()
    return lev, q


def test_ghost_fill_matches_oracle_bitwise(ws, oracle_lib):
    for bc in ("extrap", "periodic"):
        rng = np.random.default_rng(3)
        q = rng.normal(size=(3, 13 + 4, 21 + 4))
        lev, _ = uniform_level(ws, 21, ny=13, bc=bc, state=q)
        ref = oracle_lib.fill_bc(q.copy(), bc)
        assert np.array_equal(lev.download(0), ref), bc


def test_cfg1_fp64_every_step(ws, oracle_lib):
    """128^2, radial pulse, extrapolation, MC, CFL 0.9, 100 steps; host dt rule."""
    n = 128
    lev, q0 = uniform_level(ws, n)
    qo = oracle_lib.fill_bc(q0.copy(), "extrap")
    dx = 1.0 / n
    dt = 0.9 * dx / C0
    worst = 0.0
    for s in range(100):
        qo, cfl_o, _ = oracle_lib.step(qo, dx, dx, dt, RHO, KB, "mc")
        oracle_lib.fill_bc(qo, "extrap")
        cfl_g = lev.step(dt)
        assert cfl_g == cfl_o, (s, cfl_g, cfl_o)
        err = rel_linf(lev.download(0), qo)
        worst = max(worst, err.max())
        assert err.max() <= FP64_TOL, (s, err)
        dt = dt * 0.9 / cfl_o
    print(f"cfg1 fp64 worst rel Linf over 100 steps: {worst:.3e}")
    assert np.abs(qo[0] - q0[0]).max() > 0.5  # the pulse moved


def test_cfg1_fp32_error_reported(ws, oracle_lib):
    n = 128
    lev, q0 = uniform_level(ws, n, dtype=torch.float32)
    dx = 1.0 / n
    ref = oracle_lib.run(q0, 100, dx, dx, RHO, KB, limiter="mc", bc="extrap", cfl_desired=0.9)
    lev.set_dt([0.9 * dx / C0])
    lev.capture(100, 0.9)
    lev.graph_launch()
    err = rel_linf(lev.download(0), ref["q"])
    print(f"cfg1 fp32 rel Linf vs fp64 oracle: p={err[0]:.3e} u={err[1]:.3e} v={err[2]:.3e}")
    assert err.max() <= FP32_TOL, err


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_device_dt_graph_matches_oracle_and_eager(ws, oracle_lib, dtype):
    n = 96
    dx = 1.0 / n
    ref = oracle_lib.run(workloads.padded_state(n, n, 0, 0, dx, dx, 0.45, 0.52), 60, dx, dx, RHO,
                         KB, limiter="mc", bc="extrap", cfl_desired=0.9)
    lev_g, _ = uniform_level(ws, n, dtype, xc=0.45, yc=0.52)
    lev_e, _ = uniform_level(ws, n, dtype, xc=0.45, yc=0.52)
    for lev in (lev_g, lev_e):
        lev.set_dt([0.9 * dx / C0])
    lev_g.capture(60, 0.9)
    lev_g.graph_launch()
    for _ in range(60):
        lev_e.step_auto(0.9)
    qg, qe = lev_g.download(0), lev_e.download(0)
    assert np.array_equal(qg, qe)
    dt_g, cfl_last, cfl_max = lev_g.read_dt_cfl()
    assert dt_g[0] == ref["dts"][-1] * 0.9 / ref["cfls"][-1]
    assert cfl_last[0] == ref["cfls"][-1] and cfl_max[0] == ref["cfls"].max()
    err = rel_linf(qg, ref["q"])
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    print(f"graph {dtype} rel Linf: {err}")
    assert err.max() <= tol


def test_graph_replays_agree(ws):
    """Replaying a captured graph (with eager work and syncs between replays)
    gives the same trajectory as eager steps."""
    n = 64
    dx = 1.0 / n
    lev_g, _ = uniform_level(ws, n)
    lev_e, _ = uniform_level(ws, n)
    for lev in (lev_g, lev_e):
        lev.set_dt([0.9 * dx / C0])
    lev_g.capture(4, 0.9)
    for rep in range(3):
        lev_g.graph_launch()
        for _ in range(4):
            lev_e.step_auto(0.9)
        _ = lev_g.conservation_sums()  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(lev_g.download(0), lev_e.download(0)), rep


def test_cfg2_mini_fp64_500_steps(ws, oracle_lib):
    n = 256
    dx = 1.0 / n
    lev, q0 = uniform_level(ws, n)
    ref = oracle_lib.run(q0, 500, dx, dx, RHO, KB, limiter="mc", bc="extrap", cfl_desired=0.9)
    lev.set_dt([0.9 * dx / C0])
    lev.capture(500, 0.9)
    lev.graph_launch()
    err = rel_linf(lev.download(0), ref["q"])
    print(f"256^2 x 500 fp64 rel Linf: {err}")
    assert err.max() <= FP64_TOL


def test_cfg2_full_size_fp64(ws, oracle_lib):
    """2048^2 in the benchmark's launch configuration: 10 steps against the
    oracle on the whole grid, then the full 500-step graph run, checked by
    its symmetry under transpose and 90-degree rotation."""
    n = 2048
    dx = 1.0 / n
    lev, q0 = uniform_level(ws, n)
    ref = oracle_lib.run(q0, 10, dx, dx, RHO, KB, limiter="mc", bc="extrap", cfl_desired=0.9)
    lev.set_dt([0.9 * dx / C0])
    lev.capture(10, 0.9)
    lev.graph_launch()
    err = rel_linf(lev.download(0), ref["q"])
    print(f"2048^2 x 10 fp64 rel Linf: {err}")
    assert err.max() <= FP64_TOL
    lev2, _ = uniform_level(ws, n)
    lev2.set_dt([0.9 * dx / C0])
    lev2.capture(500, 0.9)
    lev2.graph_launch()
    q = lev2.download(0)
    p, u, v = q[0, 2:-2, 2:-2], q[1, 2:-2, 2:-2], q[2, 2:-2, 2:-2]
    scale = np.abs(q).max()
    assert np.abs(p - p.T).max() <= FP64_TOL * scale
    assert np.abs(u - v.T).max() <= FP64_TOL * scale
    N = n
    i = np.arange(N)[None, :]
    j = np.arange(N)[:, None]
    assert np.abs(p - p[N - 1 - i, j]).max() <= FP64_TOL * scale
    assert np.abs(u + v[N - 1 - i, j]).max() <= FP64_TOL * scale
    _dt, _last, cmax = lev2.read_dt_cfl()
    assert abs(cmax[0] - 0.9) <= 1e-15


def _amr_patches(level_index, count=None):
    lv = workloads.amr_level_batch()[level_index]
    if count is not None:
        lv = lv[:count]
    return lv


def _amr_level(ws, specs, dtype):
    lev = ws.Level([dict(mx=p.mx, my=p.my, dx=p.dx, dy=p.dy) for p in specs], [(RHO, KB)],
                   dtype=dtype)
    states = [workloads.padded_state(p.mx, p.my, p.xlo, p.ylo, p.dx, p.dy) for p in specs]
    for k, q in enumerate(states):
        lev.upload(k, q)
    return lev, states


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_amr_level_batched_equals_per_patch_and_oracle(ws, oracle_lib, dtype):
    """The finest level of the synthetic hierarchy (~2800 patches of 16..64
    cells, frozen ghosts): batched launch == per-patch launches bitwise, and
    both match the oracle."""
    specs = _amr_patches(2)
    lev_b, states = _amr_level(ws, specs, dtype)
    lev_p, _ = _amr_level(ws, specs, dtype)
    dx = specs[0].dx
    dt = 0.9 * dx / C0
    cur = states
    for s in range(3):
        cb = lev_b.step(dt)
        cp = lev_p.step_per_patch(dt)
        assert cb == cp
        cur, cfl_o = oracle_lib.step_patches(cur, dx, dx, dt, RHO, KB, "mc")
        assert cb == cfl_o.max()
    # relative L-infinity of the level's result: per component over all its
    # patches (a patch-by-patch normalisation divides the FP64 rounding floor
    # of O(1) pressures by velocities of 1e-4 in patches the pulse barely
    # reaches; that worst per-patch value is printed as a diagnostic)
    diff = np.zeros(3)
    refmax = np.zeros(3)
    worst_patch = 0.0
    for k in range(len(specs)):
        a, b = lev_b.download(k), lev_p.download(k)
        assert np.array_equal(a, b), k
        diff = np.maximum(diff, np.abs(a - cur[k]).reshape(3, -1).max(axis=1))
        refmax = np.maximum(refmax, np.abs(cur[k]).reshape(3, -1).max(axis=1))
        worst_patch = max(worst_patch, rel_linf(a, cur[k]).max())
    err = diff / refmax
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    print(f"amr level-3 {len(specs)} patches {dtype}: level rel Linf {err}, "
          f"worst single-patch {worst_patch:.3e}")
    assert err.max() <= tol
    assert np.array_equal(lev_b.patch_cfl(), lev_p.patch_cfl())


TILINGS = [("direct", 8, 32), ("direct", 16, 16), ("direct", 32, 8), ("direct", 64, 4),
           ("direct", 64, 32), ("direct", 128, 2), ("direct", 256, 1), ("direct", 256, 32),
           ("direct", 32, 256), ("march", 64, 4), ("march", 64, 36), ("march", 64, 64),
           ("march", 64, 256), ("march", 64, 8), ("march", 64, 12), ("march", 64, 28),
           ("march", 64, 40), ("march", 64, 100), ("march", 64, 160)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", ["extrap", "periodic"])
def test_results_do_not_depend_on_tiling(ws, dtype, bc):
    """Every tiling and both tile kernels (direct footprint, marching lane
    segments) give bitwise-identical states."""
    nx, ny = 200, 136  # ragged for every tile shape
    rng = np.random.default_rng(5)
    q = workloads.padded_state(nx, ny, 0, 0, 1 / nx, 1 / ny, 0.4, 0.6)
    q[1:, 2:-2, 2:-2] += 0.1 * rng.normal(size=(2, ny, nx))
    outs = []
    tilings = [t for t in TILINGS if bc != "periodic" or t[0] == "direct"]
    for var, tw, th in tilings:
        lev, _ = uniform_level(ws, nx, ny=ny, state=q, dtype=dtype, bc=bc)
        lev.set_tiling(tw, th, variant=var)
        for _ in range(5):
            lev.step(0.4 / nx)
        outs.append(lev.download(0))
    for t, o in zip(tilings[1:], outs[1:]):
        assert np.array_equal(o, outs[0]), t


def test_march_matches_oracle_on_small_and_ragged_patches(ws, oracle_lib):
    for (mx, my, tw, th) in [(5, 3, 64, 16), (13, 40, 64, 32), (29, 29, 64, 8), (61, 7, 64, 4),
                             (120, 70, 64, 32), (121, 9, 64, 12), (250, 33, 64, 20)]:
        rng = np.random.default_rng(mx * 100 + my)
        q = rng.normal(size=(3, my + 4, mx + 4))
        dx, dy = 1 / mx, 1 / my
        dt = 0.5 * min(dx, dy) / C0
        ref = oracle_lib.run(q, 4, dx, dy, RHO, KB, limiter="mc", bc="extrap", dt=dt)
        lev, _ = uniform_level(ws, mx, ny=my, state=q)
        lev.set_tiling(tw, th, variant="march")
        for _ in range(4):
            lev.step(dt)
        err = rel_linf(lev.download(0), ref["q"])
        assert err.max() <= FP64_TOL, (mx, my, err)


def test_ensemble_per_instance_dt(ws, oracle_lib):
    insts = workloads.ensemble(n=8, lo=32, hi=64)
    patches = [dict(mx=e.mx, my=e.my, dx=e.dx, dy=e.dy, instance=k, bc="extrap")
               for k, e in enumerate(insts)]
    lev = ws.Level(patches, [(e.rho, e.K) for e in insts])
    for k, e in enumerate(insts):
        lev.upload(k, e.state())
    lev.fill_ghosts()
    lev.set_dt([0.9 * min(e.dx, e.dy) / math.sqrt(e.K / e.rho) for e in insts])
    lev.capture(50, 0.9)
    lev.graph_launch()
    dts, cfl_last, _ = lev.read_dt_cfl()
    for k, e in enumerate(insts):
        ref = oracle_lib.run(e.state(), 50, e.dx, e.dy, e.rho, e.K, limiter="mc", bc="extrap",
                             cfl_desired=0.9)
        err = rel_linf(lev.download(k), ref["q"])
        assert err.max() <= FP64_TOL, (k, err)
        assert cfl_last[k] == ref["cfls"][-1]
        assert dts[k] == ref["dts"][-1] * 0.9 / ref["cfls"][-1]


@pytest.mark.parametrize("shape,bc,limiter", [
    ((1, 1), "extrap", "mc"), ((1, 7), "extrap", "mc"), ((7, 1), "extrap", "mc"),
    ((2, 2), "periodic", "mc"), ((65, 33), "periodic", "mc"), ((65, 33), "extrap", "none"),
    ((3, 130), "extrap", "mc"),
])
def test_edge_cases(ws, oracle_lib, shape, bc, limiter):
    mx, my = shape
    rng = np.random.default_rng(mx * 1000 + my)
    q = rng.normal(size=(3, my + 4, mx + 4))
    dx, dy = 1 / mx, 1 / my
    dt = 0.5 * min(dx, dy) / C0
    ref = oracle_lib.run(q, 7, dx, dy, RHO, KB, limiter=limiter, bc=bc, dt=dt)
    lev, _ = uniform_level(ws, mx, ny=my, bc=bc, limiter=limiter, state=q)
    for _ in range(7):
        lev.step(dt)
    err = rel_linf(lev.download(0), ref["q"])
    assert err.max() <= FP64_TOL, err


def test_conservation_sums(ws, oracle_lib):
    n = 80
    rng = np.random.default_rng(8)
    q = workloads.padded_state(n, n, 0, 0, 1 / n, 1 / n, 0.3, 0.7)
    q[1:, 2:-2, 2:-2] = 0.1 * rng.normal(size=(2, n, n))
    lev, _ = uniform_level(ws, n, bc="periodic", state=q)
    s0 = lev.conservation_sums()[0]
    ref0 = oracle_lib.conservation_sums(oracle_lib.fill_bc(q.copy(), "periodic"), 1 / n, 1 / n)
    np.testing.assert_allclose(s0, ref0, rtol=0, atol=1e-14)
    lev.set_dt([0.9 / n / C0])
    lev.capture(200, 0.9)
    lev.graph_launch()
    s1 = lev.conservation_sums()[0]
    assert np.all(np.abs(s1 - s0) <= 1e-13 * np.array([1.0, 0.1, 0.1]))


def test_invalid_use_reports_errors(ws):
    lev, _ = uniform_level(ws, 16)
    with pytest.raises(ws.WaveStepError) as e:
        lev.graph_launch()
    assert e.value.code == -2
    with pytest.raises(ws.WaveStepError) as e:
        lev.set_tiling(24, 8)
    assert e.value.code == -1
    with pytest.raises(ws.WaveStepError):
        lev.step(-1.0)
    lev.capture(3, 0.9)
    lev.step(0.01)  # the state moves to the other pool than at capture time
    with pytest.raises(ws.WaveStepError):
        lev.graph_launch()


def test_autotune_restores_state_and_keeps_results(ws, tmp_path):
    """The tuner times candidate tilings on the live level: afterwards the
    state is exactly what it was, and a step gives bitwise the same result as
    with the default tiling."""
    from paper_1808_02638_amd.autotune import autotune

    rng = np.random.default_rng(12)
    shapes = [(150, 40), (33, 17), (33, 20), (9, 30), (64, 64)]
    patches = [dict(mx=mx, my=my, dx=1 / mx, dy=1 / my, bc="extrap") for mx, my in shapes]
    states = [rng.normal(size=(3, my + 4, mx + 4)) for mx, my in shapes]
    levels = []
    for tuned in (False, True):
        lev = ws.Level(patches, [(RHO, KB)])
        for k, q in enumerate(states):
            lev.upload(k, q)
        lev.fill_ghosts()
        lev.set_dt([0.002])
        before = [lev.download(k) for k in range(len(shapes))]
        if tuned:
            choice = autotune(lev, launches=4, cache_path=str(tmp_path / "tiling.json"))
            assert not choice["cached"]
            for k in range(len(shapes)):
                assert np.array_equal(lev.download(k), before[k])
            again = autotune(lev, launches=4, cache_path=str(tmp_path / "tiling.json"))
            assert again["cached"] and again["classes"] == choice["classes"]
        lev.step(0.002)
        levels.append([lev.download(k) for k in range(len(shapes))])
        lev.close()
    for a, b in zip(*levels):
        assert np.array_equal(a, b)


def test_autotune_times_with_a_stable_dt_and_restores_the_levels_dt(ws, tmp_path):
    """On a level whose device dt was never set, the tuner's timed steps run
    with a stable dt (their state stays finite, so the restore is exact and
    the timings are of real data); a dt that was set comes back unchanged."""
    from paper_1808_02638_amd.autotune import autotune

    shapes = [(120, 120)] * 6
    lev = ws.Level([dict(mx=mx, my=my, dx=1 / 480, dy=1 / 480) for mx, my in shapes], [(RHO, KB)])
    rng = np.random.default_rng(5)
    states = [1.0 + 0.1 * rng.normal(size=(3, my + 4, mx + 4)) for mx, my in shapes]
    for k, q in enumerate(states):
        lev.upload(k, q)
    autotune(lev, launches=4, use_cache=False)
    dt_after = lev.read_dt_cfl()[0]
    assert np.isfinite(dt_after).all() and (dt_after > 0).all()
    for k, q in enumerate(states):
        assert np.array_equal(lev.download(k), q)
    for _ in range(3):
        lev.step(0.9 / 480 / 2.0, read_cfl=False)
    assert all(np.isfinite(lev.download(k)).all() for k in range(len(shapes)))
    lev.set_dt([1.25e-4])
    autotune(lev, launches=4, use_cache=False)
    assert lev.read_dt_cfl()[0][0] == 1.25e-4
    lev.close()


def test_ensemble_full_size_graph(ws, oracle_lib):
    """The 64-instance ensemble (sides 128-512, K in [1, 9], rho in [0.5, 2]),
    autotuned, 200 steps as one graph with per-instance FP64 Courant numbers:
    the three smallest instances against the oracle over all 200 steps, and
    for every instance the dt rule (after the first step each instance steps
    at Courant number 0.9)."""
    from paper_1808_02638_amd.autotune import autotune

    insts = workloads.ensemble()
    lev = ws.Level([dict(mx=e.mx, my=e.my, dx=e.dx, dy=e.dy, instance=k, bc="extrap")
                    for k, e in enumerate(insts)], [(e.rho, e.K) for e in insts])
    dt0 = [0.9 * min(e.dx, e.dy) / math.sqrt(e.K / e.rho) for e in insts]
    for k, e in enumerate(insts):
        lev.upload(k, e.state())
    lev.fill_ghosts()
    lev.set_dt(dt0)
    autotune(lev, launches=4, use_cache=False)
    lev.capture(200, 0.9)
    lev.graph_launch()
    dts, cfl_last, cfl_max = lev.read_dt_cfl()
    for k, e in enumerate(insts):
        c = math.sqrt(e.K / e.rho)
        assert abs(cfl_last[k] - 0.9) <= 1e-14, (k, cfl_last[k])
        assert abs(dts[k] - 0.9 * min(e.dx, e.dy) / c) <= 1e-12 * dts[k], k
        assert abs(cfl_max[k] - 0.9) <= 1e-14
    order = sorted(range(len(insts)), key=lambda k: insts[k].mx * insts[k].my)[:3]
    for k in order:
        e = insts[k]
        ref = oracle_lib.run(e.state(), 200, e.dx, e.dy, e.rho, e.K, limiter="mc", bc="extrap",
                             cfl_desired=0.9)
        err = rel_linf(lev.download(k), ref["q"])
        print(f"ensemble instance {k} ({e.mx}x{e.my}, K={e.K:.3f}, rho={e.rho:.3f}): "
              f"rel Linf {err.max():.2e}")
        assert err.max() <= FP64_TOL, (k, err)
        assert cfl_last[k] == ref["cfls"][-1]
    sums = lev.conservation_sums()
    assert np.isfinite(sums).all()
    lev.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_vanleer_matches_oracle(ws, oracle_lib, dtype):
    """The van Leer limiter (the paper's own benchmark limiter): 128^2 radial
    pulse, 100 steps at CFL 0.9 with the device dt rule, against the oracle's
    van Leer step (theta from wave dot products; the kernels use the
    equivalent 2ab/(a+b) on wave strengths)."""
    n = 128
    dx = 1.0 / n
    lev, q0 = uniform_level(ws, n, dtype=dtype, limiter="vanleer")
    lev.set_dt([0.9 * dx / C0])
    lev.capture(100, 0.9)
    lev.graph_launch()
    ref = oracle_lib.run(q0, 100, dx, dx, RHO, KB, limiter="vanleer", bc="extrap",
                         cfl_desired=0.9)
    err = rel_linf(lev.download(0), ref["q"])
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    print(f"van Leer {dtype} rel Linf: p={err[0]:.3e} u={err[1]:.3e} v={err[2]:.3e}")
    assert err.max() <= tol, err
    # the limiters differ on this data
    mc = oracle_lib.run(q0, 100, dx, dx, RHO, KB, limiter="mc", bc="extrap", cfl_desired=0.9)
    assert np.abs(mc["q"] - ref["q"]).max() > 1e-3
    lev.close()


def test_vanleer_tiling_independent_and_no_branches(ws):
    rng = np.random.default_rng(31)
    nx, ny = 150, 77
    q = rng.normal(size=(3, ny + 4, nx + 4))
    outs = []
    for var, tw, th in [("direct", 64, 4), ("direct", 16, 48), ("march", 64, 8),
                        ("march", 64, 36), ("march", 64, 100)]:
        lev, _ = uniform_level(ws, nx, ny=ny, state=q, limiter="vanleer")
        lev.set_tiling(tw, th, variant=var)
        for _ in range(3):
            lev.step(0.5 / nx / C0)
        outs.append(lev.download(0))
        if var == "direct" and tw == 64:
            with pytest.raises(ws.WaveStepError):
                lev.step_record_masks(0.5 / nx / C0, lev.new_masks())
        lev.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
