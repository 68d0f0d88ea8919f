"""GPU parity of the transverse-correction variant (the transverse solver also
splits the limited second-order correction) against the FP64 oracle's variant.

Same bar as the default method: FP64 within a relative L-infinity of 1e-12 per
component, FP32 within 1e-5 (printed), every tiling and batched vs per-patch
launches bitwise equal.
"""

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


def level(ws, mx, my, q, dtype=torch.float64, bc="extrap", limiter="mc"):
    lev = ws.Level([dict(mx=mx, my=my, dx=1 / mx, dy=1 / my, bc=bc)], [(RHO, KB)], dtype=dtype,
                   limiter=limiter, transverse_corr=True)
    lev.upload(0, q)
    if bc is not None:
        lev.fill_ghosts()
    return lev


@pytest.mark.parametrize("limiter", ["mc", "vanleer", "none"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pulse_matches_oracle(ws, oracle_lib, dtype, limiter):
    """128^2 radial pulse, extrapolation, 100 steps at CFL 0.9 with the device
    dt rule (captured graph)."""
    n = 128
    dx = 1.0 / n
    q0 = workloads.padded_state(n, n, 0.0, 0.0, dx, dx, 0.5, 0.5)
    lev = level(ws, n, n, q0, dtype=dtype, limiter=limiter)
    lev.set_dt([0.9 * dx / C0])
    lev.capture(100, 0.9)
    lev.graph_launch()
    ref = oracle_lib.run(q0, 100, dx, dx, RHO, KB, limiter=limiter, bc="extrap", cfl_desired=0.9,
                         transverse_corr=True)
    err = rel_linf(lev.download(0), ref["q"])
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    print(f"transverse-correction {limiter} {dtype} rel Linf: "
          f"p={err[0]:.3e} u={err[1]:.3e} v={err[2]:.3e}")
    assert err.max() <= tol, err
    # the variant is a different method on this data
    base = oracle_lib.run(q0, 100, dx, dx, RHO, KB, limiter=limiter, bc="extrap",
                          cfl_desired=0.9)
    assert np.abs(base["q"] - ref["q"]).max() > 1e-5
    lev.close()


TILINGS = [("direct", 8, 32), ("direct", 16, 16), ("direct", 64, 4), ("direct", 128, 2),
           ("direct", 256, 32), ("direct", 32, 256), ("march", 64, 4), ("march", 64, 8),
           ("march", 64, 12), ("march", 64, 36), ("march", 64, 64), ("march", 64, 100),
           ("march", 64, 256)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("bc", ["extrap", "periodic"])
def test_results_do_not_depend_on_tiling(ws, dtype, bc):
    nx, ny = 200, 136
    rng = np.random.default_rng(15)
    q = workloads.padded_state(nx, ny, 0, 0, 1 / nx, 1 / ny, 0.4, 0.6)
    q[1:, 2:-2, 2:-2] += 0.1 * rng.normal(size=(2, ny, nx))
    outs = []
    tilings = [t for t in TILINGS if bc != "periodic" or t[0] == "direct"]
    for var, tw, th in tilings:
        lev = level(ws, nx, ny, q, dtype=dtype, bc=bc)
        lev.set_tiling(tw, th, variant=var)
        for _ in range(5):
            lev.step(0.4 / nx)
        outs.append(lev.download(0))
        lev.close()
    for t, o in zip(tilings[1:], outs[1:]):
        assert np.array_equal(o, outs[0]), t


@pytest.mark.parametrize("shape,bc,variant,th", [
    ((1, 1), "extrap", "direct", 1), ((1, 7), "extrap", "direct", 1),
    ((7, 1), "extrap", "direct", 1), ((2, 2), "periodic", "direct", 1),
    ((65, 33), "periodic", "direct", 1), ((3, 130), "extrap", "direct", 1),
    ((5, 3), "extrap", "march", 16), ((13, 40), "extrap", "march", 32),
    ((29, 29), "extrap", "march", 8), ((61, 7), "extrap", "march", 4),
    ((121, 9), "extrap", "march", 12), ((250, 33), "extrap", "march", 20),
])
def test_small_ragged_and_degenerate_patches(ws, oracle_lib, shape, bc, variant, th):
    mx, my = shape
    rng = np.random.default_rng(mx * 1000 + my + 7)
    q = rng.normal(size=(3, my + 4, mx + 4))
    dx, dy = 1 / mx, 1 / my
    dt = 0.5 * min(dx, dy) / C0
    ref = oracle_lib.run(q, 6, dx, dy, RHO, KB, limiter="mc", bc=bc, dt=dt, transverse_corr=True)
    lev = level(ws, mx, my, q, bc=bc)
    if variant == "march":
        lev.set_tiling(64, th, variant="march")
    for _ in range(6):
        lev.step(dt)
    err = rel_linf(lev.download(0), ref["q"])
    assert err.max() <= FP64_TOL, (shape, err)
    lev.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_level_frozen_ghosts_batched_equals_per_patch(ws, oracle_lib, dtype):
    """Patches narrow enough for DIRECT tiles next to MARCH-tiled ones in one
    launch, ghosts frozen at random values (every footprint point is read)."""
    shapes = [(16, 20), (40, 33), (70, 24), (23, 64), (9, 5), (130, 17)]
    rng = np.random.default_rng(77)
    states = [rng.normal(size=(3, my + 4, mx + 4)) for mx, my in shapes]
    dx = 1.0 / 64
    specs = [dict(mx=mx, my=my, dx=dx, dy=dx) for mx, my in shapes]

    def make():
        lev = ws.Level(specs, [(RHO, KB)], dtype=dtype, transverse_corr=True)
        for k, q in enumerate(states):
            lev.upload(k, q)
        return lev

    lb, lp = make(), make()
    variants, _, _, _, _ = lb.get_tiling()
    assert set(variants) == {"direct", "march"}, variants  # both tile kernels in one launch
    dt = 0.8 * dx / C0
    cur = [s.copy() for s in states]
    for _ in range(3):
        lb.step(dt)
        lp.step_per_patch(dt)
        cur = [oracle_lib.step(q, dx, dx, dt, RHO, KB, "mc", transverse_corr=True)[0] for q in cur]
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    for k in range(len(shapes)):
        a, b = lb.download(k), lp.download(k)
        assert np.array_equal(a, b), k
        err = rel_linf(a, cur[k])
        assert err.max() <= tol, (shapes[k], err)
    lb.close()
    lp.close()


def test_full_size_2048_fp64(ws, oracle_lib):
    """The 2048^2 FP64 pulse with the default tiling, two steps at CFL 0.9,
    against the oracle on every cell."""
    n = 2048
    dx = 1.0 / n
    q0 = workloads.padded_state(n, n, 0.0, 0.0, dx, dx, 0.5, 0.5)
    rng = np.random.default_rng(5)
    q0[1:, 2:-2, 2:-2] += 1e-3 * rng.normal(size=(2, n, n))
    lev = level(ws, n, n, q0)
    dt = 0.9 * dx / C0
    lev.step(dt)
    lev.step(dt)
    ref = oracle_lib.run(q0, 2, dx, dx, RHO, KB, limiter="mc", bc="extrap", dt=dt,
                         transverse_corr=True)
    err = rel_linf(lev.download(0), ref["q"])
    print(f"transverse-correction 2048^2 rel Linf: {err}")
    assert err.max() <= FP64_TOL, err
    lev.close()


def test_branch_recording_is_refused(ws):
    n = 32
    q = workloads.padded_state(n, n, 0.0, 0.0, 1 / n, 1 / n, 0.5, 0.5)
    lev = level(ws, n, n, q)
    with pytest.raises(ws.WaveStepError):
        lev.step_record_masks(0.5 / n / C0, lev.new_masks())
    lev.close()
