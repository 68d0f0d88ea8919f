"""The level step that allocates nothing (``ws_step_level_noalloc``, its
workspace in the library's own device array) against the context step
``ws_step_level`` on the same level: bitwise equal output buffers and the
same Courant number, for two calls in a row (the second on a smaller level,
so stale contents of the shared array would show), in FP64 and FP32; and
the host-side refusal of a level whose workspace exceeds the array."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1808_02638_amd import _lib as C
from paper_1808_02638_amd.level import Level, _tables, step_level_noalloc

LEVEL_BIG = [dict(mx=200, my=150, dx=1 / 200, dy=1 / 150, instance=0, bc="extrap"),
             dict(mx=64, my=64, dx=1 / 256, dy=1 / 256, instance=1, bc=None),
             dict(mx=40, my=33, dx=1 / 160, dy=1 / 132, instance=1, bc=None),
             dict(mx=17, my=90, dx=1 / 68, dy=1 / 90, instance=0, bc="extrap"),
             dict(mx=130, my=70, dx=1 / 130, dy=1 / 70, instance=2, bc="periodic"),
             dict(mx=1, my=5, dx=0.1, dy=0.2, instance=2, bc="extrap")]
MATS_BIG = [(1.0, 4.0), (0.7, 2.5), (1.6, 8.0)]
LEVEL_SMALL = [dict(mx=33, my=20, dx=1 / 33, dy=1 / 20, instance=0, bc=None),
               dict(mx=90, my=41, dx=1 / 90, dy=1 / 41, instance=0, bc="extrap")]
MATS_SMALL = [(1.2, 3.0)]


def _context_step(patches, mats, dtype, seed):
    """A Level with seeded smooth-plus-noise states: its current pool before
    the step (a copy), the pool after ws_step_level, and the Courant number."""
    rng = np.random.default_rng(seed)
    lev = Level(patches, mats, dtype=dtype, device="cuda")
    for k, p in enumerate(patches):
        mx, my = p["mx"], p["my"]
        y, x = np.mgrid[0:my + 4, 0:mx + 4]
        q = np.stack([1.0 + 0.3 * np.sin(0.2 * x + 0.1 * y), 0.1 * np.cos(0.15 * y),
                      0.05 * np.sin(0.3 * x)]) + 0.02 * rng.standard_normal((3, my + 4, mx + 4))
        lev.upload(k, q)
    lev.fill_ghosts()
    torch.cuda.synchronize()
    q_in = lev.pools[lev.current_pool()].clone()
    dt = 0.4 * min(lev.stable_dt(1.0))
    cfl = lev.step(dt)
    torch.cuda.synchronize()
    q_ref = lev.pools[lev.current_pool()].clone()
    lev.close()
    return q_in, q_ref, dt, cfl


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_step_equals_context_step_twice(dtype):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    for patches, mats, seed in ((LEVEL_BIG, MATS_BIG, 1), (LEVEL_SMALL, MATS_SMALL, 2)):
        q_in, q_ref, dt, cfl_ref = _context_step(patches, mats, dtype, seed)
        # the output starts as the input: ghosts of frozen-ghost patches are
        # kept, everything the step writes is overwritten
        q_out = q_in.clone()
        torch.cuda.synchronize()
        print(f"noalloc step: {len(patches)} patches, {dtype}", flush=True)
        cfl = step_level_noalloc(patches, mats, q_in, q_out, dt, dtype=dtype)
        assert cfl == cfl_ref, (cfl, cfl_ref)
        assert torch.equal(q_out, q_ref), "output differs from ws_step_level's"


def test_noalloc_refuses_levels_beyond_its_array():
    """100000 one-cell patches need more workspace than the array holds: the
    call fails on the host, before any device work."""
    L = C.lib()
    n = 100000
    patches = [dict(mx=1, my=1, dx=1.0, dy=1.0, bc="extrap")] * n
    descs, mats = _tables(patches, [(1.0, 4.0)])
    pool, ws = ctypes.c_int64(), ctypes.c_int64()
    assert L.ws_layout(descs, n, 1, C.WS_F64, ctypes.byref(pool), ctypes.byref(ws)) == 0
    assert ws.value > L.ws_noalloc_scratch_bytes()
    cfl = ctypes.c_double(0.0)
    rc = L.ws_step_level_noalloc(descs, n, mats, 1, C.WS_F64, C.WS_LIM_MC, ctypes.c_void_p(16),
                                 ctypes.c_void_p(32), pool.value, 1e-3, ctypes.byref(cfl), None)
    assert rc == C.WS_ENOMEM
    assert b"no-allocation" in L.ws_last_error()
