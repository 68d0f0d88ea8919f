"""GPU parity of the two-level composite step (coarse step, r fine steps with
ghosts from the coarse level, updating, conservation fix) against the
oracle's composite step, through the ws_cf_* entry points of the C ABI.

FP64 within a relative L-infinity of 1e-12 per component, FP32 within 1e-5;
composite totals conserved to 1e-13 on a periodic coarse patch; with ratio 1
the composite step equals the plain level step bitwise.
"""

import numpy as np
import pytest
import torch

from helpers import FP32_TOL, FP64_TOL, rel_linf
from oracle import amr as oamr
import oracle.oracle as O

pytestmark = pytest.mark.gpu

RHO, KB, C0 = 1.0, 4.0, 2.0


@pytest.fixture(scope="module")
def ws():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_02638_amd as ws
    return ws


def smooth(X, Y):
    r = np.hypot(X - 0.45, Y - 0.55)
    p = 1.0 + 0.5 * np.exp(-((r / 0.12) ** 2))
    return np.stack([p, 0.1 * np.sin(2 * np.pi * X), 0.1 * np.cos(2 * np.pi * Y)])


def coarse_state(n, fn):
    xc = (np.arange(-2, n + 2) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    return np.ascontiguousarray(fn(X, Y), dtype=np.float64)


def build(ws, n, rects, r, bc, dtype=torch.float64, fn=smooth, limiter="mc"):
    """Oracle start state and the two GPU levels holding it."""
    qc = coarse_state(n, fn)
    fines = oamr.init_fines(qc, rects, r, fn)
    O.fill_bc(qc, bc)
    coarse = ws.Level([dict(mx=n, my=n, dx=1 / n, dy=1 / n, bc=bc)], [(RHO, KB)], dtype=dtype,
                      limiter=limiter)
    fine = ws.Level([dict(mx=r * w, my=r * h, dx=1 / (n * r), dy=1 / (n * r)) for (_, _, w, h) in rects],
                    [(RHO, KB)], dtype=dtype, limiter=limiter, stream=coarse.stream)
    coarse.upload(0, qc)
    for k, f in enumerate(fines):
        fine.upload(k, f.q)
    tl = ws.TwoLevel(coarse, fine, r, [(0, ci0, cj0) for (ci0, cj0, _, _) in rects])
    return qc, fines, coarse, fine, tl


RECTS = [(6, 8, 8, 10), (20, 5, 6, 6), (30, 30, 10, 8)]


@pytest.mark.parametrize("bc", ["periodic", "extrap"])
@pytest.mark.parametrize("r", [2, 4])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_composite_matches_oracle(ws, dtype, r, bc):
    n, steps = 48, 8
    dt = 0.8 / n / C0
    qc, fines, coarse, fine, tl = build(ws, n, RECTS, r, bc, dtype)
    q, fs = qc, fines
    for _ in range(steps):
        q, fs = oamr.two_level_step(q, fs, 1 / n, 1 / n, dt, RHO, KB, r, bc=bc)
        tl.step(dt)
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    err = rel_linf(coarse.download(0), q)
    print(f"two-level r={r} {bc} {dtype}: coarse rel Linf {err}")
    assert err.max() <= tol, err
    for k, f in enumerate(fs):
        got = fine.download(k)
        e = rel_linf(got[:, 2:-2, 2:-2], f.q[:, 2:-2, 2:-2])
        assert e.max() <= tol, (k, e)
    tl.close()
    fine.close()
    coarse.close()


@pytest.mark.parametrize("r", [2, 4])
def test_composite_conserves(ws, r):
    """Periodic coarse 64^2, three fine patches, 60 composite steps at CFL
    0.9: the coarse level's sums (covered cells hold the fine means) stay
    constant to 1e-13."""
    n = 64
    rects = [(6, 8, 12, 10), (26, 5, 8, 8), (40, 36, 14, 12)]
    _, _, coarse, fine, tl = build(ws, n, rects, r, "periodic")
    s0 = coarse.conservation_sums()[0]
    dt = 0.9 / n / C0
    for _ in range(60):
        tl.step(dt)
    s1 = coarse.conservation_sums()[0]
    scale = np.abs(s0).max()
    print(f"two-level r={r} conservation drift {(s1 - s0) / scale}")
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s0, s1)
    tl.close()
    fine.close()
    coarse.close()


def test_ratio_one_equals_level_step(ws):
    n = 40
    rects = [(5, 6, 12, 9), (22, 20, 14, 16)]
    qc, _, coarse, fine, tl = build(ws, n, rects, 1, "extrap")
    plain = ws.Level([dict(mx=n, my=n, dx=1 / n, dy=1 / n, bc="extrap")], [(RHO, KB)])
    plain.upload(0, qc)
    dt = 0.8 / n / C0
    for _ in range(6):
        tl.step(dt)
        plain.step(dt, read_cfl=False)
    ref = plain.download(0)
    assert np.array_equal(coarse.download(0), ref)
    for k, (ci0, cj0, w, h) in enumerate(rects):
        got = fine.download(k)[:, 2:-2, 2:-2]
        assert np.array_equal(got, ref[:, 2 + cj0:2 + cj0 + h, 2 + ci0:2 + ci0 + w])
    for lev in (tl, fine, coarse, plain):
        lev.close()


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_fine_ghost_fill_matches_oracle(ws, r):
    """Both coarse pools hold the same state after an upload, so the fill at
    any alpha is the spatial interpolation alone."""
    n = 30
    rects = [(4, 5, 7, 6), (16, 14, 9, 11)]
    rng = np.random.default_rng(60 + r)
    rough = lambda X, Y: np.stack([np.sin(7 * X) + 0.1 * rng.normal(size=X.shape),
                                   np.cos(5 * Y) * X, X * Y + 0.2 * rng.normal(size=X.shape)])
    qc, fines, coarse, fine, tl = build(ws, n, rects, r, "extrap", fn=rough)
    tl.fill_fine_ghosts(0.3)
    for k, f in enumerate(fines):
        ref = f.q.copy()
        oamr.fill_fine_ghosts(ref, f, qc, r)
        got = fine.download(k)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-15 * scale, k
    for lev in (tl, fine, coarse):
        lev.close()


def test_invalid_layouts_are_refused(ws):
    n = 32
    coarse = ws.Level([dict(mx=n, my=n, dx=1 / n, dy=1 / n, bc="extrap")], [(RHO, KB)])

    def fine_of(shapes, r=2, bc=None, mat=(RHO, KB), dx=None):
        return ws.Level([dict(mx=w, my=h, dx=dx or 1 / (n * r), dy=dx or 1 / (n * r), bc=bc)
                         for (w, h) in shapes], [mat], stream=coarse.stream)

    cases = [
        (fine_of([(8, 8)]), 2, [(0, 1, 5)]),                  # not 2 cells inside
        (fine_of([(8, 8), (8, 8)]), 2, [(0, 4, 4), (0, 7, 5)]),  # overlapping
        (fine_of([(9, 8)]), 2, [(0, 5, 5)]),                  # not whole coarse cells
        (fine_of([(8, 8)], bc="extrap"), 2, [(0, 5, 5)]),     # fine ghosts not frozen
        (fine_of([(8, 8)], mat=(1.0, 9.0)), 2, [(0, 5, 5)]),  # another material
        (fine_of([(8, 8)], dx=1 / (3 * n)), 2, [(0, 5, 5)]),  # wrong cell size
        (fine_of([(8, 8)]), 2, [(1, 5, 5)]),                  # no such coarse patch
    ]
    for fine, r, places in cases:
        with pytest.raises(ws.WaveStepError):
            ws.TwoLevel(coarse, fine, r, places)
        fine.close()
    other = ws.Level([dict(mx=8, my=8, dx=1 / (2 * n), dy=1 / (2 * n))], [(RHO, KB)])
    with pytest.raises(ValueError):
        ws.TwoLevel(coarse, other, 2, [(0, 5, 5)])  # not on the coarse stream
    other.close()
    tc = ws.Level([dict(mx=8, my=8, dx=1 / (2 * n), dy=1 / (2 * n))], [(RHO, KB)],
                  transverse_corr=True, stream=coarse.stream)
    with pytest.raises(ws.WaveStepError):
        ws.TwoLevel(coarse, tc, 2, [(0, 5, 5)])  # limiters differ
    tc.close()
    coarse.close()


def _full_layout(ws, bc):
    import workloads
    n, r = 1024, 4
    rects = workloads.two_level_layout(n)
    dx = 1.0 / n
    qc = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    O.fill_bc(qc, bc)
    fq = [workloads.padded_state(r * w, r * h, ci0 * dx, cj0 * dx, dx / r, dx / r)
          for (ci0, cj0, w, h) in rects]
    coarse = ws.Level([dict(mx=n, my=n, dx=dx, dy=dx, bc=bc)], [(RHO, KB)])
    fine = ws.Level([dict(mx=r * w, my=r * h, dx=dx / r, dy=dx / r) for (_, _, w, h) in rects],
                    [(RHO, KB)], stream=coarse.stream)
    coarse.upload(0, qc)
    for k, q in enumerate(fq):
        fine.upload(k, q)
    tl = ws.TwoLevel(coarse, fine, r, [(0, ci0, cj0) for (ci0, cj0, _, _) in rects])
    return n, r, rects, qc, fq, coarse, fine, tl


def test_full_size_layout_sampled_against_oracle(ws):
    """The benchmark's layout (1024^2 coarse, 364 ratio-4 fine patches of
    120^2): one composite step on the GPU; the oracle steps the same coarse
    state with three of the fine patches.  Fine patches are 3 coarse cells
    apart, so within one step a patch and the coarse cells it covers or
    borders depend on no other patch: those cells, the three fine states and
    every coarse cell at least 3 cells from all patches must agree."""
    n, r, rects, qc, fq, coarse, fine, tl = _full_layout(ws, "extrap")
    dt = 0.9 / n / C0
    tl.step(dt)
    got_c = coarse.download(0)
    picks = [0, len(rects) // 2, len(rects) - 1]
    fines = [oamr.FinePatch(*rects[k], fq[k]) for k in picks]
    ref_c, ref_f = oamr.two_level_step(qc, fines, 1 / n, 1 / n, dt, RHO, KB, r, bc="extrap")
    scale = np.abs(ref_c).reshape(3, -1).max(axis=1)
    for k, f in zip(picks, ref_f):
        ci0, cj0, w, h = rects[k]
        blk = (slice(None), slice(2 + cj0 - 1, 2 + cj0 + h + 1), slice(2 + ci0 - 1, 2 + ci0 + w + 1))
        err = (np.abs(got_c[blk] - ref_c[blk]).reshape(3, -1).max(axis=1)) / scale
        assert err.max() <= FP64_TOL, (k, err)
        e = rel_linf(fine.download(k)[:, 2:-2, 2:-2], f.q[:, 2:-2, 2:-2])
        assert e.max() <= FP64_TOL, (k, e)
    far = np.ones((n, n), bool)
    for (ci0, cj0, w, h) in rects:
        far[max(cj0 - 3, 0):cj0 + h + 3, max(ci0 - 3, 0):ci0 + w + 3] = False
    d = np.abs(got_c[:, 2:-2, 2:-2] - ref_c[:, 2:-2, 2:-2])[:, far]
    assert (d.max(axis=1) / scale).max() <= FP64_TOL
    for lev in (tl, fine, coarse):
        lev.close()


def test_full_size_layout_conserves_periodic(ws):
    """The benchmark's layout with a periodic coarse patch: the covered coarse
    cells start as point values, not fine means, so the totals are compared
    from the end of the first composite step on, over 8 more steps."""
    n, r, rects, qc, fq, coarse, fine, tl = _full_layout(ws, "periodic")
    tl.step(0.9 / n / C0)
    s1 = coarse.conservation_sums()[0]
    for _ in range(8):
        tl.step(0.9 / n / C0)
    s2 = coarse.conservation_sums()[0]
    scale = np.abs(s1).max()
    print(f"full-size two-level conservation drift {(s2 - s1) / scale}")
    assert np.all(np.abs(s2 - s1) <= 1e-13 * scale), (s1, s2)
    for lev in (tl, fine, coarse):
        lev.close()


# --------------------------------------------------------------------------
# Three levels (nested couplings)
# --------------------------------------------------------------------------

L1_RECTS = [(4, 4, 10, 12), (19, 6, 8, 8)]
L2_PLACES = [(0, (2, 2, 3, 3)), (1, (2, 2, 4, 3)), (0, (2, 8, 4, 2))]


def build3(ws, n, r, bc, dtype=torch.float64, fn=smooth, l1_rects=L1_RECTS, l2_places=L2_PLACES):
    """Oracle start state (level 1 and 2 means written into their parents) and
    the three GPU levels holding it."""
    L1_RECTS, L2_PLACES = l1_rects, l2_places
    qc = coarse_state(n, fn)
    l1 = oamr.init_fines(qc, L1_RECTS, r, fn)
    l2 = []
    dx1 = 1.0 / (n * r)
    for parent, (ci0, cj0, ncx, ncy) in L2_PLACES:
        P = l1[parent]
        x0, y0 = P.ci0 / n + ci0 * dx1, P.cj0 / n + cj0 * dx1
        x = x0 + (np.arange(-2, r * ncx + 2) + 0.5) * dx1 / r
        y = y0 + (np.arange(-2, r * ncy + 2) + 0.5) * dx1 / r
        X, Y = np.meshgrid(x, y, indexing="xy")
        q = np.ascontiguousarray(fn(X, Y), dtype=np.float64)
        fp = oamr.FinePatch(ci0, cj0, ncx, ncy, q, parent)
        oamr.average_down(P.q, fp, q, r)
        l2.append(fp)
    for P in l1:
        oamr.average_down(qc, P, P.q, r)
    O.fill_bc(qc, bc)
    lev0 = ws.Level([dict(mx=n, my=n, dx=1 / n, dy=1 / n, bc=bc)], [(RHO, KB)], dtype=dtype)
    lev1 = ws.Level([dict(mx=r * w, my=r * h, dx=dx1, dy=dx1) for (_, _, w, h) in L1_RECTS],
                    [(RHO, KB)], dtype=dtype, stream=lev0.stream)
    lev2 = ws.Level([dict(mx=r * p[1][2], my=r * p[1][3], dx=dx1 / r, dy=dx1 / r) for p in L2_PLACES],
                    [(RHO, KB)], dtype=dtype, stream=lev0.stream)
    lev0.upload(0, qc)
    for k, P in enumerate(l1):
        lev1.upload(k, P.q)
    for k, P in enumerate(l2):
        lev2.upload(k, P.q)
    h = ws.Hierarchy([lev0, lev1, lev2], r,
                     [[(0, ci0, cj0) for (ci0, cj0, _, _) in L1_RECTS],
                      [(parent, rc[0], rc[1]) for parent, rc in L2_PLACES]])
    return qc, [l1, l2], (lev0, lev1, lev2), h


@pytest.mark.parametrize("bc", ["periodic", "extrap"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_three_levels_match_oracle(ws, dtype, bc):
    n, r = 32, 2
    qc, levels, levs, h = build3(ws, n, r, bc, dtype)
    dt = 0.8 / n / C0
    q, lv = qc, levels
    for _ in range(4):
        q, lv = oamr.multi_level_step(q, lv, 1 / n, 1 / n, dt, RHO, KB, r, bc=bc)
        h.step(dt)
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    err = rel_linf(levs[0].download(0), q)
    print(f"three levels {bc} {dtype}: level-0 rel Linf {err}")
    assert err.max() <= tol, err
    for l in (1, 2):
        for k, P in enumerate(lv[l - 1]):
            e = rel_linf(levs[l].download(k)[:, 2:-2, 2:-2], P.q[:, 2:-2, 2:-2])
            assert e.max() <= tol, (l, k, e)
    h.close()
    for lev in levs:
        lev.close()


def test_three_levels_conserve(ws):
    n, r = 32, 2
    _, _, levs, h = build3(ws, n, r, "periodic")
    s0 = levs[0].conservation_sums()[0]
    for _ in range(30):
        h.step(0.9 / n / C0)
    s1 = levs[0].conservation_sums()[0]
    scale = np.abs(s0).max()
    print(f"three levels conservation drift {(s1 - s0) / scale}")
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s0, s1)
    h.close()
    for lev in levs:
        lev.close()


def test_tuned_composite_steps_from_poisoned_memory_match_oracle(ws):
    """Pools and workspaces start as NaN bytes (the binding allocates them
    so), every level is autotuned (many timed steps, the state saved and
    restored) and the composite steps run after that: two levels (r = 4) and
    three levels (r = 2) match the oracle at 1e-12 and stay finite, so no
    kernel of the composite step reads memory the library has not written."""
    from paper_1808_02638_amd.autotune import autotune

    probe = ws.Level([dict(mx=20, my=10, dx=0.05, dy=0.1)], [(RHO, KB)])
    torch.cuda.synchronize()
    # the pools hold nothing before an upload; the workspace holds the tables
    # and cleared slots init wrote, and poison everywhere else
    for b in probe.pools:
        assert bool((b == 0xFF).all()), "pools are not poisoned"
    assert bool((probe.workspace == 0xFF).any()), "workspace is not poisoned"
    probe.close()

    n, steps, r = 48, 8, 4
    dt = 0.8 / n / C0
    qc, fines, coarse, fine, tl = build(ws, n, RECTS, r, "extrap")
    for lev in (coarse, fine):
        autotune(lev, launches=4, use_cache=False)
    q, fs = qc, fines
    for _ in range(steps):
        q, fs = oamr.two_level_step(q, fs, 1 / n, 1 / n, dt, RHO, KB, r, bc="extrap")
        tl.step(dt)
    got = coarse.download(0)
    assert np.isfinite(got).all()
    err = rel_linf(got, q)
    print(f"tuned two-level from poisoned memory: coarse rel Linf {err}")
    assert err.max() <= FP64_TOL, err
    for k, f in enumerate(fs):
        gf = fine.download(k)
        assert np.isfinite(gf).all(), k
        assert rel_linf(gf[:, 2:-2, 2:-2], f.q[:, 2:-2, 2:-2]).max() <= FP64_TOL, k
    tl.close()
    fine.close()
    coarse.close()

    n, r = 32, 2
    qc, levels, levs, h = build3(ws, n, r, "extrap")
    for lev in levs:
        autotune(lev, launches=4, use_cache=False)
    dt = 0.8 / n / C0
    q, lv = qc, levels
    for _ in range(4):
        q, lv = oamr.multi_level_step(q, lv, 1 / n, 1 / n, dt, RHO, KB, r, bc="extrap")
        h.step(dt)
    err = rel_linf(levs[0].download(0), q)
    print(f"tuned three levels from poisoned memory: level-0 rel Linf {err}")
    assert err.max() <= FP64_TOL, err
    for l in (1, 2):
        for k, P in enumerate(lv[l - 1]):
            g = levs[l].download(k)
            assert np.isfinite(g).all(), (l, k)
            assert rel_linf(g[:, 2:-2, 2:-2], P.q[:, 2:-2, 2:-2]).max() <= FP64_TOL, (l, k)
    h.close()
    for lev in levs:
        lev.close()


def test_tuned_full_size_two_level_stays_finite(ws):
    """The benchmark's two-level leg as the benchmark runs it (1024^2 coarse,
    364 ratio-4 fine patches, both levels autotuned, then composite steps),
    from poisoned memory: every cell of both levels stays finite, and the
    coarse cells far from all patches equal those of the plain coarse step."""
    from paper_1808_02638_amd.autotune import autotune

    n, r, rects, qc, fq, coarse, fine, tl = _full_layout(ws, "extrap")
    for lev in (coarse, fine):
        autotune(lev, launches=6, use_cache=False)
    dt = 0.9 / n / C0
    plain = ws.Level([dict(mx=n, my=n, dx=1 / n, dy=1 / n, bc="extrap")], [(RHO, KB)])
    plain.upload(0, qc)
    for _ in range(3):
        tl.step(dt)
        plain.step(dt, read_cfl=False)
    got = coarse.download(0)
    assert np.isfinite(got).all()
    for k in range(len(rects)):
        assert np.isfinite(fine.download(k)).all(), k
    far = np.ones((n, n), bool)
    for (ci0, cj0, w, h) in rects:
        far[max(cj0 - 9, 0):cj0 + h + 9, max(ci0 - 9, 0):ci0 + w + 9] = False
    ref = plain.download(0)
    assert np.array_equal(got[:, 2:-2, 2:-2][:, far], ref[:, 2:-2, 2:-2][:, far])
    for lev in (tl, fine, coarse, plain):
        lev.close()


def test_nesting_is_checked(ws):
    n, r = 32, 2
    _, _, levs, h = build3(ws, n, r, "extrap")
    outer, inner = h.pairs
    L = ws._lib.lib()
    with pytest.raises(ws.WaveStepError):
        ws._lib.check(L.ws_cf_nest(inner._cf, outer._cf))  # levels do not chain
    with pytest.raises(ws.WaveStepError):
        ws._lib.check(L.ws_cf_nest(outer._cf, outer._cf))
    h.close()
    for lev in levs:
        lev.close()


# --------------------------------------------------------------------------
# Touching fine patches: ghosts from siblings, the fix gathered per coarse cell
# --------------------------------------------------------------------------

# B touches A on its right; coarse column 17 lies between B and C (its cells
# border both); D touches A's top, E touches D's right and A's and B's tops
# (concave corners whose coarse cells border two patches); F stands alone.
TOUCHING = [(6, 6, 6, 8), (12, 6, 5, 8), (18, 6, 5, 8), (6, 14, 4, 5), (10, 14, 6, 3),
            (26, 20, 6, 6)]


@pytest.mark.parametrize("r", [2, 3])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_touching_patches_match_oracle(ws, dtype, r):
    n, steps = 40, 6
    dt = 0.8 / n / C0
    qc, fines, coarse, fine, tl = build(ws, n, TOUCHING, r, "periodic", dtype)
    q, fs = qc, fines
    for _ in range(steps):
        q, fs = oamr.two_level_step(q, fs, 1 / n, 1 / n, dt, RHO, KB, r, bc="periodic")
        tl.step(dt)
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    err = rel_linf(coarse.download(0), q)
    print(f"touching r={r} {dtype}: coarse rel Linf {err}")
    assert err.max() <= tol, err
    for k, f in enumerate(fs):
        e = rel_linf(fine.download(k)[:, 2:-2, 2:-2], f.q[:, 2:-2, 2:-2])
        assert e.max() <= tol, (k, e)
    for lev in (tl, fine, coarse):
        lev.close()


@pytest.mark.parametrize("r", [2, 4])
def test_touching_patches_conserve(ws, r):
    n = 40
    _, _, coarse, fine, tl = build(ws, n, TOUCHING, r, "periodic")
    s0 = coarse.conservation_sums()[0]
    for _ in range(40):
        tl.step(0.9 / n / C0)
    s1 = coarse.conservation_sums()[0]
    scale = np.abs(s0).max()
    print(f"touching r={r} conservation drift {(s1 - s0) / scale}")
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s0, s1)
    for lev in (tl, fine, coarse):
        lev.close()


@pytest.mark.parametrize("r", [1, 2, 3])
def test_sibling_ghost_fill_matches_oracle(ws, r):
    """Ghosts inside a sibling hold the sibling's cell bitwise, the others the
    coarse interpolation (both coarse pools hold the uploaded state)."""
    n = 40
    rng = np.random.default_rng(80 + r)
    rough = lambda X, Y: np.stack([np.sin(7 * X) + 0.1 * rng.normal(size=X.shape),
                                   np.cos(5 * Y) * X, X * Y + 0.2 * rng.normal(size=X.shape)])
    qc, fines, coarse, fine, tl = build(ws, n, TOUCHING, r, "extrap", fn=rough)
    tl.fill_fine_ghosts(0.3)
    for k, f in enumerate(fines):
        ref = f.q.copy()
        sibs = [(g, g.q) for d, g in enumerate(fines) if d != k]
        oamr.fill_fine_ghosts(ref, f, qc, r, sibs)
        got = fine.download(k)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-15 * scale, k
        # the copied ghosts are exact
        gi = r * f.ci0 + np.arange(-2, r * f.ncx + 2)[None, :]
        gj = r * f.cj0 + np.arange(-2, r * f.ncy + 2)[:, None]
        for g in (x for d, x in enumerate(fines) if d != k):
            inside = ((gi >= r * g.ci0) & (gi < r * (g.ci0 + g.ncx)) &
                      (gj >= r * g.cj0) & (gj < r * (g.cj0 + g.ncy)))
            assert np.array_equal(got[:, inside], ref[:, inside]), (k, "copy")
    for lev in (tl, fine, coarse):
        lev.close()


L1_TOUCH = [(4, 4, 10, 12), (14, 4, 8, 8), (14, 12, 6, 4)]
L2_TOUCH = [(0, (2, 2, 3, 3)), (0, (5, 2, 4, 3)), (0, (2, 5, 3, 2)), (1, (2, 2, 4, 3)),
            (1, (6, 2, 3, 5))]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_three_levels_touching_match_oracle_and_conserve(ws, dtype):
    n, r = 32, 2
    qc, levels, levs, h = build3(ws, n, r, "periodic", dtype, l1_rects=L1_TOUCH,
                                 l2_places=L2_TOUCH)
    s0 = levs[0].conservation_sums()[0]
    dt = 0.8 / n / C0
    q, lv = qc, levels
    for _ in range(4):
        q, lv = oamr.multi_level_step(q, lv, 1 / n, 1 / n, dt, RHO, KB, r, bc="periodic")
        h.step(dt)
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    err = rel_linf(levs[0].download(0), q)
    print(f"three levels touching {dtype}: level-0 rel Linf {err}")
    assert err.max() <= tol, err
    for l in (1, 2):
        for k, P in enumerate(lv[l - 1]):
            e = rel_linf(levs[l].download(k)[:, 2:-2, 2:-2], P.q[:, 2:-2, 2:-2])
            assert e.max() <= tol, (l, k, e)
    if dtype == torch.float64:
        s1 = levs[0].conservation_sums()[0]
        scale = np.abs(s0).max()
        assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s0, s1)
    h.close()
    for lev in levs:
        lev.close()


def test_full_size_layout_cut_into_touching_quadrants_equals_uncut(ws):
    """The benchmark's two-level layout (1024^2 coarse, 364 ratio-4 patches
    of 30^2 coarse cells), and the same with every patch cut into four
    touching quadrants (1456 patches whose ghosts partly come from siblings,
    the cuts carrying no fix): three composite steps give the same coarse
    and fine states to rounding."""
    import workloads

    n, r = 1024, 4
    rects = workloads.two_level_layout(n)
    dx = 1.0 / n

    def run(rect_list):
        qc = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
        O.fill_bc(qc, "extrap")
        coarse = ws.Level([dict(mx=n, my=n, dx=dx, dy=dx, bc="extrap")], [(RHO, KB)])
        fine = ws.Level([dict(mx=r * w, my=r * h, dx=dx / r, dy=dx / r) for (_, _, w, h) in rect_list],
                        [(RHO, KB)], stream=coarse.stream)
        coarse.upload(0, qc)
        for k, (ci0, cj0, w, h) in enumerate(rect_list):
            fine.upload(k, workloads.padded_state(r * w, r * h, ci0 * dx, cj0 * dx, dx / r, dx / r))
        tl = ws.TwoLevel(coarse, fine, r, [(0, ci0, cj0) for (ci0, cj0, _, _) in rect_list])
        for _ in range(3):
            tl.step(0.9 * dx / C0)
        out = coarse.download(0), [fine.download(k)[:, 2:-2, 2:-2] for k in range(len(rect_list))]
        for lev in (tl, fine, coarse):
            lev.close()
        return out

    quads = []
    for (ci0, cj0, w, h) in rects:
        a, b = w // 2, h // 2
        quads += [(ci0, cj0, a, b), (ci0 + a, cj0, w - a, b), (ci0, cj0 + b, a, h - b),
                  (ci0 + a, cj0 + b, w - a, h - b)]
    qa, fa = run(rects)
    qb, fb = run(quads)
    scale = np.abs(qa).max()
    print(f"uncut vs quadrants: coarse max diff {np.abs(qa - qb).max() / scale:.2e}")
    assert np.abs(qa - qb).max() <= 1e-13 * scale
    for k, (ci0, cj0, w, h) in enumerate(rects):
        a, b = w // 2, h // 2
        whole = fa[k]
        parts = fb[4 * k:4 * k + 4]
        assert np.abs(whole[:, :r * b, :r * a] - parts[0]).max() <= 1e-13 * scale
        assert np.abs(whole[:, :r * b, r * a:] - parts[1]).max() <= 1e-13 * scale
        assert np.abs(whole[:, r * b:, :r * a] - parts[2]).max() <= 1e-13 * scale
        assert np.abs(whole[:, r * b:, r * a:] - parts[3]).max() <= 1e-13 * scale
