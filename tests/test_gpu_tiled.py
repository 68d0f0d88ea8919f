"""GPU parity of a tiled level (patches covering one domain, ghosts exchanged
after every step, ws_link_level) against the oracle's exchange and step,
through the C ABI.

FP64 within a relative L-infinity of 1e-12, FP32 within 1e-5; with periodic
or extrapolating sides in both directions the tiled level equals the domain
stepped as one patch bitwise (FP64), in plain, per-patch, automatic-dt and
captured-graph steps; a two-level composite step over a tiled coarse level
matches the oracle's composite step over the whole domain.
"""

import numpy as np
import pytest
import torch

from helpers import FP32_TOL, FP64_TOL, rel_linf
from oracle import amr as oamr
from oracle import tiled as otiled
import oracle.oracle as O

pytestmark = pytest.mark.gpu

RHO, KB, C0 = 1.0, 4.0, 2.0

# (DX, DY), [(mx, my)], [(x0, y0)]
TILINGS = {
    "2x2_uneven": ((70, 52), [(30, 20), (40, 20), (30, 32), (40, 32)],
                   [(0, 0), (30, 0), (0, 20), (30, 20)]),
    "columns_one_wide": ((50, 36), [(24, 36), (1, 36), (25, 36)], [(0, 0), (24, 0), (25, 0)]),
    "bricks": ((64, 48), [(32, 16), (32, 16), (16, 16), (32, 16), (16, 16), (64, 16)],
               [(0, 0), (32, 0), (0, 16), (16, 16), (48, 16), (0, 32)]),
}


@pytest.fixture(scope="module")
def ws():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_02638_amd as ws
    return ws


def domain_state(DX, DY, seed=7):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid((np.arange(DX) + 0.5) / DX, (np.arange(DY) + 0.5) / DY, indexing="xy")
    p = 1.0 + 0.5 * np.exp(-((X - 0.4) ** 2 + (Y - 0.6) ** 2) / 0.02)
    return np.stack([p + 0.01 * rng.normal(size=X.shape), 0.1 * np.sin(2 * np.pi * Y),
                     0.05 * rng.normal(size=X.shape)])


def tiles_of(interior, shapes, origins, domain, periodic):
    qs = []
    for (mx, my), (x0, y0) in zip(shapes, origins):
        q = np.zeros((3, my + 4, mx + 4))
        q[:, 2:-2, 2:-2] = interior[:, y0:y0 + my, x0:x0 + mx]
        qs.append(q)
    return otiled.exchange_ghosts(qs, origins, domain, periodic)


def tiled_level(ws, shapes, origins, domain, periodic, qs, dtype=torch.float64, dx=None):
    DX, DY = domain
    dx = dx or 1.0 / DX
    lev = ws.Level([dict(mx=mx, my=my, dx=dx, dy=dx) for (mx, my) in shapes], [(RHO, KB)],
                   dtype=dtype)
    lev.link(origins, domain, periodic)
    for k, q in enumerate(qs):
        lev.upload(k, q)
    return lev


@pytest.mark.parametrize("periodic", [(True, True), (False, False), (True, False)])
@pytest.mark.parametrize("tiling", sorted(TILINGS))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_tiled_level_matches_oracle(ws, dtype, tiling, periodic):
    domain, shapes, origins = TILINGS[tiling]
    qs = tiles_of(domain_state(*domain), shapes, origins, domain, periodic)
    lev = tiled_level(ws, shapes, origins, domain, periodic, qs, dtype)
    dx = 1.0 / domain[0]
    dt = 0.8 * dx / C0
    ref = [q.copy() for q in qs]
    for _ in range(6):
        ref = [O.step(q, dx, dx, dt, RHO, KB, "mc")[0] for q in ref]
        otiled.exchange_ghosts(ref, origins, domain, periodic)
        lev.step(dt, read_cfl=False)
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    for k, q in enumerate(ref):
        err = rel_linf(lev.download(k), q)  # ghosts included
        assert err.max() <= tol, (k, err)
    lev.close()


@pytest.mark.parametrize("bc", ["periodic", "extrap"])
@pytest.mark.parametrize("tiling", sorted(TILINGS))
def test_tiled_level_equals_single_patch_bitwise(ws, tiling, bc):
    domain, shapes, origins = TILINGS[tiling]
    DX, DY = domain
    periodic = (bc == "periodic",) * 2
    interior = domain_state(DX, DY, seed=3)
    whole = np.zeros((3, DY + 4, DX + 4))
    whole[:, 2:-2, 2:-2] = interior
    O.fill_bc(whole, bc)
    one = ws.Level([dict(mx=DX, my=DY, dx=1 / DX, dy=1 / DX, bc=bc)], [(RHO, KB)])
    one.upload(0, whole)
    qs = tiles_of(interior, shapes, origins, domain, periodic)
    dt = 0.8 / DX / C0
    # the four step paths: plain, per patch, automatic dt, captured graph
    for path in ("plain", "per_patch", "auto", "graph"):
        lev = tiled_level(ws, shapes, origins, domain, periodic, qs)
        ref = ws.Level([dict(mx=DX, my=DY, dx=1 / DX, dy=1 / DX, bc=bc)], [(RHO, KB)])
        ref.upload(0, whole)
        if path == "plain":
            for _ in range(5):
                lev.step(dt, read_cfl=False)
                ref.step(dt, read_cfl=False)
        elif path == "per_patch":
            for _ in range(5):
                lev.step_per_patch(dt)
                ref.step_per_patch(dt)
        elif path == "auto":
            for L in (lev, ref):
                L.set_dt([dt])
                for _ in range(5):
                    L.step_auto(0.8)
        else:
            for L in (lev, ref):
                L.set_dt([dt])
                L.capture(4, 0.8)
                L.graph_launch()
                L.graph_launch()
        R = ref.download(0)
        for k, ((mx, my), (x0, y0)) in enumerate(zip(shapes, origins)):
            got = lev.download(k)
            assert np.array_equal(got, R[:, y0:y0 + my + 4, x0:x0 + mx + 4]), (path, k)
        if path in ("auto", "graph"):
            assert np.array_equal(np.array(lev.read_dt_cfl()[0]), np.array(ref.read_dt_cfl()[0]))
        lev.close()
        ref.close()
    one.close()


def test_two_level_over_a_tiled_coarse_level(ws):
    """Coarse 40^2 periodic domain as 2x2 tiles of 20^2; two ratio-2 fine
    patches in two of the tiles.  The composite step matches the oracle's
    over the whole domain as one coarse patch."""
    n, r = 40, 2
    xc = (np.arange(-2, n + 2) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    fn = lambda X, Y: np.stack([1.0 + 0.5 * np.exp(-((X - 0.45) ** 2 + (Y - 0.55) ** 2) / 0.01),
                                0.1 * np.sin(2 * np.pi * X), 0.1 * np.cos(2 * np.pi * Y)])
    qc = np.ascontiguousarray(fn(X, Y))
    rects = [(5, 6, 8, 8), (24, 22, 10, 12)]  # whole-domain coarse cells
    fines = oamr.init_fines(qc, rects, r, fn)
    O.fill_bc(qc, "periodic")
    shapes = [(20, 20)] * 4
    origins = [(0, 0), (20, 0), (0, 20), (20, 20)]
    qs = tiles_of(qc[:, 2:-2, 2:-2], shapes, origins, (n, n), (True, True))
    coarse = tiled_level(ws, shapes, origins, (n, n), (True, True), qs)
    fine = ws.Level([dict(mx=r * w, my=r * h, dx=1 / (n * r), dy=1 / (n * r)) for (_, _, w, h) in rects],
                    [(RHO, KB)], stream=coarse.stream)
    for k, f in enumerate(fines):
        fine.upload(k, f.q)
    places = [(0, 5, 6), (3, 4, 2)]  # tile index and cells inside the tile
    tl = ws.TwoLevel(coarse, fine, r, places)
    dt = 0.8 / n / C0
    q, fs = qc, fines
    for _ in range(6):
        q, fs = oamr.two_level_step(q, fs, 1 / n, 1 / n, dt, RHO, KB, r, bc="periodic")
        tl.step(dt)
    for k, ((mx, my), (x0, y0)) in enumerate(zip(shapes, origins)):
        err = rel_linf(coarse.download(k), q[:, y0:y0 + my + 4, x0:x0 + mx + 4])
        assert err.max() <= FP64_TOL, (k, err)
    for k, f in enumerate(fs):
        e = rel_linf(fine.download(k)[:, 2:-2, 2:-2], f.q[:, 2:-2, 2:-2])
        assert e.max() <= FP64_TOL, (k, e)
    for lev in (tl, fine, coarse):
        lev.close()


def test_tiled_layouts_and_uses_are_checked(ws):
    def make(shapes, bc=None):
        return ws.Level([dict(mx=mx, my=my, dx=0.02, dy=0.02, bc=bc) for (mx, my) in shapes],
                        [(RHO, KB)])
    bad = [
        ([(10, 20), (13, 20)], [(0, 0), (11, 0)]),  # a gap
        ([(12, 20), (13, 20)], [(0, 0), (11, 0)]),  # an overlap
        ([(12, 20), (13, 20)], [(0, 0), (12, 0)]),  # outside the domain
    ]
    for shapes, origins in bad:
        lev = make(shapes)
        with pytest.raises(ws.WaveStepError):
            lev.link(origins, (24, 20))
        lev.close()
    lev = make([(12, 20), (12, 20)], bc="periodic")
    with pytest.raises(ws.WaveStepError):  # ghosts would come from two places
        lev.link([(0, 0), (12, 0)], (24, 20))
    lev.close()
    lev = make([(12, 20), (12, 20)])
    lev.link([(0, 0), (12, 0)], (24, 20), (False, False))
    with pytest.raises(ws.WaveStepError):
        lev.step_record_masks(0.001, lev.new_masks())
    coarse = ws.Level([dict(mx=40, my=40, dx=0.02, dy=0.02, bc="extrap")], [(RHO, KB)],
                      stream=lev.stream)
    with pytest.raises(ws.WaveStepError):  # a tiled level as the fine level of a coupling
        ws.TwoLevel(coarse, lev, 2, [(0, 4, 4), (0, 10, 4)])
    # and the other order: a coupling's fine level cannot be linked while it lives
    fine = ws.Level([dict(mx=8, my=8, dx=0.01, dy=0.01), dict(mx=8, my=8, dx=0.01, dy=0.01)],
                    [(RHO, KB)], stream=coarse.stream)
    tl = ws.TwoLevel(coarse, fine, 2, [(0, 4, 4), (0, 8, 4)])
    with pytest.raises(ws.WaveStepError):
        fine.link([(0, 0), (8, 0)], (16, 8))
    tl.close()
    fine.link([(0, 0), (8, 0)], (16, 8))  # allowed once the coupling is gone
    fine.close()
    coarse.close()
    lev.close()


def test_full_size_tiled_level_equals_single_patch(ws):
    """The benchmark's tiled workload at full size: the 2048^2 FP64 pulse as
    4 x 4 patches of 512^2 with extrapolating sides, autotuned, 20 steps at
    Courant number 0.9 in one captured graph, equals the domain as one patch
    bitwise, ghosts included."""
    import workloads
    from paper_1808_02638_amd.autotune import autotune

    n, t = 2048, 4
    w, dx = n // t, 1.0 / n
    q = workloads.padded_state(n, n, 0.0, 0.0, dx, dx)
    O.fill_bc(q, "extrap")
    origins = [(w * a, w * b) for b in range(t) for a in range(t)]
    tiled = ws.Level([dict(mx=w, my=w, dx=dx, dy=dx) for _ in origins], [(RHO, KB)])
    tiled.link(origins, (n, n), (False, False))
    for k, (x0, y0) in enumerate(origins):
        tiled.upload(k, np.ascontiguousarray(q[:, y0:y0 + w + 4, x0:x0 + w + 4]))
    one = ws.Level([dict(mx=n, my=n, dx=dx, dy=dx, bc="extrap")], [(RHO, KB)])
    one.upload(0, q)
    for L in (tiled, one):
        autotune(L, launches=4, use_cache=False)
        L.set_dt([0.9 * dx / C0])
        L.capture(20, 0.9)
        L.graph_launch()
    R = one.download(0)
    for k, (x0, y0) in enumerate(origins):
        assert np.array_equal(tiled.download(k), R[:, y0:y0 + w + 4, x0:x0 + w + 4]), k
    assert np.array_equal(tiled.read_dt_cfl()[0], one.read_dt_cfl()[0])
    tiled.close()
    one.close()


@pytest.mark.parametrize("bc", ["periodic", "extrap"])
def test_degenerate_tilings_equal_single_patch(ws, bc):
    """One patch linked to itself (its ghosts come from its own interior, by
    the domain's wrap or clamp) steps like the same patch with that physical
    condition; a domain cut into one-cell-wide columns does too, bitwise."""
    DX, DY = 13, 9
    periodic = (bc == "periodic",) * 2
    interior = domain_state(DX, DY, seed=21)
    whole = np.zeros((3, DY + 4, DX + 4))
    whole[:, 2:-2, 2:-2] = interior
    O.fill_bc(whole, bc)
    dt = 0.8 / DX / C0
    ref = ws.Level([dict(mx=DX, my=DY, dx=1 / DX, dy=1 / DX, bc=bc)], [(RHO, KB)])
    ref.upload(0, whole)
    for _ in range(6):
        ref.step(dt, read_cfl=False)
    R = ref.download(0)
    ref.close()
    layouts = [([(DX, DY)], [(0, 0)]), ([(1, DY)] * DX, [(x, 0) for x in range(DX)])]
    for shapes, origins in layouts:
        qs = tiles_of(interior, shapes, origins, (DX, DY), periodic)
        lev = tiled_level(ws, shapes, origins, (DX, DY), periodic, qs)
        for _ in range(6):
            lev.step(dt, read_cfl=False)
        for k, ((mx, my), (x0, y0)) in enumerate(zip(shapes, origins)):
            assert np.array_equal(lev.download(k), R[:, y0:y0 + my + 4, x0:x0 + mx + 4]), (len(shapes), k)
        lev.close()


def test_tiled_level_in_a_heterogeneous_medium_equals_single_patch(ws):
    """A 2x2 tiling of a layered, perturbed medium (each tile's medium taken
    from the domain's padded arrays, ghosts included), extrapolating sides:
    six steps equal the domain as one patch bitwise."""
    import workloads

    DX, DY = 70, 52
    rho, K = workloads.layered_medium(DX, DY)
    interior = domain_state(DX, DY, seed=9)
    whole = np.zeros((3, DY + 4, DX + 4))
    whole[:, 2:-2, 2:-2] = interior
    O.fill_bc(whole, "extrap")
    one = ws.Level([dict(mx=DX, my=DY, dx=1 / DX, dy=1 / DX, bc="extrap")], [(RHO, KB)])
    one.set_medium(0, rho, K)
    one.upload(0, whole)
    shapes, origins = [(30, 20), (40, 20), (30, 32), (40, 32)], [(0, 0), (30, 0), (0, 20), (30, 20)]
    qs = tiles_of(interior, shapes, origins, (DX, DY), (False, False))
    lev = ws.Level([dict(mx=mx, my=my, dx=1 / DX, dy=1 / DX) for (mx, my) in shapes], [(RHO, KB)])
    lev.link(origins, (DX, DY), (False, False))
    for k, ((mx, my), (x0, y0)) in enumerate(zip(shapes, origins)):
        lev.set_medium(k, rho[y0:y0 + my + 4, x0:x0 + mx + 4], K[y0:y0 + my + 4, x0:x0 + mx + 4])
        lev.upload(k, qs[k])
    dt = 0.8 / DX / float(np.sqrt(K / rho).max())
    for _ in range(6):
        c1 = one.step(dt)
        c2 = lev.step(dt)
        assert c1 == c2
    R = one.download(0)
    for k, ((mx, my), (x0, y0)) in enumerate(zip(shapes, origins)):
        assert np.array_equal(lev.download(k), R[:, y0:y0 + my + 4, x0:x0 + mx + 4]), k
    lev.close()
    one.close()
