"""Pins of the oracle's two-level composite step with the conservation fix.

What pins it (none retypes the fix): the composite total of p, u, v is
conserved to rounding on a periodic coarse patch (and is not without the fix,
so the pin has teeth); with refinement ratio 1 the composite equals the plain
single-level step bitwise; the ghost interpolation is conservative (the mean
over a coarse cell's r x r sub-cells is the coarse value), exact for linear
data and bounded by the neighbours' values; a constant state is preserved;
and a symmetric layout gives a transpose- and rotation-symmetric result, which
ties the four sides' fixes to each other.  Each case also takes a mutated copy
of the module (``mod``) so planted mistakes can be checked against these pins.
"""

import numpy as np
import pytest

import oracle.amr as amr_mod
import oracle.oracle as O

RHO, KB = 1.0, 4.0


def smooth(X, Y):
    r = np.hypot(X - 0.45, Y - 0.55)
    p = 1.0 + 0.5 * np.exp(-((r / 0.12) ** 2))
    return np.stack([p, 0.1 * np.sin(2 * np.pi * X), 0.1 * np.cos(2 * np.pi * Y)])


def coarse_state(n, fn):
    xc = (np.arange(-2, n + 2) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    return np.ascontiguousarray(fn(X, Y), dtype=np.float64)


def run_composite(mod, n, rects, r, cycles, fn=smooth, bc="periodic", fix=True, cfl=0.8):
    qc = coarse_state(n, fn)
    fines = mod.init_fines(qc, rects, r, fn)
    O.fill_bc(qc, bc)
    s0 = mod.composite_sums(qc, 1 / n, 1 / n)
    dt = cfl / n / 2.0
    q, fs = qc, fines
    for _ in range(cycles):
        q, fs = mod.two_level_step(q, fs, 1 / n, 1 / n, dt, RHO, KB, r, bc=bc, fix=fix)
    return qc, fines, q, fs, s0, mod.composite_sums(q, 1 / n, 1 / n)


@pytest.mark.parametrize("r", [2, 4])
def test_composite_conserves(r, mod=amr_mod):
    """Periodic coarse 32^2 with two fine patches, 8 composite steps: the
    composite totals are constant to rounding; without the fix they drift."""
    rects = [(6, 8, 8, 10), (20, 5, 6, 6)]
    _, _, _, _, s0, s1 = run_composite(mod, 32, rects, r, 8)
    scale = np.abs(s0).max()
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale
    if mod is amr_mod:
        _, _, _, _, t0, t1 = run_composite(mod, 32, rects, r, 8, fix=False)
        assert np.abs(t1 - t0).max() > 1e-7 * scale


def test_ratio_one_equals_single_level_step(mod=amr_mod):
    n = 24
    rects = [(5, 6, 7, 9), (15, 4, 5, 12)]
    qc, fines, q, fs, _, _ = run_composite(mod, n, rects, 1, 5, bc="extrap")
    p = qc.copy()
    dt = 0.8 / n / 2.0
    for _ in range(5):
        p, _, _ = O.step(p, 1 / n, 1 / n, dt, RHO, KB, "mc")
        O.fill_bc(p, "extrap")
    assert np.array_equal(q, p)
    for f in fs:
        sub = p[:, 2 + f.cj0:2 + f.cj0 + f.ncy, 2 + f.ci0:2 + f.ci0 + f.ncx]
        assert np.array_equal(f.q[:, 2:-2, 2:-2], sub)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_interpolation_conservative_linear_exact_and_bounded(r, mod=amr_mod):
    rng = np.random.default_rng(40 + r)
    Q = rng.normal(size=(3, 10, 10))
    offs = (np.arange(r) + 0.5) / r - 0.5
    for cj in range(1, 5):
        for ci in range(1, 5):
            vals = np.array([[mod.interp_cell(Q, ci, cj, x, y) for x in offs] for y in offs])
            assert np.allclose(vals.reshape(-1, 3).mean(axis=0), Q[:, cj + 2, ci + 2],
                               rtol=0, atol=1e-14)
            # along each axis the value stays between the cell's neighbours
            # in that direction (the MC limit keeps |slope|/2 below both
            # one-sided differences)
            for x in offs:
                vx = mod.interp_cell(Q, ci, cj, x, 0.0)
                row = Q[:, cj + 2, ci + 1:ci + 4]
                assert np.all(vx >= row.min(axis=1) - 1e-14) and np.all(vx <= row.max(axis=1) + 1e-14)
                vy = mod.interp_cell(Q, ci, cj, 0.0, x)
                col = Q[:, cj + 1:cj + 4, ci + 2]
                assert np.all(vy >= col.min(axis=1) - 1e-14) and np.all(vy <= col.max(axis=1) + 1e-14)
    # linear data: reproduced exactly at any offset
    J, I = np.mgrid[0:10, 0:10]
    L = np.stack([0.3 + 0.2 * I - 0.1 * J, -0.4 * I + 0.05 * J, 0.7 * J + 0.0 * I]).astype(float)
    for (x, y) in [(0.25, -0.25), (-0.375, 0.125), (0.0, 0.0)]:
        v = mod.interp_cell(L, 3, 4, x, y)
        exact = L[:, 6, 5] + x * np.array([0.2, -0.4, 0.0]) + y * np.array([-0.1, 0.05, 0.7])
        assert np.allclose(v, exact, rtol=0, atol=1e-14)


def test_mc_slope_bounds_a_step(mod=amr_mod):
    """At a jump the limited slope keeps every sub-cell value inside the two
    neighbours' range in that direction (an unlimited slope overshoots)."""
    Q = np.zeros((3, 7, 7))
    Q[:, :, 4:] = 3.0  # coarse cell (1, 1) (padded column 3) is 0, its right neighbour 3
    for x in (-0.5 + 1e-9, 0.5 - 1e-9):
        v = mod.interp_cell(Q, 1, 1, x, 0.0)
        assert np.all(v >= 0.0 - 1e-12) and np.all(v <= 3.0 + 1e-12), v


def test_constant_state_preserved(mod=amr_mod):
    const = lambda X, Y: np.stack([np.full_like(X, 1.5), np.full_like(X, -0.25),
                                   np.full_like(X, 0.5)])
    qc, _, q, fs, _, _ = run_composite(mod, 20, [(5, 5, 6, 8)], 2, 3, fn=const, bc="extrap")
    assert np.array_equal(q, qc)
    for f in fs:
        assert np.all(f.q[0, 2:-2, 2:-2] == 1.5) and np.all(f.q[1, 2:-2, 2:-2] == -0.25)


def test_symmetric_layout_gives_symmetric_result(mod=amr_mod):
    """Centred pulse, one centred fine patch, extrapolation: after 6 composite
    steps the coarse state is symmetric under transposition (p, u, v) ->
    (p^T, v^T, u^T) and under a 90-degree rotation, to 1e-12."""
    n = 24
    pulse = lambda X, Y: np.stack([1.0 + np.exp(-((np.hypot(X - 0.5, Y - 0.5) / 0.15) ** 2)),
                                   0.0 * X, 0.0 * X])
    _, _, q, fs, _, _ = run_composite(mod, n, [(8, 8, 8, 8)], 2, 6, fn=pulse, bc="extrap")
    p, u, v = (q[m, 2:-2, 2:-2] for m in range(3))
    scale = np.abs(q).max()
    assert np.abs(p - p.T).max() <= 1e-12 * scale
    assert np.abs(u - v.T).max() <= 1e-12 * scale
    N = p.shape[0]
    i = np.arange(N)[None, :]
    j = np.arange(N)[:, None]
    assert np.abs(p - p[N - 1 - i, j]).max() <= 1e-12 * scale
    assert np.abs(u + v[N - 1 - i, j]).max() <= 1e-12 * scale
    assert np.abs(v - u[N - 1 - i, j]).max() <= 1e-12 * scale
    fp = fs[0].q[:, 2:-2, 2:-2]
    assert np.abs(fp[0] - fp[0].T).max() <= 1e-12 * scale
    # and the fix acted (the patch's edges carry flux)
    assert np.abs(p - 1.0).max() > 0.05


def test_layout_checks(mod=amr_mod):
    bad = [mod.FinePatch(1, 5, 4, 4, np.zeros((3, 12, 12)))]
    with pytest.raises(ValueError):
        mod.check_layout(20, 20, bad, 2)
    overlapping = [mod.FinePatch(3, 3, 4, 4, np.zeros((3, 12, 12))),
                   mod.FinePatch(6, 3, 4, 4, np.zeros((3, 12, 12)))]
    with pytest.raises(ValueError):
        mod.check_layout(20, 20, overlapping, 2)


# --------------------------------------------------------------------------
# Three levels: the recursion of the composite step
# --------------------------------------------------------------------------

def three_levels(mod, n, r, fn=smooth):
    """Level 0: n^2; level 1: two patches; level 2: patches nested in them."""
    qc = coarse_state(n, fn)
    l1 = mod.init_fines(qc, [(4, 4, 10, 12), (19, 6, 8, 8)], r, fn)
    # level-2 patches in level-1 cells: fine states from fn at their centres
    l2 = []
    for parent, (ci0, cj0, ncx, ncy) in [(0, (2, 2, 3, 3)), (1, (2, 2, 4, 3)), (0, (2, 8, 4, 2))]:
        P = l1[parent]
        dx1 = 1.0 / (n * r)
        x0 = P.ci0 / n + ci0 * dx1
        y0 = P.cj0 / n + cj0 * dx1
        x = x0 + (np.arange(-2, r * ncx + 2) + 0.5) * dx1 / r
        y = y0 + (np.arange(-2, r * ncy + 2) + 0.5) * dx1 / r
        X, Y = np.meshgrid(x, y, indexing="xy")
        q = np.ascontiguousarray(fn(X, Y), dtype=np.float64)
        fp = mod.FinePatch(ci0, cj0, ncx, ncy, q, parent)
        mod.average_down(P.q, fp, q, r)
        l2.append(fp)
    for P in l1:  # level-1 cells covered by level 2 changed: refresh level 0
        mod.average_down(qc, P, P.q, r)
    for P in l1:
        P.parent = 0
    return qc, [l1, l2]


def test_three_levels_conserve(mod=amr_mod):
    n, r = 32, 2
    qc, levels = three_levels(mod, n, r)
    O.fill_bc(qc, "periodic")
    s0 = mod.composite_sums(qc, 1 / n, 1 / n)
    q, lv = qc, levels
    dt = 0.8 / n / 2.0
    for _ in range(4):
        q, lv = mod.multi_level_step(q, lv, 1 / n, 1 / n, dt, RHO, KB, r, bc="periodic")
    s1 = mod.composite_sums(q, 1 / n, 1 / n)
    scale = np.abs(s0).max()
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale
    # the finest level moved
    assert np.abs(lv[1][0].q - levels[1][0].q).max() > 1e-4


def test_one_level_recursion_equals_two_level_step(mod=amr_mod):
    n, r = 32, 2
    rects = [(6, 8, 8, 10), (20, 5, 6, 6)]
    qc = coarse_state(n, smooth)
    fines = mod.init_fines(qc, rects, r, smooth)
    O.fill_bc(qc, "extrap")
    dt = 0.8 / n / 2.0
    a, fa = mod.two_level_step(qc, fines, 1 / n, 1 / n, dt, RHO, KB, r, bc="extrap")
    b, lb = mod.multi_level_step(qc, [fines], 1 / n, 1 / n, dt, RHO, KB, r, bc="extrap")
    assert np.array_equal(a, b)
    for x, y in zip(fa, lb[0]):
        assert np.array_equal(x.q, y.q)


def test_three_levels_ratio_one_equal_single_level(mod=amr_mod):
    n, r = 32, 1
    qc, levels = three_levels(mod, n, r)
    O.fill_bc(qc, "extrap")
    p = qc.copy()
    q, lv = qc, levels
    dt = 0.8 / n / 2.0
    for _ in range(3):
        q, lv = mod.multi_level_step(q, lv, 1 / n, 1 / n, dt, RHO, KB, r, bc="extrap")
        p, _, _ = O.step(p, 1 / n, 1 / n, dt, RHO, KB, "mc")
        O.fill_bc(p, "extrap")
    assert np.array_equal(q, p)
    for P in lv[0]:
        assert np.array_equal(P.q[:, 2:-2, 2:-2],
                              p[:, 2 + P.cj0:2 + P.cj0 + P.ncy, 2 + P.ci0:2 + P.ci0 + P.ncx])


# --------------------------------------------------------------------------
# Touching fine patches: same-level ghosts and the fix at covered cells
# --------------------------------------------------------------------------

def _composite_steps(mod, driver, n, rects, r, steps, bc="extrap"):
    qc = coarse_state(n, smooth)
    fines = mod.init_fines(qc, rects, r, smooth)
    O.fill_bc(qc, bc)
    dt = 0.8 / n / 2.0
    q, fs = qc, fines
    for _ in range(steps):
        if driver == "two":
            q, fs = mod.two_level_step(q, fs, 1 / n, 1 / n, dt, RHO, KB, r, bc=bc)
        else:
            q, lv = mod.multi_level_step(q, [fs], 1 / n, 1 / n, dt, RHO, KB, r, bc=bc)
            fs = lv[0]
    return q, fs


def _assemble(fs, r):
    """The fine interiors of patches that tile a rectangle, as one array."""
    i0 = min(f.ci0 for f in fs)
    j0 = min(f.cj0 for f in fs)
    i1 = max(f.ci0 + f.ncx for f in fs)
    j1 = max(f.cj0 + f.ncy for f in fs)
    out = np.full((3, r * (j1 - j0), r * (i1 - i0)), np.nan)
    for f in fs:
        a, b = r * (f.ci0 - i0), r * (f.cj0 - j0)
        out[:, b:b + r * f.ncy, a:a + r * f.ncx] = f.q[:, 2:-2, 2:-2]
    return out


SPLITS = {
    "x": [(6, 7, 4, 8), (10, 7, 5, 8)],
    "y": [(6, 7, 9, 3), (6, 10, 9, 5)],
    "quadrants": [(6, 7, 4, 3), (10, 7, 5, 3), (6, 10, 4, 5), (10, 10, 5, 5)],
}


@pytest.mark.parametrize("driver", ["two", "multi"])
@pytest.mark.parametrize("split", sorted(SPLITS))
@pytest.mark.parametrize("r", [2, 3])
def test_split_patch_equals_whole_patch(r, split, driver, mod=amr_mod):
    """A fine patch cut into touching pieces gives the composite of the whole
    patch: the pieces see each other's cells as ghosts (the quadrants also at
    the corners), the cut edges carry no fix, and the covered coarse cells
    take the means of their fine cells."""
    n = 24
    whole = [(6, 7, 9, 8)]
    qa, fa = _composite_steps(mod, driver, n, whole, r, 3)
    qb, fb = _composite_steps(mod, driver, n, SPLITS[split], r, 3)
    scale = np.abs(qa).max()
    assert np.abs(qa - qb).max() <= 1e-13 * scale, np.abs(qa - qb).max()
    fw, fs = _assemble(fa, r), _assemble(fb, r)
    assert not np.isnan(fs).any()
    assert np.abs(fw - fs).max() <= 1e-13 * scale, np.abs(fw - fs).max()


TOUCHING = [(4, 4, 5, 6), (9, 4, 4, 6), (14, 4, 4, 6), (4, 10, 3, 4)]
# (9, 4) touches (4, 4) on its right; coarse column 13 lies between (9, 4) and
# (14, 4), so its cells border two patches; cell (7, 10) borders (4, 4) below
# and (4, 10) on its left (a concave corner).


@pytest.mark.parametrize("r", [2, 4])
def test_touching_patches_conserve(r, mod=amr_mod):
    _, _, _, _, s0, s1 = run_composite(mod, 24, TOUCHING, r, 6)
    scale = np.abs(s0).max()
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s1 - s0) / scale


def test_covered_cells_hold_the_means_of_their_fine_cells(mod=amr_mod):
    r = 2
    for driver in ("two", "multi"):
        q, fs = _composite_steps(mod, driver, 24, TOUCHING, r, 2, bc="periodic")
        scale = np.abs(q).max()
        for f in fs:
            blk = f.q[:, 2:-2, 2:-2].reshape(3, f.ncy, r, f.ncx, r).mean(axis=(2, 4))
            cov = q[:, 2 + f.cj0:2 + f.cj0 + f.ncy, 2 + f.ci0:2 + f.ci0 + f.ncx]
            assert np.abs(cov - blk).max() <= 1e-14 * scale, (driver, np.abs(cov - blk).max())


def test_touching_layout_accepted_overlap_refused(mod=amr_mod):
    z = lambda ncx, ncy: np.zeros((3, 2 * ncy + 4, 2 * ncx + 4))
    mod.check_layout(20, 20, [mod.FinePatch(3, 3, 4, 4, z(4, 4)),
                              mod.FinePatch(7, 3, 4, 4, z(4, 4)),
                              mod.FinePatch(11, 7, 2, 2, z(2, 2))], 2)
    with pytest.raises(ValueError):
        mod.check_layout(20, 20, [mod.FinePatch(3, 3, 4, 4, z(4, 4)),
                                  mod.FinePatch(6, 6, 4, 4, z(4, 4))], 2)
