"""Pins of the oracle's ghost exchange for a level whose patches tile a
domain (oracle/tiled.py).

None retypes the exchange: on a single patch covering the domain it equals
numpy's own padding (``np.pad`` with mode "wrap" for a periodic direction,
"edge" for an extrapolating one, corners included); a domain cut into
tiles (uneven, one tile a single cell wide, a brick layout with
T-junctions) and stepped with the exchange gives, bitwise, the single-patch
step whose ghosts come from that padding (and from the C oracle's own
periodic fill).  Each case also takes a copy of the module (``mod``) so
planted mistakes can be checked against these pins.
"""

import numpy as np
import pytest

import oracle.oracle as O
import oracle.tiled as tiled_mod

RHO, KB = 1.0, 4.0


def padded(interior, periodic):
    """Ghosts of a whole-domain state from numpy's padding, per axis."""
    mode_x = "wrap" if periodic[0] else "edge"
    mode_y = "wrap" if periodic[1] else "edge"
    a = np.pad(interior, ((0, 0), (0, 0), (2, 2)), mode=mode_x)
    return np.ascontiguousarray(np.pad(a, ((0, 0), (2, 2), (0, 0)), mode=mode_y))


def random_interior(DX, DY, seed):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid((np.arange(DX) + 0.5) / DX, (np.arange(DY) + 0.5) / DY, indexing="xy")
    p = 1.0 + 0.5 * np.exp(-((X - 0.4) ** 2 + (Y - 0.6) ** 2) / 0.02)
    return np.stack([p + 0.01 * rng.normal(size=X.shape), 0.1 * np.sin(2 * np.pi * Y),
                     0.05 * rng.normal(size=X.shape)])


def cut(interior, shapes, origins):
    qs = []
    for (mx, my), (x0, y0) in zip(shapes, origins):
        q = np.zeros((3, my + 4, mx + 4))
        q[:, 2:-2, 2:-2] = interior[:, y0:y0 + my, x0:x0 + mx]
        qs.append(q)
    return qs


@pytest.mark.parametrize("periodic", [(True, True), (False, False), (True, False), (False, True)])
def test_single_patch_exchange_is_numpy_padding(periodic, mod=tiled_mod):
    DX, DY = 13, 9
    interior = random_interior(DX, DY, 3)
    q = cut(interior, [(DX, DY)], [(0, 0)])
    mod.exchange_ghosts(q, [(0, 0)], (DX, DY), periodic)
    assert np.array_equal(q[0], padded(interior, periodic))


# (DX, DY), [(mx, my)], [(x0, y0)]
TILINGS = {
    "2x2_uneven": ((24, 20), [(10, 8), (14, 8), (10, 12), (14, 12)],
                   [(0, 0), (10, 0), (0, 8), (10, 8)]),
    "columns_one_wide": ((24, 20), [(11, 20), (1, 20), (12, 20)], [(0, 0), (11, 0), (12, 0)]),
    "bricks": ((24, 20), [(12, 7), (12, 7), (6, 6), (12, 6), (6, 6), (24, 7)],
               [(0, 0), (12, 0), (0, 7), (6, 7), (18, 7), (0, 13)]),
}


@pytest.mark.parametrize("periodic", [(True, True), (False, False), (True, False)])
@pytest.mark.parametrize("tiling", sorted(TILINGS))
def test_tiled_steps_equal_the_single_patch_step(tiling, periodic, mod=tiled_mod):
    (DX, DY), shapes, origins = TILINGS[tiling]
    interior = random_interior(DX, DY, 11)
    whole = padded(interior, periodic)
    if periodic == (True, True):  # the C oracle's own periodic fill agrees
        w2 = whole.copy()
        w2[:, :2] = w2[:, -2:] = 0.0
        assert np.array_equal(O.fill_bc(w2, "periodic"), whole)
    qs = mod.exchange_ghosts(cut(interior, shapes, origins), origins, (DX, DY), periodic)
    dt = 0.8 / max(DX, DY) / 2.0
    for _ in range(5):
        whole, _, _ = O.step(whole, 1 / DX, 1 / DY, dt, RHO, KB, "mc")
        whole = padded(whole[:, 2:-2, 2:-2], periodic)
        qs = [O.step(q, 1 / DX, 1 / DY, dt, RHO, KB, "mc")[0] for q in qs]
        mod.exchange_ghosts(qs, origins, (DX, DY), periodic)
    for q, (mx, my), (x0, y0) in zip(qs, shapes, origins):
        assert np.array_equal(q, whole[:, y0:y0 + my + 4, x0:x0 + mx + 4]), (x0, y0)


def test_tilings_are_checked(mod=tiled_mod):
    with pytest.raises(ValueError):  # a gap
        mod.owner_map([(10, 20), (13, 20)], [(0, 0), (11, 0)], (24, 20))
    with pytest.raises(ValueError):  # an overlap
        mod.owner_map([(12, 20), (13, 20)], [(0, 0), (11, 0)], (24, 20))
    with pytest.raises(ValueError):  # outside the domain
        mod.owner_map([(12, 20), (13, 20)], [(0, 0), (12, 0)], (24, 20))
    own = mod.owner_map([(12, 20), (12, 20)], [(0, 0), (12, 0)], (24, 20))
    assert (own[:, :12] == 0).all() and (own[:, 12:] == 1).all()
