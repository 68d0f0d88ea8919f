"""Input generators for the five acoustics workloads (seeded, synthetic).

The physical setting follows the paper's benchmark (Sec. 4.1): linear 2D
acoustics in a homogeneous medium, a ring-shaped pressure perturbation that
expands radially, outflow boundaries, double precision.  The sizes are
synthetic stand-ins for the paper's AMR run:

* ``uniform_patch(128)``  -- one 128x128 patch, rho=1, K=4, 100 steps at CFL 0.9;
* ``uniform_patch(2048)`` -- one 2048x2048 grid, 500 steps at CFL 0.9;
* ``amr_level_batch()``   -- ~3000 patches on 3 levels (ratio 4) over the ring;
* ``ensemble()``          -- 64 independent problems of uneven sizes;
* ``adjoint_setup()``     -- 512x512, fixed dt, 16 receivers, shifted target;
* ``two_level_layout()``  -- a 1024x1024 coarse grid and ratio-4 fine patches
  over the ring's annulus, for the composite step with the conservation fix;
* ``three_level_layout()`` -- 512x512, ratio-4 level-1 patches over the
  annulus and ratio-4 level-2 patches inside them near the ring;
* ``layered_medium()``    -- per-cell rho, K of a heterogeneous medium (two
  slanted interfaces and a seeded +-10% perturbation) for the variable-
  coefficient step.

A patch state is a C-contiguous float64 array (3, my+4, mx+4): components
(p, u, v), two ghost layers on each side, x fastest.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

RING_RADIUS = 0.25
RING_HALF_WIDTH = 0.1


def radial_pulse(x, y, xc=0.5, yc=0.5):
    """Initial pressure: p = 1 + cos(pi (r - 0.25) / 0.1) where |r - 0.25| < 0.1,
    else 1, with r measured from (xc, yc).  Taken literally, this jumps from 0
    back to 1 at the two rims of the ring."""
    r = np.hypot(np.asarray(x, np.float64) - xc, np.asarray(y, np.float64) - yc)
    d = r - RING_RADIUS
    return np.where(np.abs(d) < RING_HALF_WIDTH,
                    1.0 + np.cos(np.pi * d / RING_HALF_WIDTH), 1.0)


def padded_centres(mx, my, xlo, ylo, dx, dy):
    """Cell-centre coordinates of every padded cell (ghosts included).
    Returns (X, Y) of shape (my+4, mx+4)."""
    xs = xlo + (np.arange(-2, mx + 2, dtype=np.float64) + 0.5) * dx
    ys = ylo + (np.arange(-2, my + 2, dtype=np.float64) + 0.5) * dy
    return np.meshgrid(xs, ys, indexing="xy")


def padded_state(mx, my, xlo, ylo, dx, dy, xc=0.5, yc=0.5):
    """Radial-pulse state evaluated at every padded cell centre, u = v = 0."""
    X, Y = padded_centres(mx, my, xlo, ylo, dx, dy)
    q = np.zeros((3, my + 4, mx + 4), np.float64)
    q[0] = radial_pulse(X, Y, xc, yc)
    return q


@dataclasses.dataclass
class PatchSpec:
    """One rectangular patch: mx x my cells, lower-left corner (xlo, ylo)."""
    mx: int
    my: int
    xlo: float
    ylo: float
    dx: float
    dy: float
    level: int = 1
    instance: int = 0


def uniform_patch(n, xc=0.5, yc=0.5):
    """Single n x n patch on the unit square with the radial pulse."""
    spec = PatchSpec(n, n, 0.0, 0.0, 1.0 / n, 1.0 / n)
    return spec, padded_state(n, n, 0.0, 0.0, spec.dx, spec.dy, xc, yc)


def plane_wave_state(mx, my, kx, ky, Z, t=0.0, c=1.0, amp=0.5, periodic_len=1.0):
    """Smooth oblique plane wave p = 1 + amp sin(2 pi (kx x + ky y - |k| c t)),
    (u, v) = (p - 1)/Z * k/|k| on the unit square, evaluated at the padded cell
    centres (cell averages are approximated by centre values).  Used only as a
    test input and exact solution: a right-going simple wave of the acoustics
    system translates at speed c along k."""
    dx, dy = periodic_len / mx, periodic_len / my
    X, Y = padded_centres(mx, my, 0.0, 0.0, dx, dy)
    kn = math.hypot(kx, ky)
    phase = 2.0 * np.pi * (kx * X + ky * Y - kn * c * t)
    pp = amp * np.sin(phase)
    q = np.zeros((3, my + 4, mx + 4), np.float64)
    q[0] = 1.0 + pp
    q[1] = pp / Z * (kx / kn)
    q[2] = pp / Z * (ky / kn)
    return q


# ---------------------------------------------------------------------------
# Synthetic AMR level batch: 3 levels, refinement ratio 4, ~3000 patches
# ---------------------------------------------------------------------------

#: Half-width of the finest level's annulus around the ring radius 0.25.  The
#: annulus 0.165 <= r <= 0.335 yields ~2000 patches in total; it was widened
#: (this is the only tuned value) until the seeded batch held 3000 +- 10 %
#: patches in total.
AMR_LEVEL3_HALF_WIDTH = 0.135

_AMR_LEVELS = (
    # (level, cells per unit length, annulus (r_lo, r_hi) or None = everything)
    (1, 256, None),
    (2, 1024, (0.10, 0.40)),
    (3, 4096, "level3"),
)


def _strip_pack(rng, n_per_unit, box_lo, box_hi, keep, level):
    """Walk the box in strips 64 cells high; inside a strip draw patch width and
    height from U{16..64} left to right; keep a patch when ``keep`` accepts its
    centre.  Indices are cells of this level's grid."""
    dx = 1.0 / n_per_unit
    i_lo = int(math.floor(box_lo * n_per_unit))
    i_hi = int(math.ceil(box_hi * n_per_unit))
    patches = []
    j = i_lo
    while j < i_hi:
        i = i_lo
        while i < i_hi:
            w = int(rng.integers(16, 65))
            h = int(rng.integers(16, 65))
            w = min(w, i_hi - i)
            h = min(h, i_hi - j)
            if w >= 1 and h >= 1:
                xc = (i + 0.5 * w) * dx
                yc = (j + 0.5 * h) * dx
                if keep(xc, yc):
                    patches.append(PatchSpec(w, h, i * dx, j * dx, dx, dx, level))
            i += w
        j += 64
    return patches


def amr_level_batch(seed=18083, level3_half_width=AMR_LEVEL3_HALF_WIDTH, max_levels=3):
    """Patches of a synthetic 3-level hierarchy (ratio 4) over the ring.

    Level 1: 256^2 cells over the unit square (all patches kept).
    Level 2: dx = 1/1024, patches whose centre lies in 0.10 <= r <= 0.40.
    Level 3: dx = 1/4096, centre within ``level3_half_width`` of r = 0.25.
    Returns a list of lists of PatchSpec, one list per level.  Every patch's
    cells, ghosts included, are filled from the radial pulse at t = 0 by
    ``padded_state``; its ghosts then stay frozen.
    """
    rng = np.random.default_rng(seed)
    levels = []
    for level, n, ann in _AMR_LEVELS[:max_levels]:
        if ann is None:
            lo, hi = 0.0, 1.0
            keep = lambda x, y: True  # noqa: E731
        else:
            if ann == "level3":
                ann = (RING_RADIUS - level3_half_width, RING_RADIUS + level3_half_width)
            r_lo, r_hi = ann
            lo, hi = 0.5 - r_hi, 0.5 + r_hi

            def keep(x, y, r_lo=r_lo, r_hi=r_hi):
                r = math.hypot(x - 0.5, y - 0.5)
                return r_lo <= r <= r_hi
        levels.append(_strip_pack(rng, n, lo, hi, keep, level))
    return levels


# ---------------------------------------------------------------------------
# Ensemble of independent problems
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class EnsembleInstance:
    mx: int
    my: int
    xc: float
    yc: float
    K: float
    rho: float

    @property
    def dx(self):
        return 1.0 / self.mx

    @property
    def dy(self):
        return 1.0 / self.my

    def state(self):
        return padded_state(self.mx, self.my, 0.0, 0.0, self.dx, self.dy, self.xc, self.yc)


def ensemble(seed=18084, n=64, lo=128, hi=512):
    """n instances; each draws mx, my ~ U{lo..hi}, centre ~ U(0.4, 0.6)^2,
    K ~ U(1, 9), rho ~ U(0.5, 2), in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        mx = int(rng.integers(lo, hi + 1))
        my = int(rng.integers(lo, hi + 1))
        xc, yc = (float(v) for v in rng.uniform(0.4, 0.6, size=2))
        K = float(rng.uniform(1.0, 9.0))
        rho = float(rng.uniform(0.5, 2.0))
        out.append(EnsembleInstance(mx, my, xc, yc, K, rho))
    return out


# ---------------------------------------------------------------------------
# Adjoint workload
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class AdjointSetup:
    n: int
    steps: int
    dt: float
    receivers: np.ndarray  # (nr, 2) int: (i, j)
    target_centre: tuple
    checkpoint_every: int

    @property
    def dx(self):
        return 1.0 / self.n

    def p0(self):
        q = padded_state(self.n, self.n, 0.0, 0.0, self.dx, self.dx)
        return q[0, 2:-2, 2:-2].copy()

    def target_p0(self):
        q = padded_state(self.n, self.n, 0.0, 0.0, self.dx, self.dx, *self.target_centre)
        return q[0, 2:-2, 2:-2].copy()


def adjoint_setup(seed=18085, n=512, steps=200, courant=0.8, c=2.0, n_receivers=16,
                  checkpoint_every=20):
    """Fixed dt = courant * dx / c; 16 distinct receiver cells drawn uniformly
    over the interior, then the target pulse centre shifted by U(-0.05, 0.05)^2."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n * n, size=n_receivers, replace=False)
    rec = np.stack([flat % n, flat // n], axis=1).astype(np.int64)
    off = rng.uniform(-0.05, 0.05, size=2)
    dt = courant * (1.0 / n) / c
    return AdjointSetup(n, steps, dt, rec, (0.5 + float(off[0]), 0.5 + float(off[1])),
                        checkpoint_every)


def two_level_layout(n=1024, size=30, gap=3, r_lo=0.15, r_hi=0.35):
    """Fine patches of size x size coarse cells (at ratio 4, 120 x 120 fine
    cells: two 60-column MARCH segments) on a pitch of size + gap over
    the n x n coarse grid of the unit square, kept where any of the patch's
    coarse-cell centres lies in the annulus r_lo <= r <= r_hi around the
    ring's centre (0.5, 0.5).  Returns a list of (ci0, cj0, ncx, ncy)."""
    pitch = size + gap
    rects = []
    for cj0 in range(2, n - size - 1, pitch):
        for ci0 in range(2, n - size - 1, pitch):
            xs = (ci0 + np.arange(size) + 0.5) / n - 0.5
            ys = (cj0 + np.arange(size) + 0.5) / n - 0.5
            rr = np.hypot(xs[None, :], ys[:, None])
            if np.any((rr >= r_lo) & (rr <= r_hi)):
                rects.append((ci0, cj0, size, size))
    return rects


def three_level_layout(n=512, size=30, gap=3, r=4, r_lo=0.15, r_hi=0.35, r2_lo=0.2, r2_hi=0.3):
    """Level 1: ``two_level_layout(n, size, gap, r_lo, r_hi)``.  Level 2: in
    each level-1 patch (r*size cells a side), patches of size x size level-1
    cells on a pitch of size + gap starting 2 cells in, kept where any of their
    level-1 cell centres lies in r2_lo <= r <= r2_hi.  Returns (level-1 rects,
    level-2 places (parent, ci0, cj0, ncx, ncy))."""
    l1 = two_level_layout(n, size, gap, r_lo, r_hi)
    dx1 = 1.0 / (n * r)
    l2 = []
    m = r * size
    for k, (ci0, cj0, _, _) in enumerate(l1):
        for b0 in range(2, m - size - 1, size + gap):
            for a0 in range(2, m - size - 1, size + gap):
                xs = ci0 / n + (a0 + np.arange(size) + 0.5) * dx1 - 0.5
                ys = cj0 / n + (b0 + np.arange(size) + 0.5) * dx1 - 0.5
                rr = np.hypot(xs[None, :], ys[:, None])
                if np.any((rr >= r2_lo) & (rr <= r2_hi)):
                    l2.append((k, a0, b0, size, size))
    return l1, l2


def layered_medium(mx, my, seed=18086):
    """rho and K per padded cell of the unit square: three layers separated by
    the lines x + 0.3 y = 0.45 and x - 0.2 y = 0.75 (impedances 2, 3 and 1.2;
    sound speeds 2, 1.2 and 3), each cell perturbed by a factor U(0.9, 1.1)
    in rho and in K.  Returns (rho, K), each (my+4, mx+4)."""
    rng = np.random.default_rng(seed)
    X, Y = padded_centres(mx, my, 0.0, 0.0, 1.0 / mx, 1.0 / my)
    layer = (X + 0.3 * Y > 0.45).astype(int) + (X - 0.2 * Y > 0.75).astype(int)
    rho = np.choose(layer, [1.0, 2.5, 0.4])
    K = np.choose(layer, [4.0, 3.6, 3.6])
    rho = rho * rng.uniform(0.9, 1.1, size=rho.shape)
    K = K * rng.uniform(0.9, 1.1, size=K.shape)
    return np.ascontiguousarray(rho), np.ascontiguousarray(K)
