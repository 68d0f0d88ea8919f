"""Two-level composite step with the conservation fix, FP64, plain numpy
around the C oracle's step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One coarse step of a coarse patch and the fine patches nested in it,
following the flow chart of the paper's Sec. 2.2 (advance the coarse patch,
advance each fine patch r times with ghosts from the coarse level, then
update the covered coarse cells and apply the conservation fix of Sec. 2.3):

1. coarse step Q_c^n -> Q_c^{n+1} over the whole coarse patch; the terms of
   eq. (2.3) at the coarse-fine interface edges are kept from Q_c^n;
2. for k = 0..r-1: the fine ghosts are filled from the coarse level at
   t_n + k dt/r (linear in time between Q_c^n and Q_c^{n+1}, then
   MC-limited linear in space inside the coarse cell that holds the ghost),
   the fine terms at the patch's boundary edges are accumulated, and the
   fine patch steps with dt/r (its ghosts frozen during the step);
3. updating: each covered coarse cell takes the mean of its r x r fine cells;
4. conservation fix (Sec. 2.3 eqs. for C1, C2, C3): each coarse cell next to
   a fine patch (outside it) replaces the coarse flux through their shared
   edge by the mean of the fine fluxes through it over the r fine steps.

The fix in fluctuation form, for a coarse cell O whose left edge is the
fine patch's right side (the configuration the paper writes out):
  O += dt/dx [ (1/r^2) sum_{k,b} (C1_{k,b} - A+dQ^_{k,b} + F~^_{k,b})
               + A+dQ_c - F~_c ]
with C1_{k,b} = A+dQ + A-dQ of the Riemann problem between Q_O^n (left) and
the fine ghost cell next to fine edge b at step k (right), i.e. f(ghost) -
f(Q_O^n); A+dQ^, F~^ at fine edge b of step k; A+dQ_c, F~_c at the coarse
edge of the coarse step.  The other three sides are the mirror images.  The
coarse F~_c enters with weight dt/dx (the printed 1/4 in front of it would
not conserve; the conservation pin decides).

Same-level ghosts: fine patches of one coarse patch may touch (they must not
overlap).  A fine ghost cell that lies in a sibling patch takes the sibling's
value at the same fine step (all fine patches advance in lockstep), every
other ghost comes from the coarse level as in step 2; a coarse cell covered by
a sibling takes no fix (updating sets it), and a coarse cell bordered by
several fine patches takes the fix of each.

Layout: states are padded (3, my+4, mx+4) arrays as in the C oracle.  A fine
patch covers coarse cells [ci0, ci0+ncx) x [cj0, cj0+ncy), so it has
r*ncx x r*ncy cells of size dx/r; patches lie at least 2 coarse cells inside
the coarse patch and do not overlap.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import oracle as O


@dataclass
class FinePatch:
    ci0: int
    cj0: int
    ncx: int
    ncy: int
    q: np.ndarray  # padded fine state (3, r*ncy+4, r*ncx+4)
    parent: int = 0  # index of the patch of the next coarser level it lies in


def check_layout(mxc, myc, fines, r):
    """The nesting and separation the composite step assumes."""
    if r < 1:
        raise ValueError("refinement ratio must be >= 1")
    for f in fines:
        if f.ncx < 1 or f.ncy < 1:
            raise ValueError("empty fine patch")
        if f.ci0 < 2 or f.cj0 < 2 or f.ci0 + f.ncx > mxc - 2 or f.cj0 + f.ncy > myc - 2:
            raise ValueError("fine patch must lie at least 2 coarse cells inside the coarse patch")
        if f.q.shape != (3, r * f.ncy + 4, r * f.ncx + 4):
            raise ValueError("fine state has the wrong shape")
    for a in range(len(fines)):
        for b in range(a + 1, len(fines)):
            fa, fb = fines[a], fines[b]
            gap_x = max(fb.ci0 - (fa.ci0 + fa.ncx), fa.ci0 - (fb.ci0 + fb.ncx))
            gap_y = max(fb.cj0 - (fa.cj0 + fa.ncy), fa.cj0 - (fb.cj0 + fb.ncy))
            if max(gap_x, gap_y) < 0:
                raise ValueError("fine patches must not overlap")


def covered_cells(fines):
    """The coarse cells (ci, cj) that some fine patch covers."""
    return {(f.ci0 + I, f.cj0 + J) for f in fines for I in range(f.ncx) for J in range(f.ncy)}


def mc_slope(a, b):
    """MC-limited slope from the one-sided differences a (left) and b (right):
    0 unless they share a sign, else the smallest of 2|a|, 2|b|, |a+b|/2."""
    s = np.where(a * b > 0.0, np.sign(a), 0.0)
    return s * np.minimum(np.minimum(2.0 * np.abs(a), 2.0 * np.abs(b)), 0.5 * np.abs(a + b))


def interp_cell(Qt, ci, cj, xi, eta):
    """Value at offset (xi, eta) (coarse-cell units, |xi|, |eta| < 1/2) from the
    centre of coarse interior cell (ci, cj) of the padded coarse state Qt:
    Q + xi sx + eta sy with MC-limited slopes."""
    I, J = ci + 2, cj + 2
    q0 = Qt[:, J, I]
    sx = mc_slope(q0 - Qt[:, J, I - 1], Qt[:, J, I + 1] - q0)
    sy = mc_slope(q0 - Qt[:, J - 1, I], Qt[:, J + 1, I] - q0)
    return q0 + xi * sx + eta * sy


def fill_fine_ghosts(qf, fp, Qt, r, siblings=()):
    """Every ghost cell of the fine patch: from the sibling that holds it, if
    one does, else from the coarse state Qt.  siblings: (FinePatch, current
    padded state) pairs of the other fine patches of the same coarse patch."""
    myf, mxf = qf.shape[1] - 4, qf.shape[2] - 4
    for j in range(-2, myf + 2):
        for i in range(-2, mxf + 2):
            if 0 <= i < mxf and 0 <= j < myf:
                continue
            # global fine index of the ghost, and the sibling that holds it
            gi, gj = r * fp.ci0 + i, r * fp.cj0 + j
            src = None
            for sp, sq in siblings:
                si, sj = gi - r * sp.ci0, gj - r * sp.cj0
                if 0 <= si < r * sp.ncx and 0 <= sj < r * sp.ncy:
                    src = sq[:, sj + 2, si + 2]
                    break
            if src is not None:
                qf[:, j + 2, i + 2] = src
                continue
            X = fp.ci0 + (i + 0.5) / r  # fine centre in coarse index units
            Y = fp.cj0 + (j + 0.5) / r
            ci, cj = math.floor(X), math.floor(Y)
            qf[:, j + 2, i + 2] = interp_cell(Qt, ci, cj, X - (ci + 0.5), Y - (cj + 0.5))


def average_down(qc, fp, qf, r):
    """Covered coarse cells take the mean of their r x r fine cells."""
    for J in range(fp.ncy):
        for I in range(fp.ncx):
            blk = qf[:, 2 + J * r:2 + (J + 1) * r, 2 + I * r:2 + (I + 1) * r]
            qc[:, 2 + fp.cj0 + J, 2 + fp.ci0 + I] = blk.reshape(3, -1).sum(axis=1) / (r * r)


def _fsum(direction, rho, K, ql, qr):
    """A+dQ + A-dQ (or B) of the Riemann problem (ql, qr): f(qr) - f(ql)."""
    _w, _s, am, ap = O.riemann_edge(direction, rho, K, ql, qr)
    return am + ap


def accumulate_fine(acc, fp, qf, Tf, qc_n, r, rho, K):
    """Add step k's fine-side terms at the patch's boundary edges.
    acc: dict side -> (n_edges, 3).  qc_n: coarse state at t_n."""
    myf, mxf = qf.shape[1] - 4, qf.shape[2] - 4
    for b in range(myf):
        J = fp.cj0 + b // r
        # left side: ghost column -1 is the left state; out cell (ci0-1, J)
        out = qc_n[:, J + 2, fp.ci0 - 1 + 2]
        g = qf[:, b + 2, 1]
        acc["left"][b] += _fsum(0, rho, K, out, g) + Tf["amx"][b, 0] + Tf["Fx"][b, 0]
        # right side: ghost column mxf is the right state; out cell (ci0+ncx, J)
        out = qc_n[:, J + 2, fp.ci0 + fp.ncx + 2]
        g = qf[:, b + 2, mxf + 2]
        acc["right"][b] += _fsum(0, rho, K, out, g) - Tf["apx"][b, mxf] + Tf["Fx"][b, mxf]
    for a in range(mxf):
        I = fp.ci0 + a // r
        out = qc_n[:, fp.cj0 - 1 + 2, I + 2]
        g = qf[:, 1, a + 2]
        acc["bottom"][a] += _fsum(1, rho, K, out, g) + Tf["amy"][0, a] + Tf["Gy"][0, a]
        out = qc_n[:, fp.cj0 + fp.ncy + 2, I + 2]
        g = qf[:, myf + 2, a + 2]
        acc["top"][a] += _fsum(1, rho, K, out, g) - Tf["apy"][myf, a] + Tf["Gy"][myf, a]


def apply_fix(qc, fp, acc, Tc, dt, dxc, dyc, r, covered=frozenset()):
    """Conservation fix of the coarse cells around one fine patch; an out
    cell in `covered` (covered by a sibling, so set by updating) is skipped."""
    w = 1.0 / (r * r)
    for J in range(fp.ncy):
        rows = slice(J * r, (J + 1) * r)
        e = fp.ci0  # left side: the out cell's right edge
        if (e - 1, fp.cj0 + J) not in covered:
            Pc = Tc["amx"][fp.cj0 + J, e] + Tc["Fx"][fp.cj0 + J, e]
            qc[:, fp.cj0 + J + 2, fp.ci0 - 1 + 2] -= dt / dxc * (w * acc["left"][rows].sum(axis=0) - Pc)
        e = fp.ci0 + fp.ncx  # right side: the out cell's left edge
        if (e, fp.cj0 + J) not in covered:
            Pc = -Tc["apx"][fp.cj0 + J, e] + Tc["Fx"][fp.cj0 + J, e]
            qc[:, fp.cj0 + J + 2, e + 2] += dt / dxc * (w * acc["right"][rows].sum(axis=0) - Pc)
    for I in range(fp.ncx):
        cols = slice(I * r, (I + 1) * r)
        f = fp.cj0  # bottom side: the out cell's top edge
        if (fp.ci0 + I, f - 1) not in covered:
            Pc = Tc["amy"][f, fp.ci0 + I] + Tc["Gy"][f, fp.ci0 + I]
            qc[:, fp.cj0 - 1 + 2, fp.ci0 + I + 2] -= dt / dyc * (w * acc["bottom"][cols].sum(axis=0) - Pc)
        f = fp.cj0 + fp.ncy  # top side: the out cell's bottom edge
        if (fp.ci0 + I, f) not in covered:
            Pc = -Tc["apy"][f, fp.ci0 + I] + Tc["Gy"][f, fp.ci0 + I]
            qc[:, f + 2, fp.ci0 + I + 2] += dt / dyc * (w * acc["top"][cols].sum(axis=0) - Pc)


def two_level_step(qc, fines, dxc, dyc, dt, rho, K, r, limiter="mc", bc="periodic", fix=True):
    """One composite coarse step.  qc: padded coarse state at t_n with its
    ghosts filled; fines: FinePatch list (states at t_n).  Returns the new
    coarse state (ghosts filled) and the new fine states (their ghosts hold
    the values of the last fill)."""
    mxc, myc = qc.shape[2] - 4, qc.shape[1] - 4
    check_layout(mxc, myc, fines, r)
    dxf, dyf, dtf = dxc / r, dyc / r, dt / r
    Tc = O.step_terms(qc, dxc, dyc, dt, rho, K, limiter)
    qc1, _, _ = O.step(qc, dxc, dyc, dt, rho, K, limiter)
    O.fill_bc(qc1, bc)
    new_q = [fp.q.copy() for fp in fines]
    accs = []
    for fp in fines:
        myf, mxf = r * fp.ncy, r * fp.ncx
        accs.append({"left": np.zeros((myf, 3)), "right": np.zeros((myf, 3)),
                     "bottom": np.zeros((mxf, 3)), "top": np.zeros((mxf, 3))})
    for k in range(r):
        # every fine patch's ghosts (siblings at step k), then every patch's step
        a = k / r
        Qt = (1.0 - a) * qc + a * qc1
        for c, fp in enumerate(fines):
            sibs = [(fines[d], new_q[d]) for d in range(len(fines)) if d != c]
            fill_fine_ghosts(new_q[c], fp, Qt, r, sibs)
        for c, fp in enumerate(fines):
            Tf = O.step_terms(new_q[c], dxf, dyf, dtf, rho, K, limiter)
            accumulate_fine(accs[c], fp, new_q[c], Tf, qc, r, rho, K)
            new_q[c] = O.step(new_q[c], dxf, dyf, dtf, rho, K, limiter)[0]
    qc2 = qc1.copy()
    for fp, qf in zip(fines, new_q):
        average_down(qc2, fp, qf, r)
    if fix:
        cov = covered_cells(fines)
        for fp, acc in zip(fines, accs):
            apply_fix(qc2, fp, acc, Tc, dt, dxc, dyc, r, cov)
    O.fill_bc(qc2, bc)
    return qc2, [FinePatch(fp.ci0, fp.cj0, fp.ncx, fp.ncy, q) for fp, q in zip(fines, new_q)]


def composite_sums(qc, dxc, dyc):
    """Sums of p, u, v times the coarse cell area over the coarse interior
    (covered cells hold the mean of their fine cells, so this is the
    composite solution's total)."""
    return qc[:, 2:-2, 2:-2].reshape(3, -1).sum(axis=1) * dxc * dyc


def init_fines(qc, fines_rect, r, fn):
    """Fine states from a point-value function fn(x, y) -> (3, ...) on the
    unit square (coarse cell size 1/mxc), and the covered coarse cells set to
    their means, so the composite starts consistent."""
    mxc, myc = qc.shape[2] - 4, qc.shape[1] - 4
    dxc, dyc = 1.0 / mxc, 1.0 / myc
    out = []
    for (ci0, cj0, ncx, ncy) in fines_rect:
        mxf, myf = r * ncx, r * ncy
        x = ci0 * dxc + (np.arange(-2, mxf + 2) + 0.5) * dxc / r
        y = cj0 * dyc + (np.arange(-2, myf + 2) + 0.5) * dyc / r
        X, Y = np.meshgrid(x, y, indexing="xy")
        q = np.ascontiguousarray(fn(X, Y), dtype=np.float64)
        fp = FinePatch(ci0, cj0, ncx, ncy, q)
        average_down(qc, fp, q, r)
        out.append(fp)
    return out


def multi_level_step(q0, levels, dx0, dy0, dt, rho, K, r, limiter="mc", bc="periodic"):
    """One composite step of a hierarchy: level 0 is the single padded patch
    q0 (ghosts filled); levels[l-1] lists the FinePatch objects of level l,
    each nested (ratio r) in patch `parent` of level l-1, with coordinates in
    its parent's cells.  Level l advances r^l steps of dt / r^l: every step of
    a level is its step followed, r times, by its children's ghost fill from
    it (between its old and new state), their boundary terms and their own
    composite step; then updating and the fix of the level's cells around its
    children (the recursion of the paper's flow chart, Sec. 2.2).  Returns the
    new level-0 state and the new levels."""
    states = [[q0.copy()]] + [[p.q.copy() for p in lv] for lv in levels]
    geo = [None] + [list(lv) for lv in levels]
    for l in range(1, len(geo)):
        by_parent = {}
        for p in geo[l]:
            by_parent.setdefault(p.parent, []).append(p)
        for k, ps in by_parent.items():
            P = states[l - 1][k]
            check_layout(P.shape[2] - 4, P.shape[1] - 4, [FinePatch(p.ci0, p.cj0, p.ncx, p.ncy,
                                                                   p.q) for p in ps], r)

    def advance(l, dt_l, dx, dy):
        old = states[l]
        Tc = [O.step_terms(q, dx, dy, dt_l, rho, K, limiter) for q in old]
        new = [O.step(q, dx, dy, dt_l, rho, K, limiter)[0] for q in old]
        if l == 0:
            O.fill_bc(new[0], bc)
        kids = geo[l + 1] if l + 1 < len(geo) else []
        if kids:
            accs = []
            for p in kids:
                myf, mxf = p.ncy * r, p.ncx * r
                accs.append({"left": np.zeros((myf, 3)), "right": np.zeros((myf, 3)),
                             "bottom": np.zeros((mxf, 3)), "top": np.zeros((mxf, 3))})
            for k in range(r):
                a = k / r
                for c, p in enumerate(kids):
                    qf = states[l + 1][c]
                    Qt = (1.0 - a) * old[p.parent] + a * new[p.parent]
                    sibs = [(s, states[l + 1][d]) for d, s in enumerate(kids)
                            if d != c and s.parent == p.parent]
                    fill_fine_ghosts(qf, p, Qt, r, sibs)
                for c, p in enumerate(kids):
                    qf = states[l + 1][c]
                    Tf = O.step_terms(qf, dx / r, dy / r, dt_l / r, rho, K, limiter)
                    accumulate_fine(accs[c], p, qf, Tf, old[p.parent], r, rho, K)
                advance(l + 1, dt_l / r, dx / r, dy / r)
            for c, p in enumerate(kids):
                average_down(new[p.parent], p, states[l + 1][c], r)
            for c, p in enumerate(kids):
                cov = covered_cells([s for s in kids if s.parent == p.parent])
                apply_fix(new[p.parent], p, accs[c], Tc[p.parent], dt_l, dx, dy, r, cov)
            if l == 0:
                O.fill_bc(new[0], bc)
        states[l] = new

    advance(0, dt, dx0, dy0)
    out = [[FinePatch(p.ci0, p.cj0, p.ncx, p.ncy, q, p.parent) for p, q in zip(geo[l], states[l])]
           for l in range(1, len(geo))]
    return states[0][0], out
