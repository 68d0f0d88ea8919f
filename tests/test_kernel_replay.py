"""CPU replays of the index and lane arithmetic of two kernels, against the
oracle and against the sets they must cover (no GPU):

* the adjoint kernel's march: numpy arrays stand for a wavefront's 64 lanes
  (lane shifts with a zero fill past the wave, as the kernel's DPP shifts
  read), rows are walked as the kernel walks them, with its prologue, its
  carried y-terms, the ghost-column fold by two lane shifts and the
  ghost-row fold; the result equals the oracle's adjoint step (the
  transposed frozen-branch step with the transposed extrapolation fill) on
  patches from 1 x 1 to 130 x 70 with segment heights 1 to 16;
* the coarse-fine fine-step kernel's blocks: every strip cell a block reads
  is filled (interior cells loaded, ghost cells evaluated once per coarse
  cell), every ghost of the ring is written by exactly one block, the coarse
  cell found by integer floor division equals the floating-point one, every
  strip index lies in the block's LDS array, and the coarse box a block
  stages holds every coarse cell its ghosts' stencils read and fits the LDS
  the launch gives it.
"""

import math

import numpy as np
import pytest

import oracle

def shr(a):
    """Lane l takes lane l-1's value; lane 0 reads 0."""
    out = np.zeros_like(a)
    out[1:] = a[:-1]
    return out


def shl(a):
    """Lane l takes lane l+1's value; the last lane reads 0."""
    out = np.zeros_like(a)
    out[:-1] = a[1:]
    return out


def w_own(c):
    return np.where(c == 1, 0.5, np.where(c == 2, 2.0, 0.0))


def w_up(c):
    return np.where(c == 1, 0.5, np.where(c == 3, 2.0, 0.0))


def replay_adjoint(lam, masks, mx, my, dx, dy, dt, rho, K, fold=True, H=16):
    """The adjoint kernel's segments (60 columns by H rows) on one patch:
    lam (3, my, mx) interior cotangents, masks (my+1, mx+1) branch bytes;
    returns the padded output (ghosts included)."""
    c = math.sqrt(K / rho); Z = rho * c
    dtdx, dtdy, iz = dt / dx, dt / dy, 1 / Z
    fx = 0.25 * c * (1 - c * dtdx); fy = 0.25 * c * (1 - c * dtdy)
    gx = 0.125 * dtdx * c * c; gy = 0.125 * dtdy * c * c
    k = dict(Z=Z, h=0.5 * c, hz=0.5 * c * iz, fx=fx, fxz=fx * iz, fy=fy, fyz=fy * iz, gx=gx, gxz=gx * iz, gy=gy, gyz=gy * iz, dtdx=dtdx, dtdy=dtdy)
    out = np.full((3, my + 4, mx + 4), np.nan)
    ntx = (mx + 59) // 60
    nty = (my + H - 1) // H
    for tx in range(ntx):
        cols = tx * 60 - 2 + np.arange(64)
        colin = (cols >= 0) & (cols < mx)
        colm = (cols >= 0) & (cols <= mx)
        cl = np.clip(cols, 0, mx - 1); cm = np.clip(cols, 0, mx)
        def fetch(r):
            rr = min(max(r, 0), my - 1); rm = min(max(r, 0), my)
            rin = 0 <= r < my
            P = np.where(colin & rin, lam[0, rr, cl], 0.0)
            U = np.where(colin & rin, lam[1, rr, cl], 0.0)
            V = np.where(colin & rin, lam[2, rr, cl], 0.0)
            M = np.where(colm & (0 <= r <= my), masks[rm, cm], 0).astype(np.int64)
            return P, U, V, M
        def y_edge(plo, vlo, phi, vhi, code):
            gp = k['dtdy'] * (phi - plo); gv = k['dtdy'] * (vhi - vlo)
            m1 = -k['fy'] * gp + k['fyz'] * gv; m2 = k['fy'] * gp + k['fyz'] * gv
            c1 = (code >> 4) & 3; c2 = (code >> 6) & 3
            return dict(gp=gp, gv=gv, n1=w_own(c1) * m1, t1=w_up(c1) * m1, n2=w_own(c2) * m2, t2=w_up(c2) * m2)
        def x_row(p, u, v):
            fp = k['dtdx'] * (p - shr(p)); fu = k['dtdx'] * (u - shr(u))
            ys = -k['dtdy'] * k['h'] * p + k['gy'] * (fp - shl(fp)) - k['gyz'] * (fu + shl(fu))
            yd = -k['dtdy'] * k['hz'] * v
            return dict(fp=fp, fu=fu, ys=ys, yd=yd)
        l = np.arange(64)
        st_val = (l >= 2) & (l <= 61) & (cols >= 0) & (cols < mx)
        st_zero = (cols == -2) | (cols == -1) | (((cols == mx) | (cols == mx + 1)) & (l >= 2))
        xedge = tx == 0 or tx == ntx - 1
        for ty in range(nty):
            r0 = ty * H; r1 = min(r0 + H, my)
            a0 = -2 if r0 == 0 else r0
            a1 = my + 2 if r1 == my else r1
            Pa, Ua, Va, Ma = fetch(a0 - 2); Pb, Ub, Vb, Mb = fetch(a0 - 1)
            P0, U0, V0, M0 = fetch(a0); P1, U1, V1, M1 = fetch(a0 + 1)
            em = y_edge(Pa, Va, Pb, Vb, Mb)
            xm = x_row(Pb, Ub, Vb)
            e0 = y_edge(Pb, Vb, P0, V0, M0)
            x0 = x_row(P0, U0, V0)
            e1 = y_edge(P0, V0, P1, V1, M1)
            gp0, gv0, t1_0 = e0['gp'], e0['gv'], e0['t1']
            b1 = e0['n1'] + em['t1'] + xm['ys'] - xm['yd']; b2 = e0['n2'] + e1['t2'] + x0['ys'] + x0['yd']
            DY0, SY0 = b2 - b1, b1 + b2
            lo = np.zeros((3, 64)); hi = np.zeros((3, 64))
            for r in range(a0, a1):
                p0, u0, v0, m0 = fetch(r); p1, u1, v1, _ = fetch(r + 1); p2, u2, v2, m2c = fetch(r + 2)
                e2 = y_edge(p1, v1, p2, v2, m2c)
                x1 = x_row(p1, u1, v1)
                b1 = e1['n1'] + t1_0 + x0['ys'] - x0['yd']; b2 = e1['n2'] + e2['t2'] + x1['ys'] + x1['yd']
                DY1, SY1 = b2 - b1, b1 + b2
                l1 = -k['fx'] * x0['fp'] + k['fxz'] * x0['fu']; l2 = k['fx'] * x0['fp'] + k['fxz'] * x0['fu']
                c1 = m0 & 3; c2 = (m0 >> 2) & 3
                o1, u1w, o2, u2w = w_own(c1) * l1, w_up(c1) * l1, w_own(c2) * l2, w_up(c2) * l2
                xs = -k['dtdx'] * k['h'] * p0 + k['gx'] * (gp0 - e1['gp']) - k['gxz'] * (gv0 + e1['gv'])
                xd = -k['dtdx'] * k['hz'] * u0
                A1 = ((o1 + shr(u1w)) + shr(xs)) - shr(xd); A2 = ((o2 + shl(u2w)) + xs) + xd
                DX, SX = A2 - A1, A1 + A2
                o = np.stack([p0 + (DX - shl(DX)) + (DY0 - DY1), u0 + Z * (SX - shl(SX)), v0 + Z * (SY0 - SY1)])
                if fold and xedge:
                    L1 = np.stack([shr(x) for x in o]); L2 = np.stack([shr(x) for x in L1])
                    R1 = np.stack([shl(x) for x in o]); R2 = np.stack([shl(x) for x in R1])
                    o = np.where(cols == 0, o + (L1 + L2), o)
                    o = np.where(cols == mx - 1, o + (R1 + R2), o)
                def put(rr, vals, sel):
                    for m in range(3):
                        out[m, rr + 2, cols[sel] + 2] = vals[m][sel] if np.ndim(vals[m]) else vals[m]
                if r < 0:
                    lo += o; put(r, [0.0] * 3, st_val | st_zero)
                elif r < my:
                    if fold and r == 0: o = o + lo
                    put(r, [0.0] * 3, st_zero)
                    if fold and r == my - 1: hi = o.copy()
                    else: put(r, o, st_val)
                else:
                    hi += o; put(r, [0.0] * 3, st_val | st_zero)
                    if fold and r == my + 1: put(my - 1, hi, st_val)
                gp0, gv0, t1_0 = e1['gp'], e1['gv'], e1['t1']
                e1 = e2; x0 = x1; DY0, SY0 = DY1, SY1
    return out



@pytest.mark.parametrize("mx,my,H", [(7, 5, 16), (1, 1, 16), (61, 37, 2), (130, 70, 4),
                                     (60, 16, 1), (121, 33, 8), (2, 40, 3), (3, 3, 2)])
@pytest.mark.parametrize("bc", ["extrap", None])
def test_adjoint_march_replay_equals_oracle(oracle_lib, mx, my, H, bc):
    rng = np.random.default_rng(mx * 1000 + my * 10 + H)
    dx, dy = 1 / mx, 1.3 / my
    rho, K = 1.2, 3.0
    dt = 0.4 * min(dx, dy) / math.sqrt(K / rho)
    lam = rng.standard_normal((3, my, mx))
    masks = rng.integers(0, 256, (my + 1, mx + 1)).astype(np.uint8)
    q = np.zeros((3, my + 4, mx + 4))
    ref = oracle_lib.adjoint_step(lam, q, dx, dy, dt, rho, K, masks, bc=bc)
    got = replay_adjoint(lam, masks, mx, my, dx, dy, dt, rho, K, fold=(bc == "extrap"), H=H)
    assert np.isfinite(got).all()
    ghost = got.copy()
    ghost[:, 2:-2, 2:-2] = 0
    assert np.abs(ghost).max() == 0  # every ghost written, with 0
    assert np.abs(got[:, 2:-2, 2:-2] - ref).max() <= 1e-14 * np.abs(ref).max()


def strip_of(max_side):
    """Edges (threads) per block: a multiple of 64 covering the longest side,
    at most 256."""
    return max(64, min(256, (max_side + 63) // 64 * 64))


def fdiv(a, b):
    return a // b  # floor division, as the kernel's fdiv


def replay_fine_step_blocks(mx, my, r, ci0=2, cj0=2, kStrip=None):
    """Walk every block of the fine-step kernel of one mx x my fine patch
    (blocks of kStrip edges; by default the launch's choice for this patch)."""
    kStrip = kStrip or strip_of(max(mx, my))
    nxb = (my + kStrip - 1) // kStrip; nyb = (mx + kStrip - 1) // kStrip
    owned = {}
    ring = set()
    for j in range(-2, my + 2):
        for i in range(-2, mx + 2):
            if not (0 <= i < mx and 0 <= j < my): ring.add((i, j))
    LDS = 3 * (kStrip + 2) * 4
    box_cells = ((3 + r - 1) // r + 3) * ((kStrip + 3 + r - 1) // r + 3)  # cf_box_cells
    LDS_BYTES = 8 * (LDS + 3 * box_cells)
    assert LDS_BYTES <= 64 * 1024
    def region(ia, ib, ja, jb, sink):
        CIa, CIb = fdiv(2*ia+1, 2*r), fdiv(2*(ib-1)+1, 2*r)
        CJa, CJb = fdiv(2*ja+1, 2*r), fdiv(2*(jb-1)+1, 2*r)
        nI, nJ = CIb - CIa + 1, CJb - CJa + 1
        # the staged coarse box and the stencil cells read from it
        bw, bh = nI + 2, nJ + 2
        assert bw * bh <= box_cells, (ia, ib, ja, jb, r, kStrip)
        def box_index(ci, cj):  # absolute coarse indices, as the kernel's at()
            x, y = ci - ci0 - CIa + 1, cj - cj0 - CJa + 1
            assert 0 <= x < bw and 0 <= y < bh
            return y * bw + x
        seen = set()
        for k in range(nI * nJ):
            I, J = CIa + k % nI, CJa + k // nI
            for j in range(max(ja, J*r), min(jb, J*r + r)):
                for i in range(max(ia, I*r), min(ib, I*r + r)):
                    if 0 <= i < mx and 0 <= j < my: continue
                    X = ci0 + (i + 0.5) / r; Y = cj0 + (j + 0.5) / r
                    assert math.floor(X) == ci0 + I and math.floor(Y) == cj0 + J
                    ci, cj = math.floor(X), math.floor(Y)
                    for (di, dj) in ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)):
                        box_index(ci + di, cj + dj)
                    assert (i, j) not in seen; seen.add((i, j))
                    sink(i, j)
        want = {(i, j) for i in range(ia, ib) for j in range(ja, jb) if not (0 <= i < mx and 0 <= j < my)}
        assert seen == want, (ia, ib, ja, jb)
    for b in range(2 * nxb + 2 * nyb):
        filled = set()
        if b < 2 * nxb:
            left = b < nxb
            j0 = (b if left else b - nxb) * kStrip; j1 = min(j0 + kStrip, my)
            e = 0 if left else mx
            rows = j1 - j0 + 2
            for x in range(rows * 4):
                j = j0 - 1 + x // 4; i = e - 2 + x % 4
                if 0 <= i < mx and 0 <= j < my:
                    idx = (2 * (kStrip + 2) + (j - j0 + 1)) * 4 + (i - e + 2); assert 0 <= idx < LDS
                    filled.add((i, j))
            def sink(i, j):
                idx = (2 * (kStrip + 2) + (j - j0 + 1)) * 4 + (i - e + 2)
                assert 0 <= idx < LDS and 0 <= (j - j0 + 1) < kStrip + 2 and 0 <= i - e + 2 < 4
                filled.add((i, j))
                if (i < 0 if left else i >= mx) and j0 <= j < j1:
                    owned[(i, j)] = owned.get((i, j), 0) + 1
            region(e - 2, e + 2, j0 - 1, j1 + 1, sink)
            need = {(i, j) for i in range(e - 2, e + 2) for j in range(j0 - 1, j1 + 1)}
            assert filled == need
        else:
            bb = b - 2 * nxb
            bottom = bb < nyb; c = bb if bottom else bb - nyb
            i0 = c * kStrip; i1 = min(i0 + kStrip, mx); f = 0 if bottom else my
            lo = -2 if c == 0 else i0; hi = mx + 2 if i1 == mx else i1
            cols = i1 - i0 + 2
            for x in range(cols * 4):
                j = f - 2 + x // cols; i = i0 - 1 + x % cols
                if 0 <= i < mx and 0 <= j < my:
                    filled.add((i, j))
            def sink(i, j):
                if i0 - 1 <= i <= i1:
                    idx = (2 * (kStrip + 2) + (i - i0 + 1)) * 4 + (j - f + 2)
                    assert 0 <= idx < LDS and 0 <= j - f + 2 < 4
                    filled.add((i, j))
                if (j < 0 if bottom else j >= my) and lo <= i < hi:
                    owned[(i, j)] = owned.get((i, j), 0) + 1
            region(min(lo, i0 - 1), max(hi, i1 + 1), f - 2, f + 2, sink)
            need = {(i, j) for i in range(i0 - 1, i1 + 1) for j in range(f - 2, f + 2)}
            assert filled == need, (mx, my, r, b)
    assert set(owned) == ring and all(v == 1 for v in owned.values()), (mx, my, r)



@pytest.mark.parametrize("r", [1, 2, 3, 4, 5])
def test_fine_step_blocks_cover_strips_and_ring(r):
    for mx in sorted({r, 2 * r, 3 * r, 30 * r, 120 - 120 % r, 256 - 256 % r, 300 - 300 % r,
                      516 - 516 % r}):
        for my in sorted({r, 2 * r, 7 * r, 120 - 120 % r, 600 - 600 % r}):
            replay_fine_step_blocks(mx, my, r, ci0=2 + r, cj0=3)
            replay_fine_step_blocks(mx, my, r, ci0=2, cj0=2, kStrip=64)
