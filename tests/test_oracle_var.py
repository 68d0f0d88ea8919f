"""Pins of the oracle's step in a heterogeneous medium (rho, K per cell).

None retypes the oracle's formulas: a uniform medium reduces to the
constant-coefficient step; with phi = 0 the first step of a Riemann problem
at a material interface gives the cell averages of the exact solution, whose
middle state follows from the characteristic relations
p* + Z_l u* = p_l + Z_l u_l and p* - Z_r u* = p_r - Z_r u_r (a textbook result
written here, not the oracle's wave split); transposing medium and data
transposes the result; the
Courant number is max over edges of the larger sound speed times dt/dx; the
MC step dissipates the acoustic energy on a rough random medium (which a
transverse split with the wrong impedance or speed does not).
Each pin also takes a copy of the oracle library (``lib``) so that planted
mistakes can be checked against it.
"""

import math

import numpy as np
import pytest

import oracle.oracle as O

RHO, KB = 1.0, 4.0


def step_var(lib, q, dx, dy, dt, rho, K, limiter):
    if lib is None:
        return O.step_var(q, dx, dy, dt, rho, K, limiter)
    saved = O._lib
    O._lib = lib
    try:
        return O.step_var(q, dx, dy, dt, rho, K, limiter)
    finally:
        O._lib = saved


def uniform_medium(mx, my, rho=RHO, K=KB):
    return np.full((my + 4, mx + 4), rho), np.full((my + 4, mx + 4), K)


@pytest.mark.parametrize("limiter", ["mc", "vanleer", "none", "zero"])
def test_uniform_medium_is_the_constant_coefficient_step(limiter, lib=None):
    rng = np.random.default_rng(70)
    mx, my = 23, 17
    q = rng.normal(size=(3, my + 4, mx + 4))
    O.fill_bc(q, "extrap")
    rho, K = uniform_medium(mx, my, 1.3, 2.9)
    dx, dy = 1 / mx, 1 / my
    dt = 0.7 * min(dx, dy) / math.sqrt(2.9 / 1.3)
    a, ca = step_var(lib, q, dx, dy, dt, rho, K, limiter)
    b, cb, _ = O.step(q, dx, dy, dt, 1.3, 2.9, limiter)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()
    assert abs(ca - cb) <= 4 * np.spacing(cb)


def _exact_middle(ql, qr, Zl, Zr, n):
    """Middle state (p*, normal velocity*) of the interface Riemann problem."""
    us = (Zl * ql[n] + Zr * qr[n] + ql[0] - qr[0]) / (Zl + Zr)
    ps = ql[0] + Zl * ql[n] - Zl * us
    return ps, us


@pytest.mark.parametrize("direction", [0, 1])
def test_interface_riemann_problem_first_step_is_exact(direction, lib=None):
    """phi = 0, data and medium uniform along the interface: after one step the
    two cells next to the interface hold (1 - nu) Q + nu Q*, every other cell
    is unchanged."""
    n_cells, width = 20, 5
    e = 10  # the interface is the edge between cells e-1 and e
    rho_l, K_l, rho_r, K_r = 1.0, 4.0, 2.5, 3.6  # Z = 2 and 3, c = 2 and 1.2
    cl, cr = math.sqrt(K_l / rho_l), math.sqrt(K_r / rho_r)
    Zl, Zr = rho_l * cl, rho_r * cr
    ql = np.array([1.2, 0.3, -0.4])
    qr = np.array([0.7, -0.5, 0.9])
    mx, my = (n_cells, width) if direction == 0 else (width, n_cells)
    q = np.zeros((3, my + 4, mx + 4))
    rho = np.zeros((my + 4, mx + 4))
    K = np.zeros((my + 4, mx + 4))
    idx = np.arange(-2, n_cells + 2)
    left = idx < e
    for m in range(3):
        prof = np.where(left, ql[m], qr[m])
        if direction == 0:
            q[m] = prof[None, :]
        else:
            q[m] = prof[:, None]
    prof_r, prof_k = np.where(left, rho_l, rho_r), np.where(left, K_l, K_r)
    rho[:] = prof_r[None, :] if direction == 0 else prof_r[:, None]
    K[:] = prof_k[None, :] if direction == 0 else prof_k[:, None]
    h = 1.0 / n_cells
    dt = 0.6 * h / max(cl, cr)
    out, _ = step_var(lib, q, h, h, dt, rho, K, "zero")
    nrm = 1 if direction == 0 else 2
    tang = 2 if direction == 0 else 1
    ps, us = _exact_middle(ql, qr, Zl, Zr, nrm)
    nu_l, nu_r = cl * dt / h, cr * dt / h
    exp = np.zeros((3, n_cells))
    for i in range(n_cells):
        base = ql if i < e else qr
        exp[:, i] = base
    star_l = np.array(ql, float)
    star_l[0], star_l[nrm] = ps, us
    star_r = np.array(qr, float)
    star_r[0], star_r[nrm] = ps, us
    exp[:, e - 1] = (1 - nu_l) * ql + nu_l * star_l
    exp[:, e] = (1 - nu_r) * qr + nu_r * star_r
    assert star_l[tang] == ql[tang] and star_r[tang] == qr[tang]
    for k in range(width):
        got = out[:, 2 + k, 2:-2] if direction == 0 else out[:, 2:-2, 2 + k]
        assert np.abs(got - exp).max() <= 1e-14, (k, np.abs(got - exp).max())


def _smooth_medium(mx, my):
    xs = (np.arange(-2, mx + 2) + 0.5) / mx
    ys = (np.arange(-2, my + 2) + 0.5) / my
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    rho = 1.0 + 0.4 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    K = 4.0 + 1.5 * np.cos(2 * np.pi * (X + 2 * Y))
    return rho, K, X, Y


def test_transpose_symmetry(lib=None):
    mx = my = 24
    rho, K, X, Y = _smooth_medium(mx, my)
    rho = rho + 0.3 * (X > 0.6)  # a jump too, off the diagonal
    q = np.stack([1 + np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.01), 0.1 * X, -0.2 * Y])
    O.fill_bc(q, "extrap")
    dt = 0.5 / mx / 3.0
    a, ca = step_var(lib, q, 1 / mx, 1 / my, dt, rho, K, "mc")
    qt = np.ascontiguousarray(np.stack([q[0].T, q[2].T, q[1].T]))
    b, cb = step_var(lib, qt, 1 / mx, 1 / my, dt, np.ascontiguousarray(rho.T),
                     np.ascontiguousarray(K.T), "mc")
    assert np.abs(a[0] - b[0].T).max() <= 1e-13
    assert np.abs(a[1] - b[2].T).max() <= 1e-13
    assert np.abs(a[2] - b[1].T).max() <= 1e-13
    assert ca == cb


def test_mc_step_dissipates_energy_on_a_rough_medium(lib=None):
    """Random medium (log-normal rho and K, impedance contrasts up to ~10),
    random data, periodic, MC limiter, Courant 0.9: the acoustic energy
    sum p^2/(2K) + rho (u^2 + v^2)/2 decreases at every one of 100 steps.  A
    transverse split that takes the wrong cell's impedance or sound speed
    gains energy on some steps."""
    rng = np.random.default_rng(5)
    n = 40
    rho = np.exp(0.8 * rng.normal(size=(n + 4, n + 4)))
    K = np.exp(0.8 * rng.normal(size=(n + 4, n + 4)))
    q = rng.normal(size=(3, n + 4, n + 4))
    O.fill_bc(q, "periodic")
    dt = 0.9 / n / np.sqrt(K / rho).max()

    def energy(q):
        p, u, v = q[:, 2:-2, 2:-2]
        return 0.5 * (p ** 2 / K[2:-2, 2:-2] + rho[2:-2, 2:-2] * (u ** 2 + v ** 2)).sum()

    e = energy(q)
    for s in range(100):
        q, _ = step_var(lib, q, 1 / n, 1 / n, dt, rho, K, "mc")
        O.fill_bc(q, "periodic")
        e1 = energy(q)
        assert e1 < e, (s, e, e1)
        e = e1


def test_courant_number_is_the_largest_edge_speed(lib=None):
    mx, my = 9, 7
    rho, K = uniform_medium(mx, my)
    K[2 + 3, 2 + 4] = 16.0  # one interior cell with c = 4
    K[0, 0] = 100.0  # a corner ghost: on no edge of an interior cell
    q = np.ones((3, my + 4, mx + 4))
    dx, dy = 1 / mx, 1 / my
    dt = 0.01
    _, cfl = step_var(lib, q, dx, dy, dt, rho, K, "mc")
    assert abs(cfl - 4.0 * dt / min(dx, dy)) <= 2 * np.spacing(cfl)
