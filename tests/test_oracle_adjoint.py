"""Pins of the oracle's frozen-branch adjoint.

The adjoint is a separate code path (each forward stage transposed in scatter
form); it is checked against the oracle's forward step run with the same
frozen branches: frozen forward == nonlinear forward at the recording state,
linearity, the dot-product identity <S x, y> = <x, S^T y>, the dense
Jacobian of an 8x8 patch built column by column, and central finite
differences of the receiver loss (exact for a piecewise-quadratic loss away
from branch changes).
"""

import math

import numpy as np
import pytest

import workloads

RHO, KB = 1.0, 4.0


def _recorded_state(n, steps=6, seed=0, xc=0.5, yc=0.5, ny=None):
    """A state a few steps into the pulse run on an n x ny grid of the unit
    square, its masks and dt."""
    ny = ny or n
    q = workloads.padded_state(n, ny, 0, 0, 1 / n, 1 / ny, xc, yc)
    rng = np.random.default_rng(seed)
    q[1:, 2:-2, 2:-2] += 0.05 * rng.normal(size=(2, ny, n))
    import oracle
    dt = 0.8 / max(n, ny) / 2.0
    res = oracle.run(q, steps, 1 / n, 1 / ny, RHO, KB, limiter="mc", bc="extrap", dt=dt)
    q = res["q"]
    _out, _cfl, masks = oracle.step(q, 1 / n, 1 / ny, dt, RHO, KB, "mc", record_masks=True)
    return q, masks, dt


def test_masks_take_several_branches(oracle_lib):
    q, masks, _dt = _recorded_state(24)
    nib = np.concatenate([(masks >> s) & 3 for s in (0, 2, 4, 6)]).ravel()
    counts = np.bincount(nib, minlength=4)
    assert (counts > 0).all(), counts


def test_frozen_forward_equals_nonlinear_step(oracle_lib):
    n = 24
    q, masks, dt = _recorded_state(n)
    out, _, _ = oracle_lib.step(q, 1 / n, 1 / n, dt, RHO, KB, "mc")
    fz = oracle_lib.frozen_step(q[:, 2:-2, 2:-2], 1 / n, 1 / n, dt, RHO, KB, masks)
    assert np.abs(fz - out[:, 2:-2, 2:-2]).max() <= 1e-14 * np.abs(out).max()


def test_frozen_step_is_linear(oracle_lib):
    n = 16
    _q, masks, dt = _recorded_state(n)
    rng = np.random.default_rng(3)
    x, y = rng.normal(size=(2, 3, n, n))
    S = lambda v: oracle_lib.frozen_step(v, 1 / n, 1 / n, dt, RHO, KB, masks)  # noqa: E731
    lhs = S(2.5 * x - 1.5 * y)
    rhs = 2.5 * S(x) - 1.5 * S(y)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


@pytest.mark.parametrize("bc", ["extrap", None])
def test_dot_product_identity(oracle_lib, bc):
    n, ny = 20, 14  # dx != dy
    q, masks, dt = _recorded_state(n, ny=ny)
    rng = np.random.default_rng(4)
    x, y = rng.normal(size=(2, 3, ny, n))
    Sx = oracle_lib.frozen_step(x, 1 / n, 1 / ny, dt, RHO, KB, masks, bc=bc)
    STy = oracle_lib.adjoint_step(y, q, 1 / n, 1 / ny, dt, RHO, KB, masks, bc=bc)
    a, b = float(np.vdot(Sx, y)), float(np.vdot(x, STy))
    assert abs(a - b) <= 1e-13 * max(abs(a), 1.0), (a, b)


def test_dense_jacobian_of_small_patch(oracle_lib):
    n, ny = 8, 6
    q, masks, dt = _recorded_state(n, steps=3, xc=0.52, yc=0.47, ny=ny)
    N = 3 * n * ny
    S = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        S[:, c] = oracle_lib.frozen_step(e.reshape(3, ny, n), 1 / n, 1 / ny, dt, RHO, KB,
                                         masks).ravel()
    ST = np.zeros((N, N))
    for r in range(N):
        e = np.zeros(N)
        e[r] = 1.0
        ST[:, r] = oracle_lib.adjoint_step(e.reshape(3, ny, n), q, 1 / n, 1 / ny, dt, RHO, KB,
                                           masks).ravel()
    assert np.abs(ST - S.T).max() <= 1e-14 * np.abs(S).max()


def fd_check(oracle_lib, p0, state0, steps, dx, dt, receivers, target, directions, h=1e-6):
    """Central differences of J along each direction, graded only where no
    MC branch changes between p0 - h v, p0 and p0 + h v (a branch change is
    a kink of the piecewise-quadratic J, where the frozen adjoint takes one
    side).  Returns (list of (fd, adjoint) pairs, number of flipped probes)."""
    J, grad, _tr, masks0 = oracle_lib.adjoint_run(p0, steps, dx, dx, dt, RHO, KB, receivers,
                                                   target, state0=state0)
    graded, flipped = [], 0
    for v in directions:
        Jp, _, _, mp = oracle_lib.forward_traces(p0 + h * v, steps, dx, dx, dt, RHO, KB, receivers,
                                                 target, state0)
        Jm, _, _, mm = oracle_lib.forward_traces(p0 - h * v, steps, dx, dx, dt, RHO, KB, receivers,
                                                 target, state0)
        if any((a != b).any() or (a != c).any() for a, b, c in zip(masks0, mp, mm)):
            flipped += 1
            continue
        graded.append(((Jp - Jm) / (2 * h), float(np.vdot(grad, v))))
    return graded, flipped


def test_gradient_matches_central_differences(oracle_lib):
    """Receiver misfit after 12 steps on 32^2, smooth data on a random smooth
    background (no exactly flat region): adjoint gradient vs central
    differences, h = 1e-6, in flip-free directions."""
    n, steps = 32, 12
    dx = 1 / n
    setup = workloads.adjoint_setup(n=n, steps=steps)
    xs = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    rng = np.random.default_rng(11)
    bg = sum(rng.uniform(0.05, 0.2) * np.sin(2 * np.pi * (rng.integers(1, 4) * X + rng.integers(1, 4) * Y) + rng.uniform(0, 6))
             for _ in range(4))
    p0 = 1.0 + np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.02) + bg
    state0 = np.zeros((3, n, n))
    state0[1] = 0.1 * np.cos(2 * np.pi * Y)
    target = oracle_lib.forward_traces(p0 * 0.9, steps, dx, dx, setup.dt, RHO, KB,
                                       setup.receivers, None, state0)[1]
    dirs = [rng.normal(size=(n, n)) for _ in range(10)]
    graded, flipped = fd_check(oracle_lib, p0, state0, steps, dx, setup.dt, setup.receivers,
                               target, dirs)
    assert len(graded) >= 5, flipped
    for fd, ad in graded:
        assert abs(fd - ad) <= 1e-8 * max(abs(ad), 1e-8), (fd, ad)


def test_flat_background_kinks_are_detected(oracle_lib):
    """With the literal ring pulse (exactly flat outside the ring) directions
    over the ring change branches where the wave meets the flat background;
    the harness must count them instead of grading them."""
    n, steps = 32, 12
    dx = 1 / n
    setup = workloads.adjoint_setup(n=n, steps=steps)
    p0 = setup.p0()
    target = oracle_lib.forward_traces(setup.target_p0(), steps, dx, dx, setup.dt, RHO, KB,
                                       setup.receivers)[1]
    rng = np.random.default_rng(7)
    r = np.hypot(*np.meshgrid((np.arange(n) + .5) / n - .5, (np.arange(n) + .5) / n - .5))
    ring = np.abs(r - 0.25) < 0.08
    dirs = [np.where(ring, rng.normal(size=(n, n)), 0.0) for _ in range(3)]
    graded, flipped = fd_check(oracle_lib, p0, None, steps, dx, setup.dt, setup.receivers,
                               target, dirs)
    assert flipped >= 1
    for fd, ad in graded:
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-8), (fd, ad)
