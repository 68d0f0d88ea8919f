"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: they check it against the
matrices of the acoustics system (paper Sec. 4.1 eq. (4.2)) taken through
numpy's eigen-solver, textbook one-dimensional schemes written here in matrix
form, exact solutions (translation, smooth plane waves), invariants
(conservation, rotation / transpose symmetry, constant states) and the
closed-form Courant number of eq. (2.10).
"""

import math

import numpy as np
import pytest

import workloads

RHO, KB = 1.0, 4.0  # c = 2, Z = 2 (the benchmark medium)


def acoustics_matrices(rho, K):
    """A and B of Sec. 4.1 eq. (4.2), written out from the paper."""
    A = np.array([[0.0, K, 0.0], [1.0 / rho, 0.0, 0.0], [0.0, 0.0, 0.0]])
    B = np.array([[0.0, 0.0, K], [0.0, 0.0, 0.0], [1.0 / rho, 0.0, 0.0]])
    return A, B


def split_matrices(M):
    """M+ and M- from numpy's eigen-decomposition (independent of the oracle)."""
    lam, V = np.linalg.eig(M)
    lam, V = lam.real, V.real
    Vi = np.linalg.inv(V)
    Mp = V @ np.diag(np.maximum(lam, 0.0)) @ Vi
    Mm = V @ np.diag(np.minimum(lam, 0.0)) @ Vi
    return Mp, Mm


# --------------------------------------------------------------------------
# Riemann solver
# --------------------------------------------------------------------------

@pytest.mark.parametrize("rho,K", [(1.0, 4.0), (0.7, 2.3), (1.9, 8.1)])
@pytest.mark.parametrize("direction", [0, 1])
def test_riemann_solver_eigen_structure(oracle_lib, rho, K, direction):
    A, B = acoustics_matrices(rho, K)
    M = A if direction == 0 else B
    lam = np.sort(np.linalg.eigvals(M).real)
    c = math.sqrt(K / rho)
    np.testing.assert_allclose(lam, [-c, 0.0, c], atol=1e-14 * c)
    rng = np.random.default_rng(7)
    for _ in range(20):
        ql, qr = rng.normal(size=3), rng.normal(size=3)
        waves, s, am, ap = oracle_lib.riemann_edge(direction, rho, K, ql, qr)
        dq = qr - ql
        np.testing.assert_allclose(np.sort(s), [-c, 0.0, c], rtol=0, atol=1e-15 * c)
        # waves decompose the jump
        np.testing.assert_allclose(waves.sum(axis=0), dq, rtol=0, atol=1e-14 * np.abs(dq).max())
        # each wave is an eigenvector of M with its speed
        for p in range(3):
            np.testing.assert_allclose(M @ waves[p], s[p] * waves[p], rtol=0,
                                       atol=1e-14 * (1 + np.abs(waves[p]).max() * K))
        # fluctuations add up to M dq, and equal M+/- dq
        np.testing.assert_allclose(am + ap, M @ dq, rtol=0, atol=1e-13 * (1 + np.abs(M @ dq).max()))
        Mp, Mm = split_matrices(M)
        np.testing.assert_allclose(ap, Mp @ dq, rtol=0, atol=1e-13 * (1 + np.abs(dq).max() * K))
        np.testing.assert_allclose(am, Mm @ dq, rtol=0, atol=1e-13 * (1 + np.abs(dq).max() * K))


@pytest.mark.parametrize("direction", [0, 1])
def test_transverse_split_matches_matrix_split(oracle_lib, direction):
    rho, K = 1.3, 3.1
    A, B = acoustics_matrices(rho, K)
    M = A if direction == 0 else B
    Mp, Mm = split_matrices(M)
    rng = np.random.default_rng(11)
    for _ in range(20):
        a = rng.normal(size=3)
        mn, pl = oracle_lib.split_vec(direction, rho, K, a)
        np.testing.assert_allclose(pl, Mp @ a, rtol=0, atol=1e-13 * (1 + K))
        np.testing.assert_allclose(mn, Mm @ a, rtol=0, atol=1e-13 * (1 + K))


# --------------------------------------------------------------------------
# Limiter
# --------------------------------------------------------------------------

def test_mc_limiter_table(oracle_lib):
    table = {-1.0: 0.0, 0.0: 0.0, 0.25: 0.5, 1.0: 1.0, 2.0: 1.5, 3.0: 2.0, 5.0: 2.0}
    for th, val in table.items():
        assert oracle_lib.phi("mc", th) == val
    assert oracle_lib.phi("none", -3.0) == 1.0
    assert oracle_lib.phi("zero", 2.0) == 0.0
    vl = {-1.0: 0.0, 0.0: 0.0, 1.0: 1.0, 3.0: 1.5}
    for th, val in vl.items():
        assert oracle_lib.phi("vanleer", th) == val


def test_mc_branch_table(oracle_lib):
    # 0: zero, 1: (1+theta)/2, 2: 2, 3: 2 theta; ties -> lowest index
    assert oracle_lib.mc_branch(1.0, -0.5) == 0
    assert oracle_lib.mc_branch(1.0, 0.0) == 0
    assert oracle_lib.mc_branch(0.0, 2.0) == 0
    assert oracle_lib.mc_branch(1.0, 0.25) == 3
    assert oracle_lib.mc_branch(1.0, 1.0 / 3.0 + 1e-12) == 1
    assert oracle_lib.mc_branch(1.0, 1.0) == 1
    assert oracle_lib.mc_branch(1.0, 3.0) == 1  # tie (1+3)/2 = 2
    assert oracle_lib.mc_branch(1.0, 5.0) == 2
    # branch value times theta-form equals phi
    for th in np.linspace(-2, 6, 81):
        b = oracle_lib.mc_branch(1.0, th)
        val = [0.0, 0.5 * (1 + th), 2.0, 2.0 * th][b]
        assert val == pytest.approx(oracle_lib.phi("mc", th), abs=1e-15)


# --------------------------------------------------------------------------
# Whole-step invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("tc", [False, True])
def test_constant_state_is_preserved_bitwise(oracle_lib, tc):
    q = np.empty((3, 20, 28))
    q[0], q[1], q[2] = 1.25, -0.5, 0.75
    out, cfl, _ = oracle_lib.step(q, 1 / 24, 1 / 16, 0.004, RHO, KB, "mc", transverse_corr=tc)
    assert np.array_equal(out[:, 2:-2, 2:-2], q[:, 2:-2, 2:-2])


def _y_uniform_state(mx, my, rng):
    q = np.zeros((3, my + 4, mx + 4))
    row = rng.normal(size=(3, mx))
    q[:, 2:-2, 2:-2] = row[:, None, :]
    return q


def _periodic_x(a):
    return np.roll(a, -1, axis=-1), np.roll(a, 1, axis=-1)


@pytest.mark.parametrize("tc", [False, True])
def test_one_dimensional_reduction_lax_wendroff(oracle_lib, tc):
    """y-uniform data, phi = 1: the unsplit step is the textbook Lax-Wendroff
    scheme Q - nu/2 Ahat (Q+ - Q-) + nu^2/2 Ahat^2 (Q+ - 2Q + Q-), with either
    transverse solver (their terms cancel between the two y-edges)."""
    rng = np.random.default_rng(3)
    mx, my = 32, 6
    q = _y_uniform_state(mx, my, rng)
    oracle_lib.fill_bc(q, "periodic")
    dx, dy, dt = 1 / mx, 1 / my, 0.7 / (2 * mx)
    out, _, _ = oracle_lib.step(q, dx, dy, dt, RHO, KB, "none", transverse_corr=tc)
    A, _ = acoustics_matrices(RHO, KB)
    Q = q[:, 2, 2:-2]
    Qp, Qm = _periodic_x(Q)
    ref = Q - 0.5 * (dt / dx) * (A @ (Qp - Qm)) + 0.5 * (dt / dx) ** 2 * (A @ A @ (Qp - 2 * Q + Qm))
    for j in range(my):
        np.testing.assert_allclose(out[:, 2 + j, 2:-2], ref, rtol=0, atol=1e-14)


def test_one_dimensional_reduction_upwind(oracle_lib):
    """y-uniform data, phi = 0: first-order upwind Q - dt/dx (A+ (Q - Q-) + A- (Q+ - Q))."""
    rng = np.random.default_rng(4)
    mx, my = 32, 5
    q = _y_uniform_state(mx, my, rng)
    oracle_lib.fill_bc(q, "periodic")
    dx, dy, dt = 1 / mx, 1 / my, 0.9 / (2 * mx)
    out, _, _ = oracle_lib.step(q, dx, dy, dt, RHO, KB, "zero")
    A, _ = acoustics_matrices(RHO, KB)
    Ap, Am = split_matrices(A)
    Q = q[:, 2, 2:-2]
    Qp, Qm = _periodic_x(Q)
    ref = Q - (dt / dx) * (Ap @ (Q - Qm) + Am @ (Qp - Q))
    for j in range(my):
        np.testing.assert_allclose(out[:, 2 + j, 2:-2], ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("tc", [False, True])
@pytest.mark.parametrize("limiter", ["mc", "none", "zero"])
def test_plane_wave_translates_exactly_at_courant_one(oracle_lib, limiter, tc):
    """A right-going simple wave (p' = Z u, v = 0) moves one cell per step at
    nu = 1, whatever the limiter: the correction weight (1 - nu) vanishes."""
    mx, my = 128, 4
    c, Z = 2.0, 2.0
    rng = np.random.default_rng(5)
    prof = rng.normal(size=mx)
    q = np.zeros((3, my + 4, mx + 4))
    q[0, 2:-2, 2:-2] = 1.0 + prof[None, :]
    q[1, 2:-2, 2:-2] = prof[None, :] / Z
    dx = 1.0 / mx
    dt = dx / c
    res = oracle_lib.run(q, 100, dx, 1.0 / my, RHO, KB, limiter=limiter, bc="periodic", dt=dt,
                         transverse_corr=tc)
    expect = np.roll(q[:, 2:-2, 2:-2], 100, axis=-1)
    err = np.abs(res["q"][:, 2:-2, 2:-2] - expect).max()
    assert err <= 1e-13, err


@pytest.mark.parametrize("tc", [False, True])
def test_conservation_periodic(oracle_lib, tc):
    n = 48
    spec, q = workloads.uniform_patch(n)
    # make the pulse reach the boundary: shift the centre off the middle
    q = workloads.padded_state(n, n, 0.0, 0.0, 1 / n, 1 / n, xc=0.3, yc=0.6)
    rng = np.random.default_rng(9)
    q[1:, 2:-2, 2:-2] = 0.1 * rng.normal(size=(2, n, n))
    s0 = oracle_lib.conservation_sums(oracle_lib.fill_bc(q.copy(), "periodic"), 1 / n, 1 / n)
    res = oracle_lib.run(q, 500, 1 / n, 1 / n, RHO, KB, limiter="mc", bc="periodic", cfl_desired=0.9,
                         transverse_corr=tc)
    s1 = oracle_lib.conservation_sums(res["q"], 1 / n, 1 / n)
    scale = np.abs(q[:, 2:-2, 2:-2]).sum(axis=(1, 2)) / n**2
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale), (s0, s1)


@pytest.mark.parametrize("tc", [False, True])
def test_rotation_and_transpose_symmetry(oracle_lib, tc):
    """Centred pulse on the 128^2 square, extrapolation BCs, 100 steps at CFL 0.9."""
    spec, q = workloads.uniform_patch(128)
    res = oracle_lib.run(q, 100, spec.dx, spec.dy, RHO, KB, limiter="mc", bc="extrap",
                         cfl_desired=0.9, transverse_corr=tc)
    p, u, v = (res["q"][m, 2:-2, 2:-2] for m in range(3))  # arrays [j, i]
    scale = np.abs(res["q"]).max()
    # transpose: p(i,j) = p(j,i), u(i,j) = v(j,i)
    assert np.abs(p - p.T).max() <= 1e-12 * scale
    assert np.abs(u - v.T).max() <= 1e-12 * scale
    # rotation by 90 degrees: p(i,j) = p(j, N-1-i), u(i,j) = -v(j, N-1-i), v(i,j) = u(j, N-1-i)
    N = p.shape[0]
    i = np.arange(N)[None, :]
    j = np.arange(N)[:, None]
    assert np.abs(p - p[N - 1 - i, j]).max() <= 1e-12 * scale
    assert np.abs(u + v[N - 1 - i, j]).max() <= 1e-12 * scale
    assert np.abs(v - u[N - 1 - i, j]).max() <= 1e-12 * scale
    # and the pulse has actually moved
    assert np.abs(p - q[0, 2:-2, 2:-2]).max() > 0.1


def _plane_wave_cell_average(n, kx, ky, Z, t, c):
    """Exact cell averages of the translating plane wave (closed form)."""
    h = 1.0 / n
    xs = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    kn = math.hypot(kx, ky)
    phase = 2 * np.pi * (kx * X + ky * Y - kn * c * t)
    damp = (np.sinc(kx * h) * np.sinc(ky * h))  # numpy sinc(x) = sin(pi x)/(pi x)
    pp = 0.5 * np.sin(phase) * damp
    return np.stack([1.0 + pp, pp / Z * kx / kn, pp / Z * ky / kn])


@pytest.mark.slow
@pytest.mark.parametrize("tc", [False, True])
def test_second_order_convergence_oblique_plane_wave(oracle_lib, tc):
    """phi = 1, periodic unit square, oblique smooth wave (kx, ky) = (1, 2),
    nu = 0.8, t = 0.25: errors fall by 4x per refinement.  The cross term is
    only second-order accurate with the transverse terms present, with the
    right factor and signs."""
    kx, ky = 1, 2
    c, Z = 2.0, 2.0
    T = 0.25
    errs1, errsinf = [], []
    for n in (32, 64, 128, 256):
        h = 1.0 / n
        nsteps = int(round(T / (0.8 * h / c)))
        dt = T / nsteps
        q = np.zeros((3, n + 4, n + 4))
        q[:, 2:-2, 2:-2] = _plane_wave_cell_average(n, kx, ky, Z, 0.0, c)
        res = oracle_lib.run(q, nsteps, h, h, RHO, KB, limiter="none", bc="periodic", dt=dt,
                             transverse_corr=tc)
        ex = _plane_wave_cell_average(n, kx, ky, Z, T, c)
        d = res["q"][:, 2:-2, 2:-2] - ex
        errs1.append(np.abs(d).sum() * h * h)
        errsinf.append(np.abs(d).max())
    o1 = [math.log2(errs1[k] / errs1[k + 1]) for k in range(3)]
    oi = [math.log2(errsinf[k] / errsinf[k + 1]) for k in range(3)]
    assert 1.9 <= o1[-1] <= 2.1, o1
    assert 1.9 <= oi[-1] <= 2.1, oi


def test_cfl_closed_form(oracle_lib):
    for (mx, my, rho, K) in [(16, 16, 1.0, 4.0), (24, 40, 0.6, 7.5), (50, 17, 1.7, 1.2)]:
        q = np.ones((3, my + 4, mx + 4))
        dx, dy = 1 / mx, 1 / my
        c = math.sqrt(K / rho)
        dt = 0.37 * min(dx, dy) / c
        _, cfl, _ = oracle_lib.step(q, dx, dy, dt, rho, K, "mc")
        expect = c * dt / min(dx, dy)
        assert abs(cfl - expect) <= 2 * np.spacing(expect)


@pytest.mark.parametrize("limiter", ["mc", "vanleer"])
def test_step_patches_equals_each_patch_stepped_alone(oracle_lib, limiter):
    """The batched wrapper (the reference of a whole AMR level, one step of
    eq. (2.3) per patch with that patch's own cell sizes, time step and
    medium) equals the single-patch step of every patch, bitwise, and returns
    each patch's Courant number, c dt / min(dx, dy) (eq. (2.10))."""
    rng = np.random.default_rng(2361)
    # differing shapes, dx != dy, time steps and media; one patch a single cell
    specs = [(13, 7, 1 / 40, 1 / 25, 0.7, 2.3), (24, 31, 1 / 64, 1 / 48, 1.9, 8.1),
             (5, 40, 1 / 16, 1 / 90, 1.0, 4.0), (32, 32, 1 / 32, 1 / 32, 0.55, 1.4),
             (1, 1, 1 / 8, 1 / 11, 1.3, 3.3)]
    states, dxs, dys, dts, rhos, Ks = [], [], [], [], [], []
    for mx, my, dx, dy, rho, K in specs:
        q = np.ascontiguousarray(rng.normal(size=(3, my + 4, mx + 4)))
        q[0] += 2.0
        states.append(q)
        c = math.sqrt(K / rho)
        dxs.append(dx), dys.append(dy), rhos.append(rho), Ks.append(K)
        dts.append(rng.uniform(0.3, 0.95) * min(dx, dy) / c)
    outs, cfls = oracle_lib.step_patches(states, dxs, dys, dts, rhos, Ks, limiter)
    assert len(outs) == len(specs) and cfls.shape == (len(specs),)
    for k, q in enumerate(states):
        ref, cfl, _ = oracle_lib.step(q, dxs[k], dys[k], dts[k], rhos[k], Ks[k], limiter)
        assert np.array_equal(outs[k][:, 2:-2, 2:-2], ref[:, 2:-2, 2:-2]), k
        assert cfls[k] == cfl, (k, cfls[k], cfl)
        expect = math.sqrt(Ks[k] / rhos[k]) * dts[k] / min(dxs[k], dys[k])
        assert abs(cfls[k] - expect) <= 2 * np.spacing(expect), k
        # the wrapper steps every patch once: not a patch stepped twice or left
        assert not np.array_equal(outs[k][:, 2:-2, 2:-2], q[:, 2:-2, 2:-2]), k


def test_zero_speed_wave_changes_nothing(oracle_lib):
    """Two-wave and three-wave solvers give equal updates (the speed-0 wave has
    no fluctuation, no correction weight and no speed)."""
    spec, q = workloads.uniform_patch(40, xc=0.45, yc=0.55)
    rng = np.random.default_rng(12)
    q[1:, 2:-2, 2:-2] = 0.2 * rng.normal(size=(2, 40, 40))
    oracle_lib.fill_bc(q, "extrap")
    a, ca, _ = oracle_lib.step(q, spec.dx, spec.dy, 0.002, RHO, KB, "mc")
    b, cb, _ = oracle_lib.step(q, spec.dx, spec.dy, 0.002, RHO, KB, "mc", drop_zero_wave=True)
    assert np.array_equal(a, b) and ca == cb


def test_extrapolation_ghosts_take_nearest_interior(oracle_lib):
    rng = np.random.default_rng(1)
    mx, my = 7, 5
    q = rng.normal(size=(3, my + 4, mx + 4))
    oracle_lib.fill_bc(q, "extrap")
    jj = np.clip(np.arange(-2, my + 2), 0, my - 1) + 2
    ii = np.clip(np.arange(-2, mx + 2), 0, mx - 1) + 2
    assert np.array_equal(q, q[:, jj][:, :, ii])
    q2 = rng.normal(size=(3, my + 4, mx + 4))
    oracle_lib.fill_bc(q2, "periodic")
    jj = (np.arange(-2, my + 2) % my) + 2
    ii = (np.arange(-2, mx + 2) % mx) + 2
    assert np.array_equal(q2, q2[:, jj][:, :, ii])


def _scalar_tvd_step(w, nu, phi):
    """Textbook flux-limited upwind scheme for w_t + a w_x = 0 on a periodic
    line, nu = a dt/dx (either sign):
    w - nu d_up - 1/2 |nu| (1 - |nu|) (phi(theta_R) d_R - phi(theta_L) d_L) * sign
    written with jumps d_{i-1/2} = w_i - w_{i-1} and theta = d_upwind / d."""
    d = w - np.roll(w, 1)              # d[i] = jump at i-1/2
    if nu >= 0:
        dup = np.roll(d, 1)            # jump at i-3/2 for the edge i-1/2
    else:
        dup = np.roll(d, -1)           # jump at i+1/2
    with np.errstate(divide="ignore", invalid="ignore"):
        theta = np.where(d != 0.0, dup / np.where(d != 0.0, d, 1.0), 0.0)
    lim = np.where(d != 0.0, np.vectorize(phi)(theta) * d, 0.0)
    flux = 0.5 * abs(nu) * (1.0 - abs(nu)) * lim    # F~ at i-1/2 (times dx/dt)
    first = nu * d if nu >= 0 else nu * np.roll(d, -1)
    return w - first - (np.roll(flux, -1) - flux)


@pytest.mark.parametrize("tc", [False, True])
@pytest.mark.parametrize("limiter", ["mc", "vanleer"])
def test_one_dimensional_reduction_limited_scheme(oracle_lib, limiter, tc):
    """y-uniform data: each characteristic field of A (numpy eigenvectors)
    follows the scalar flux-limited scheme with the same limiter."""
    rng = np.random.default_rng(21)
    mx, my = 40, 4
    q = _y_uniform_state(mx, my, rng)
    q[:, 2:-2, 2 + 10:2 + 18] += 1.5  # a plateau gives both smooth and steep ratios
    oracle_lib.fill_bc(q, "periodic")
    dx, dy, dt = 1 / mx, 1 / my, 0.8 / (2 * mx)
    out, _, _ = oracle_lib.step(q, dx, dy, dt, RHO, KB, limiter, transverse_corr=tc)
    A, _ = acoustics_matrices(RHO, KB)
    lam, V = np.linalg.eig(A)
    lam, V = lam.real, V.real
    Vi = np.linalg.inv(V)
    W = Vi @ q[:, 2, 2:-2]
    W1 = np.stack([_scalar_tvd_step(W[p], lam[p] * dt / dx, lambda t: oracle_lib.phi(limiter, t))
                   if lam[p] != 0 else W[p] for p in range(3)])
    ref = V @ W1
    for j in range(my):
        np.testing.assert_allclose(out[:, 2 + j, 2:-2], ref, rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# The variant that also splits the second-order correction transversely
# --------------------------------------------------------------------------

def _step_matrix(oracle_lib, n, nu_x, nu_y, tc):
    """Matrix of the phi = 1 step (a linear map) on a periodic n x n grid,
    columns from unit inputs: the oracle is used as a black box."""
    c = math.sqrt(KB / RHO)
    dx = 1.0 / n
    dt = nu_x * dx / c
    dy = c * dt / nu_y
    m = 3 * n * n
    M = np.empty((m, m))
    for k in range(m):
        x = np.zeros(m)
        x[k] = 1.0
        q = np.zeros((3, n + 4, n + 4))
        q[:, 2:-2, 2:-2] = x.reshape(3, n, n)
        oracle_lib.fill_bc(q, "periodic")
        out, _, _ = oracle_lib.step(q, dx, dy, dt, RHO, KB, "none", transverse_corr=tc,
                                    parallel=False)
        M[:, k] = out[:, 2:-2, 2:-2].ravel()
    return M


@pytest.mark.parametrize("tc", [False, True])
def test_von_neumann_stable_up_to_courant_one(oracle_lib, tc):
    """The unsplit method with transverse terms is stable for Courant numbers up
    to one in each direction (Sec. 2.4 eq. (2.10) and the time-step rule of
    Sec. 2.5 rely on it): on a periodic grid the spectral radius of the linear
    phi = 1 step stays at most 1 (the constant mode gives exactly 1).  Moving the
    correction the wrong way, or too much of it, into the split fluctuations
    makes some mode grow."""
    for nu_x, nu_y in [(0.8, 0.8), (1.0, 0.5), (0.9, 0.3), (0.5, 0.95)]:
        M = _step_matrix(oracle_lib, 10, nu_x, nu_y, tc)
        r = np.abs(np.linalg.eigvals(M)).max()
        assert r <= 1.0 + 1e-12, (nu_x, nu_y, r)


def test_transverse_correction_variant_is_distinct_and_reduces_without_correction(oracle_lib):
    """The variant differs from the default only through the limited correction:
    with phi = 0 there is none and the two steps agree bitwise; with a live
    limiter they differ at the size of the transverse correction terms,
    (c dt)^2 / (dx dy) times second differences, and so not at rounding level."""
    spec, q = workloads.uniform_patch(48, xc=0.4, yc=0.55)
    rng = np.random.default_rng(31)
    q[1:, 2:-2, 2:-2] = 0.1 * rng.normal(size=(2, 48, 48))
    oracle_lib.fill_bc(q, "extrap")
    dt = 0.8 * spec.dx / 2.0
    a, ca, _ = oracle_lib.step(q, spec.dx, spec.dy, dt, RHO, KB, "zero")
    b, cb, _ = oracle_lib.step(q, spec.dx, spec.dy, dt, RHO, KB, "zero", transverse_corr=True)
    assert np.array_equal(a, b) and ca == cb
    a, _, _ = oracle_lib.step(q, spec.dx, spec.dy, dt, RHO, KB, "mc")
    b, _, _ = oracle_lib.step(q, spec.dx, spec.dy, dt, RHO, KB, "mc", transverse_corr=True)
    d = np.abs(a - b)[:, 2:-2, 2:-2].max()
    assert d > 1e-4 * np.abs(q[:, 2:-2, 2:-2] - q[:, 2:-2, 2:-2].mean()).max(), d
    # the two variants agree to second order: one step differs by O(h^3)
    # relative to the O(h) change of the step itself
    assert d < 0.2 * np.abs(a - q)[:, 2:-2, 2:-2].max(), d


def test_transverse_correction_variant_rejects_masks(oracle_lib):
    """The variant limits on the outer ghost rows too, which have no mask bytes."""
    q = np.ones((3, 12, 12))
    try:
        oracle_lib.step(q, 0.1, 0.1, 0.01, RHO, KB, "mc", transverse_corr=True, record_masks=True)
    except RuntimeError:
        return
    raise AssertionError("masks were accepted with the transverse-correction variant")
