"""ctypes driver of the C oracle (``wave_oracle.c``) plus its step loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Arrays follow the oracle's storage: one patch is a C-contiguous float64 array
of shape (3, my+4, mx+4) -- components (p, u, v), two ghost layers per side.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wave_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

LIM = {"mc": 0, "none": 1, "zero": 2, "vanleer": 3}
BC = {"extrap": 0, "periodic": 1}
OPT_DROP_ZERO_WAVE = 1
OPT_TRANSVERSE_CORR = 2

_lib = None


def build(src=_SRC, out=_SO) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP on)."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
        "-shared", "-Wall", "-Wextra", src, "-o", out, "-lm",
    ]
    subprocess.run(cmd, check=True)
    return out


def load_lib(path):
    """Load an oracle shared object and declare its argument types."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    L.oracle_step_ex.argtypes = [
        dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
        ctypes.c_int, u8p, u8p, dp, ctypes.c_int,
    ]
    L.oracle_step_ex.restype = ctypes.c_int
    L.oracle_fill_bc.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.oracle_fill_bc.restype = None
    L.oracle_phi.argtypes = [ctypes.c_int, ctypes.c_double]
    L.oracle_phi.restype = ctypes.c_double
    L.oracle_mc_branch.argtypes = [ctypes.c_double, ctypes.c_double]
    L.oracle_mc_branch.restype = ctypes.c_int
    L.oracle_step_patches.argtypes = [
        ctypes.c_int, dp, dp, i64p, ip, ip, dp, dp, dp, dp, dp, ctypes.c_int, dp,
    ]
    L.oracle_step_patches.restype = ctypes.c_int
    L.oracle_riemann_edge.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      dp, dp, dp, dp, dp, dp]
    L.oracle_riemann_edge.restype = None
    L.oracle_split_vec.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
    L.oracle_split_vec.restype = None
    L.oracle_step_var.argtypes = [
        dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        dp, dp, ctypes.c_int, dp,
    ]
    L.oracle_step_var.restype = ctypes.c_int
    L.oracle_step_terms.argtypes = [
        dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp,
    ]
    L.oracle_step_terms.restype = ctypes.c_int
    if hasattr(L, "oracle_adjoint_step"):
        L.oracle_adjoint_step.argtypes = [
            dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, u8p, ctypes.c_int,
        ]
        L.oracle_adjoint_step.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    _lib = load_lib(_SO)
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8ptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_uint8)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check_state(q):
    if not (isinstance(q, np.ndarray) and q.dtype == np.float64 and q.ndim == 3
            and q.shape[0] == 3 and q.flags.c_contiguous):
        raise ValueError("state must be a C-contiguous float64 array (3, my+4, mx+4)")
    my, mx = q.shape[1] - 4, q.shape[2] - 4
    if mx < 1 or my < 1:
        raise ValueError("patch must have at least one interior cell")
    return mx, my


def riemann_edge(direction, rho, K, ql, qr):
    """Single-edge normal Riemann solve: returns (waves (3,3), speeds (3,),
    amdq (3,), apdq (3,)).  direction 0 = x (matrix A), 1 = y (matrix B)."""
    ql = np.ascontiguousarray(ql, np.float64)
    qr = np.ascontiguousarray(qr, np.float64)
    waves = np.zeros((3, 3))
    s = np.zeros(3)
    am = np.zeros(3)
    ap = np.zeros(3)
    lib().oracle_riemann_edge(int(direction), float(rho), float(K), _dptr(ql), _dptr(qr),
                              _dptr(waves), _dptr(s), _dptr(am), _dptr(ap))
    return waves, s, am, ap


def split_vec(direction, rho, K, a):
    """Transverse split of a 3-vector: returns (minus part, plus part)."""
    a = np.ascontiguousarray(a, np.float64)
    mn = np.zeros(3)
    pl = np.zeros(3)
    lib().oracle_split_vec(int(direction), float(rho), float(K), _dptr(a), _dptr(mn), _dptr(pl))
    return mn, pl


def phi(lim: str, theta: float) -> float:
    return lib().oracle_phi(LIM[lim], float(theta))


def mc_branch(ww: float, theta: float) -> int:
    return lib().oracle_mc_branch(float(ww), float(theta))


def fill_bc(q: np.ndarray, bc: str) -> np.ndarray:
    """Fill the ghost cells of q in place from its interior."""
    mx, my = _check_state(q)
    if bc == "periodic" and (mx < 2 or my < 2):
        raise ValueError("periodic ghosts need at least 2 interior cells per side")
    lib().oracle_fill_bc(_dptr(q), mx, my, BC[bc])
    return q


def step(q, dx, dy, dt, rho, K, limiter="mc", *, drop_zero_wave=False,
         transverse_corr=False, frozen=None, record_masks=False, parallel=True):
    """One unsplit step.  Returns (q_new, cfl, masks-or-None).

    transverse_corr selects the variant whose transverse solver also splits
    the limited second-order correction (no masks with it)."""
    mx, my = _check_state(q)
    out = np.empty_like(q)
    cfl = ctypes.c_double(0.0)
    masks = np.zeros((my + 1, mx + 1), np.uint8) if record_masks else None
    if frozen is not None:
        frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
        if frozen.shape != (my + 1, mx + 1):
            raise ValueError("frozen masks must have shape (my+1, mx+1)")
    rc = lib().oracle_step_ex(
        _dptr(q), _dptr(out), mx, my, float(dx), float(dy), float(dt), float(rho),
        float(K), LIM[limiter],
        (OPT_DROP_ZERO_WAVE if drop_zero_wave else 0)
        | (OPT_TRANSVERSE_CORR if transverse_corr else 0), _u8ptr(frozen),
        _u8ptr(masks), ctypes.byref(cfl), int(bool(parallel)))
    if rc != 0:
        raise RuntimeError("oracle_step_ex failed")
    return out, cfl.value, masks


def step_var(q, dx, dy, dt, rho, K, limiter="mc"):
    """One step in a heterogeneous medium: rho, K padded (my+4, mx+4) arrays
    (ghost cells included).  Returns (q_new, cfl)."""
    mx, my = _check_state(q)
    rho = np.ascontiguousarray(rho, np.float64)
    K = np.ascontiguousarray(K, np.float64)
    if rho.shape != (my + 4, mx + 4) or K.shape != rho.shape:
        raise ValueError("rho and K must have the padded shape (my+4, mx+4)")
    out = np.empty_like(q)
    cfl = ctypes.c_double(0.0)
    rc = lib().oracle_step_var(_dptr(q), _dptr(out), mx, my, float(dx), float(dy), float(dt),
                               _dptr(rho), _dptr(K), LIM[limiter], ctypes.byref(cfl))
    if rc != 0:
        raise RuntimeError("oracle_step_var failed")
    return out, cfl.value


def run_var(q0, nsteps, dx, dy, rho, K, dt, *, limiter="mc", bc="extrap"):
    """nsteps heterogeneous steps of fixed dt; ghosts refilled after each."""
    q = np.array(q0, dtype=np.float64, order="C", copy=True)
    if bc is not None:
        fill_bc(q, bc)
    cfls = []
    for _ in range(nsteps):
        q, cfl = step_var(q, dx, dy, dt, rho, K, limiter)
        if bc is not None:
            fill_bc(q, bc)
        cfls.append(cfl)
    return {"q": q, "cfls": np.array(cfls)}


def step_terms(q, dx, dy, dt, rho, K, limiter="mc", *, transverse_corr=False):
    """The terms of eq. (2.3) at every edge of the interior cells, as one step
    of q would use them: dict of arrays
      Fx, amx, apx: (my, mx+1, 3) at x-edges (i-1/2, j)  (F~, A-dQ, A+dQ)
      Gy, amy, apy: (my+1, mx, 3) at y-edges (i, j-1/2)  (G~, B-dQ, B+dQ)."""
    mx, my = _check_state(q)
    X = [np.zeros((my, mx + 1, 3)) for _ in range(3)]
    Y = [np.zeros((my + 1, mx, 3)) for _ in range(3)]
    rc = lib().oracle_step_terms(
        _dptr(q), mx, my, float(dx), float(dy), float(dt), float(rho), float(K), LIM[limiter],
        OPT_TRANSVERSE_CORR if transverse_corr else 0,
        *[_dptr(a) for a in X], *[_dptr(a) for a in Y])
    if rc != 0:
        raise RuntimeError("oracle_step_terms failed")
    return dict(Fx=X[0], amx=X[1], apx=X[2], Gy=Y[0], amy=Y[1], apy=Y[2])


def step_patches(states, dxs, dys, dts, rhos, Ks, limiter="mc"):
    """One step of many independent patches (ghosts left as given)."""
    n = len(states)
    sizes = [s.size for s in states]
    off = np.zeros(n, np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    flat_in = np.concatenate([s.ravel() for s in states]) if n else np.zeros(0)
    flat_out = np.empty_like(flat_in)
    mx = np.array([s.shape[2] - 4 for s in states], np.intc)
    my = np.array([s.shape[1] - 4 for s in states], np.intc)
    f64 = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (n,)))
    dxa, dya, dta, rhoa, Ka = f64(dxs), f64(dys), f64(dts), f64(rhos), f64(Ks)
    cfl = np.zeros(n, np.float64)
    rc = lib().oracle_step_patches(
        n, _dptr(flat_in), _dptr(flat_out),
        off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        mx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        my.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        _dptr(dxa), _dptr(dya), _dptr(dta), _dptr(rhoa), _dptr(Ka), LIM[limiter],
        _dptr(cfl))
    if rc != 0:
        raise RuntimeError("oracle_step_patches failed")
    outs = [flat_out[o:o + s].reshape(st.shape) for o, s, st in zip(off, sizes, states)]
    return outs, cfl


def run(q0, nsteps, dx, dy, rho, K, *, limiter="mc", bc="extrap", dt=None,
        cfl_desired=None, dt0=None, drop_zero_wave=False, transverse_corr=False,
        parallel=True):
    """Advance ``nsteps`` unsplit steps.

    Ghosts are filled from the interior (``bc``) before the first step and
    after every step, so the returned state has valid ghosts.  With ``bc=None``
    ghosts stay as given.  The time step is either fixed (``dt``) or chosen from
    the desired Courant number: dt0 = nu * min(dx, dy) / c (or the given
    ``dt0``, to continue an earlier run) and then dt_{n+1} = dt_n * nu / cfl_n
    (Sec. 2.5 eq. (2.11)).  Returns dict(q, dts, cfls, next_dt).
    """
    q = np.array(q0, dtype=np.float64, order="C", copy=True)
    if bc is not None:
        fill_bc(q, bc)
    c = math.sqrt(K / rho)
    if dt is None:
        if cfl_desired is None:
            raise ValueError("give dt or cfl_desired")
        cur_dt = cfl_desired * min(dx, dy) / c if dt0 is None else float(dt0)
    else:
        cur_dt = float(dt)
    dts, cfls = [], []
    for _ in range(nsteps):
        q, cfl, _m = step(q, dx, dy, cur_dt, rho, K, limiter,
                          drop_zero_wave=drop_zero_wave, transverse_corr=transverse_corr,
                          parallel=parallel)
        if bc is not None:
            fill_bc(q, bc)
        dts.append(cur_dt)
        cfls.append(cfl)
        if dt is None:
            cur_dt = cur_dt * cfl_desired / cfl
    return {"q": q, "dts": np.array(dts), "cfls": np.array(cfls), "next_dt": cur_dt}


def frozen_step(x, dx, dy, dt, rho, K, masks, bc="extrap"):
    """The frozen-branch step as a map of the interior: x (3, my, mx) ->
    (3, my, mx), ghosts filled from x by ``bc`` (or zero when None)."""
    my, mx = x.shape[1], x.shape[2]
    q = np.zeros((3, my + 4, mx + 4))
    q[:, 2:-2, 2:-2] = x
    if bc is not None:
        fill_bc(q, bc)
    out, _cfl, _m = step(q, dx, dy, dt, rho, K, "mc", frozen=masks)
    return out[:, 2:-2, 2:-2].copy()


def conservation_sums(q, dx, dy):
    """Sum of q_m * dx * dy over the interior cells, m = p, u, v (exact fsum)."""
    return np.array([math.fsum(q[m, 2:-2, 2:-2].ravel().tolist()) * dx * dy
                     for m in range(3)])


def adjoint_step(lam_next, q, dx, dy, dt, rho, K, masks, bc="extrap"):
    """Oracle adjoint of one frozen-branch step including the boundary fill.

    lam_next: cotangent of the interior of Q^{n+1}, shape (3, my, mx).
    q: the state Q^n the forward step started from (ghosts filled), only
    used for its shape.  masks: the branches recorded on that forward step.
    bc: "extrap" (ghosts are filled from the interior before the step) or None
    (ghosts are frozen input and carry no cotangent).
    Returns the cotangent of the interior of Q^n, shape (3, my, mx).
    """
    L = lib()
    if not hasattr(L, "oracle_adjoint_step"):
        raise RuntimeError("oracle built without the adjoint")
    mx, my = _check_state(q)
    lam_in = np.ascontiguousarray(lam_next, dtype=np.float64)
    if lam_in.shape != (3, my, mx):
        raise ValueError("cotangent must have shape (3, my, mx)")
    out = np.zeros_like(lam_in)
    masks = np.ascontiguousarray(masks, dtype=np.uint8)
    rc = L.oracle_adjoint_step(_dptr(lam_in), _dptr(out), mx, my, float(dx), float(dy),
                               float(dt), float(rho), float(K), _u8ptr(masks),
                               BC[bc] if bc is not None else -1)
    if rc != 0:
        raise RuntimeError("oracle_adjoint_step failed")
    return out


def forward_traces(p0, nsteps, dx, dy, dt, rho, K, receivers, target=None, state0=None):
    """Forward run with extrapolation ghosts and fixed dt, recording the MC
    branches of every step and the pressure at the receivers after every step.
    p0: interior pressure (my, mx); u = v = 0 unless ``state0`` (3, my, mx) gives
    the velocities.  Returns (J or None, traces (nsteps, nr), states, masks)."""
    my, mx = p0.shape
    q = np.zeros((3, my + 4, mx + 4))
    if state0 is not None:
        q[:, 2:-2, 2:-2] = state0
    q[0, 2:-2, 2:-2] = p0
    fill_bc(q, "extrap")
    states, masks_all = [], []
    ri, rj = receivers[:, 0], receivers[:, 1]
    traces = np.zeros((nsteps, len(receivers)))
    for n in range(nsteps):
        states.append(q)
        q, _cfl, m = step(q, dx, dy, dt, rho, K, "mc", record_masks=True)
        fill_bc(q, "extrap")
        masks_all.append(m)
        traces[n] = q[0, rj + 2, ri + 2]
    J = None
    if target is not None:
        resid = traces - target
        J = 0.5 * math.fsum((resid * resid).ravel().tolist())
    return J, traces, states, masks_all


def adjoint_run(p0, nsteps, dx, dy, dt, rho, K, receivers, target, state0=None):
    """Gradient of J = 1/2 sum_n sum_r (p^n_r - d^n_r)^2 w.r.t. the interior p^0.

    Forward with extrapolation ghosts and fixed dt, recording the MC branches
    of every step; then the frozen-branch adjoint sweep in reverse.
    receivers: int array (nr, 2) of (i, j); target: (nsteps, nr).
    Returns (J, grad_p0 of shape (my, mx), traces (nsteps, nr), masks per step).
    """
    my, mx = p0.shape
    J, traces, states, masks_all = forward_traces(p0, nsteps, dx, dy, dt, rho, K, receivers,
                                                  target, state0)
    resid = traces - target
    ri, rj = receivers[:, 0], receivers[:, 1]
    lam = np.zeros((3, my, mx))
    for n in range(nsteps - 1, -1, -1):
        np.add.at(lam[0], (rj, ri), resid[n])
        lam = adjoint_step(lam, states[n], dx, dy, dt, rho, K, masks_all[n])
    return J, lam[0].copy(), traces, masks_all
