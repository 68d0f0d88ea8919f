"""Receiver traces of a fixed-dt acoustics run and their gradient with respect
to the initial pressure, as a ``torch.autograd.Function``.

Forward: the initial state (p0, u = v = 0) is stepped ``nsteps`` times with a
fixed dt on one extrapolation-boundary FP64 patch; after every step the
pressure at the receiver cells is gathered into ``traces[n]``.  The padded
state is checkpointed every ``checkpoint_every`` steps.

Backward: segments are walked last to first.  Each segment restarts from its
checkpoint and re-runs its steps recording the MC branches (the kernels are
deterministic, so the branches are those of the first forward pass); then the
frozen-branch adjoint steps run in reverse, each first adding the trace
cotangent of its step at the receivers.  The result is the cotangent of the
interior pressure p0.  All work runs in the library's kernels on the level's
stream; torch provides the buffers.

With ``store_branches=True`` the forward pass itself records every step's
branches (one byte per cell and step: 52 MB for 200 steps of 512^2, small
beside the GPU's memory) and keeps no checkpoints; the backward pass then
runs only the adjoint steps.  The recording step gives the same state as the
plain one, so the traces and the gradient are the same bits either way.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import _lib as C
from .level import Level


class _Traces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0, runner):
        traces, ckpts = runner._forward(p0)
        ctx.runner = runner
        ctx.ckpts = ckpts
        return traces

    @staticmethod
    def backward(ctx, g):
        grad = ctx.runner._backward(ctx.ckpts, g)
        ctx.ckpts = None
        return grad, None


class AcousticsAdjoint:
    """Receiver traces p^n(receivers), n = 1..nsteps, of a fixed-dt run on one
    mx x my FP64 patch with extrapolation boundaries and the MC limiter.

    receivers: (nr, 2) integer (i, j) interior cells.  dt: fixed time step.
    velocity0: optional (2, my, mx) initial (u, v), held fixed (default 0).
    ``traces(p0)`` returns an (nsteps, nr) tensor that autograd differentiates
    with respect to p0 (shape (my, mx), FP64, on the GPU)."""

    def __init__(self, mx, my, dx, dy, rho, K, receivers, nsteps, dt, checkpoint_every=20,
                 velocity0=None, device="cuda", store_branches=False):
        if nsteps < 1 or checkpoint_every < 1:
            raise ValueError("nsteps and checkpoint_every must be >= 1")
        self.store_branches = bool(store_branches)
        if not (dt > 0.0 and math.isfinite(dt)):
            raise ValueError("dt must be finite and > 0")
        self.mx, self.my = int(mx), int(my)
        self.nsteps, self.dt, self.k = int(nsteps), float(dt), int(checkpoint_every)
        self.level = Level([dict(mx=mx, my=my, dx=dx, dy=dy, bc="extrap")], [(rho, K)],
                           dtype=torch.float64, limiter="mc", device=device)
        rc = torch.as_tensor(receivers).to(torch.int64).reshape(-1, 2)
        if rc.numel() and (rc[:, 0].min() < 0 or rc[:, 0].max() >= mx or rc[:, 1].min() < 0
                           or rc[:, 1].max() >= my):
            raise ValueError("receivers must be interior cells")
        self.ij = rc.to(torch.int32).contiguous().to(self.level.device)
        self.nr = int(rc.shape[0])
        self.velocity0 = None
        if velocity0 is not None:
            v0 = torch.as_tensor(velocity0, dtype=torch.float64)
            if v0.shape != (2, self.my, self.mx):
                raise ValueError(f"velocity0 must have shape {(2, self.my, self.mx)}")
            self.velocity0 = v0.to(self.level.device)

    # -------------------------------------------------------------- public
    def traces(self, p0: torch.Tensor) -> torch.Tensor:
        return _Traces.apply(p0, self)

    def misfit(self, p0: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        """J = 1/2 sum_n sum_r (p^n_r - d^n_r)^2."""
        r = self.traces(p0) - target
        return 0.5 * (r * r).sum()

    def close(self):
        self.level.close()

    # ------------------------------------------------------------ internals
    def _start(self, p0):
        lev = self.level
        q = torch.zeros((3, self.my + 4, self.mx + 4), dtype=torch.float64, device=lev.device)
        q[0, 2:-2, 2:-2] = p0
        if self.velocity0 is not None:
            q[1:, 2:-2, 2:-2] = self.velocity0
        lev.upload(0, q)
        lev.fill_ghosts()

    # The step loops call the C entry points directly with arguments built
    # once (every buffer lives on the level's stream, so no stream waits are
    # needed); the Level methods' checks have been done on the buffers here.
    def _forward(self, p0):
        lev = self.level
        if p0.shape != (self.my, self.mx):
            raise ValueError(f"p0 must have shape {(self.my, self.mx)}")
        p0 = p0.detach().to(device=lev.device, dtype=torch.float64)
        L, ctx = lev._L, lev._ctx
        with torch.cuda.stream(lev.stream):
            traces = torch.empty((self.nsteps, self.nr), dtype=torch.float64, device=lev.device)
            self._start(p0)
            ckpts = []
            ij, nr, dt = ctypes.c_void_p(self.ij.data_ptr()), self.nr, self.dt
            base = traces.data_ptr()
            if self.store_branches:
                # every step records its branches; no checkpoints
                nb = (lev.mask_bytes() + 255) // 256 * 256
                masks = torch.empty(self.nsteps * nb, dtype=torch.uint8, device=lev.device)
                mb = masks.data_ptr()
                for n in range(self.nsteps):
                    C.check(L.ws_step_record_masks(ctx, dt, ctypes.c_void_p(mb + nb * n), None))
                    C.check(L.ws_gather(ctx, None, 0, 0, nr, ij,
                                        ctypes.c_void_p(base + 8 * nr * n)))
                ckpts = masks
            else:
                for n in range(self.nsteps):
                    if n % self.k == 0:
                        ckpts.append(lev.state_view(0).clone())
                    C.check(L.ws_step_level(ctx, dt, None))
                    C.check(L.ws_gather(ctx, None, 0, 0, nr, ij,
                                        ctypes.c_void_p(base + 8 * nr * n)))
        lev.stream.synchronize()
        return traces, ckpts

    def _backward(self, ckpts, g):
        lev = self.level
        L, ctx = lev._L, lev._ctx
        with torch.cuda.stream(lev.stream):
            g = g.detach().to(device=lev.device, dtype=torch.float64).contiguous()
            if g.shape != (self.nsteps, self.nr):
                raise ValueError("trace cotangent has the wrong shape")
            lam, lam_next = lev.new_buffer(), lev.new_buffer()
            if self.store_branches:
                # the forward pass recorded every step's branches (ckpts)
                bufs = [ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(lam_next.data_ptr())]
                ij, nr, dt, gb = ctypes.c_void_p(self.ij.data_ptr()), self.nr, self.dt, g.data_ptr()
                nb, mb = (lev.mask_bytes() + 255) // 256 * 256, ckpts.data_ptr()
                cur = 0
                for n in range(self.nsteps - 1, -1, -1):
                    C.check(L.ws_add_at(ctx, bufs[cur], 0, 0, nr, ij,
                                        ctypes.c_void_p(gb + 8 * nr * n)))
                    C.check(L.ws_adjoint_step(ctx, dt, ctypes.c_void_p(mb + nb * n), bufs[cur],
                                              bufs[1 - cur]))
                    cur = 1 - cur
                grad = lev.patch_view(lam if cur == 0 else lam_next, 0)[0, 2:-2, 2:-2].clone()
                lev.stream.synchronize()
                return grad
            masks = [lev.new_masks() for _ in range(min(self.k, self.nsteps))]
            mp = [ctypes.c_void_p(m.data_ptr()) for m in masks]
            bufs = [ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(lam_next.data_ptr())]
            ij, nr, dt, gb = ctypes.c_void_p(self.ij.data_ptr()), self.nr, self.dt, g.data_ptr()
            cur = 0
            for seg in range(len(ckpts) - 1, -1, -1):
                s0, s1 = seg * self.k, min(self.nsteps, (seg + 1) * self.k)
                lev.state_view(0).copy_(ckpts[seg])  # restore, asynchronously
                for s in range(s0, s1):
                    C.check(L.ws_step_record_masks(ctx, dt, mp[s - s0], None))
                for n in range(s1 - 1, s0 - 1, -1):
                    C.check(L.ws_add_at(ctx, bufs[cur], 0, 0, nr, ij,
                                        ctypes.c_void_p(gb + 8 * nr * n)))
                    C.check(L.ws_adjoint_step(ctx, dt, mp[n - s0], bufs[cur], bufs[1 - cur]))
                    cur = 1 - cur
            grad = lev.patch_view(lam if cur == 0 else lam_next, 0)[0, 2:-2, 2:-2].clone()
        lev.stream.synchronize()
        return grad
