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
"""

from __future__ import annotations

import math

import torch

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
                 velocity0=None, device="cuda"):
        if nsteps < 1 or checkpoint_every < 1:
            raise ValueError("nsteps and checkpoint_every must be >= 1")
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

    def _forward(self, p0):
        lev = self.level
        if p0.shape != (self.my, self.mx):
            raise ValueError(f"p0 must have shape {(self.my, self.mx)}")
        p0 = p0.detach().to(device=lev.device, dtype=torch.float64)
        with torch.cuda.stream(lev.stream):
            traces = torch.empty((self.nsteps, self.nr), dtype=torch.float64, device=lev.device)
            self._start(p0)
            ckpts = []
            for n in range(self.nsteps):
                if n % self.k == 0:
                    ckpts.append(lev.state_view(0).clone())
                lev.step(self.dt, read_cfl=False)
                lev.gather(0, 0, self.ij, traces[n])
        lev.stream.synchronize()
        return traces, ckpts

    def _backward(self, ckpts, g):
        lev = self.level
        with torch.cuda.stream(lev.stream):
            g = g.detach().to(device=lev.device, dtype=torch.float64).contiguous()
            lam, lam_next = lev.new_buffer(), lev.new_buffer()
            masks = [lev.new_masks() for _ in range(min(self.k, self.nsteps))]
            for seg in range(len(ckpts) - 1, -1, -1):
                s0, s1 = seg * self.k, min(self.nsteps, (seg + 1) * self.k)
                lev.upload(0, ckpts[seg])
                for s in range(s0, s1):
                    lev.step_record_masks(self.dt, masks[s - s0])
                for n in range(s1 - 1, s0 - 1, -1):
                    lev.add_at(0, 0, self.ij, g[n], buf=lam)
                    lev.adjoint_step(self.dt, masks[n - s0], lam, lam_next)
                    lam, lam_next = lam_next, lam
            grad = lev.patch_view(lam, 0)[0, 2:-2, 2:-2].clone()
        lev.stream.synchronize()
        return grad
