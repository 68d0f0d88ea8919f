"""Ghost cells of a level whose patches tile a rectangular domain, FP64,
plain numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The ghost-cell rules of the paper's Sec. 2.2 applied to the coarsest level:
a ghost cell outside the computational domain takes its value from the
physical boundary condition, and one that lies in another patch of the same
level is copied from it.  The physical conditions are the ones the
single-patch step uses, per direction: periodic (the global index wraps
around the domain) or zero-order extrapolation (the global index is clamped
to the domain's edge cell).  A ghost is first mapped into the domain that
way, then copied from the patch that holds the image (possibly the patch
itself).  The patches must cover the domain exactly, without overlap.

Layout: states are padded (3, my+4, mx+4) arrays as in the C oracle; patch k
has its interior cell (0, 0) at global cell origins[k] = (x0, y0).
"""

from __future__ import annotations

import numpy as np


def owner_map(shapes, origins, domain):
    """(DY, DX) array of the patch index holding each domain cell; raises
    unless the patches (mx, my) at origins (x0, y0) tile the domain."""
    DX, DY = domain
    own = np.full((DY, DX), -1, dtype=np.int64)
    for k, ((mx, my), (x0, y0)) in enumerate(zip(shapes, origins)):
        if mx < 1 or my < 1 or x0 < 0 or y0 < 0 or x0 + mx > DX or y0 + my > DY:
            raise ValueError(f"patch {k} does not lie in the domain")
        blk = own[y0:y0 + my, x0:x0 + mx]
        if (blk >= 0).any():
            raise ValueError(f"patch {k} overlaps another patch")
        blk[:] = k
    if (own < 0).any():
        raise ValueError("the patches do not cover the domain")
    return own


def ghost_source(gx, gy, domain, periodic):
    """The domain cell whose value a ghost at global (gx, gy) takes."""
    DX, DY = domain
    gx = gx % DX if periodic[0] else min(max(gx, 0), DX - 1)
    gy = gy % DY if periodic[1] else min(max(gy, 0), DY - 1)
    return gx, gy


def exchange_ghosts(qs, origins, domain, periodic=(True, True)):
    """Fill every ghost cell of every patch state in qs, in place."""
    shapes = [(q.shape[2] - 4, q.shape[1] - 4) for q in qs]
    own = owner_map(shapes, origins, domain)
    for k, q in enumerate(qs):
        mx, my = shapes[k]
        x0, y0 = origins[k]
        for j in range(-2, my + 2):
            for i in range(-2, mx + 2):
                if 0 <= i < mx and 0 <= j < my:
                    continue
                sx, sy = ghost_source(x0 + i, y0 + j, domain, periodic)
                o = own[sy, sx]
                ox, oy = origins[o]
                q[:, j + 2, i + 2] = qs[o][:, sy - oy + 2, sx - ox + 2]
    return qs
