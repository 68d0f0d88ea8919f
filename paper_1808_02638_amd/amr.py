"""Levels coupled for the composite coarse step with the conservation fix:
a thin binding of the ``ws_cf_*`` entry points of the C ABI (``TwoLevel``
for one coarse-fine pair, ``Hierarchy`` for more levels).

The coarse ``Level`` and the fine ``Level`` (patches nested in the coarse ones,
``bc=None``, created on the coarse level's stream) stay usable on their own;
``TwoLevel.step(dt)`` advances both by one coarse step: the coarse step, r fine
steps with ghosts from the coarse level, the update of the covered coarse
cells and the conservation fix, all in the library's kernels on the shared
stream.
"""

from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib as C
from .level import Level, poisoned


class TwoLevel:
    """coarse, fine: Level objects; ratio: refinement ratio r; places: one
    (coarse_patch, ci0, cj0) per fine patch (the coarse cell under the fine
    patch's interior cell (0, 0))."""

    def __init__(self, coarse: Level, fine: Level, ratio: int, places: Sequence):
        if coarse.stream != fine.stream:
            raise ValueError("create the fine Level with stream=coarse.stream")
        if len(places) != fine.n:
            raise ValueError("one place per fine patch")
        self._L = C.lib()
        self.coarse, self.fine, self.ratio = coarse, fine, int(ratio)
        nb = ctypes.c_int64(0)
        C.check(self._L.ws_cf_layout(fine._ctx, self.ratio, ctypes.byref(nb)))
        self.workspace = poisoned(nb.value, coarse.device)
        torch.cuda.synchronize(coarse.device)
        pl = (C.FinePlace * fine.n)()
        for k, (cp, ci0, cj0) in enumerate(places):
            pl[k].coarse_patch, pl[k].ci0, pl[k].cj0 = int(cp), int(ci0), int(cj0)
        cf = ctypes.c_void_p()
        C.check(self._L.ws_cf_init(ctypes.byref(cf), coarse._ctx, fine._ctx, self.ratio, pl,
                                   ctypes.c_void_p(self.workspace.data_ptr()), nb.value))
        self._cf = cf

    def step(self, dt: float):
        """One composite coarse step of size dt (asynchronous on the stream)."""
        with torch.cuda.stream(self.coarse.stream):
            C.check(self._L.ws_cf_step(self._cf, float(dt)))

    def fill_fine_ghosts(self, alpha: float):
        C.check(self._L.ws_cf_fill_fine_ghosts(self._cf, float(alpha)))

    def close(self):
        if getattr(self, "_cf", None):
            self._L.ws_cf_destroy(self._cf)
            self._cf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    """Levels 0..L coupled pairwise and nested: levels[l+1]'s patches lie in
    levels[l]'s (ratio ratios[l]); places[l] lists, per patch of level l+1,
    (parent patch in level l, ci0, cj0).  Every level must be created on
    levels[0]'s stream.  ``step(dt)`` advances level 0 by dt and level l by
    r^l steps of dt / r^l, with the updating and the fix at every pair."""

    def __init__(self, levels: Sequence[Level], ratios, places: Sequence):
        if len(levels) < 2:
            raise ValueError("a hierarchy needs at least two levels")
        if isinstance(ratios, int):
            ratios = [ratios] * (len(levels) - 1)
        if len(ratios) != len(levels) - 1 or len(places) != len(levels) - 1:
            raise ValueError("one ratio and one place list per coupled pair")
        self.levels = list(levels)
        self.pairs = [TwoLevel(levels[l], levels[l + 1], ratios[l], places[l])
                      for l in range(len(levels) - 1)]
        for outer, inner in zip(self.pairs, self.pairs[1:]):
            C.check(C.lib().ws_cf_nest(outer._cf, inner._cf))

    def step(self, dt: float):
        self.pairs[0].step(dt)

    def close(self):
        for p in self.pairs:
            p.close()
