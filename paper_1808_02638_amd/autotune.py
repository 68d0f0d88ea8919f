"""Tile autotuner for a ``Level``.

Patches are grouped into size classes; for each class (largest total cell
count first) the tuner times candidate tilings (HIP events on the level's
stream around back-to-back level steps, as a captured step loop runs them),
keeping the other classes fixed, then tunes the persistent launch's
workgroups per CU; the four fastest configurations seen then play off in
turns with more launches.  The
state is saved before tuning and restored afterwards, and an even number of
steps is timed per candidate, so the level is left exactly as it was.  The
tiling never changes results (the library's arithmetic per cell does not
depend on it), so tuning is safe on a live level.

Choices are cached in a JSON file keyed by GPU architecture, the library's
step-kernel and tiling sources, dtype, limiter (with the transverse variant)
and the patch-size histogram.  A table of choices the tuner made on an MI355X for the
benchmark workloads ships beside this module (``tuned_tilings.json``) and is
consulted before the user's cache, so a run on a fresh machine uses the same
tilings as the runs its measurements were taken with; ``autotune(...,
use_cache=False)`` always times the candidates.
"""

from __future__ import annotations

import hashlib
import json
import os
from collections import defaultdict

import numpy as np
import torch

from ._lib import WaveStepError

DIRECT, MARCH, PACKED = "direct", "march", "packed"
_BUCKETS = (0, 12, 24, 40, 72, 136, 264, 1 << 30)
_WG_CHOICES = (0, 1, 2, 3, 4, 6, 8, 12, 16, 32)


def _bucket(n):
    for k in range(len(_BUCKETS) - 1):
        if _BUCKETS[k] <= n < _BUCKETS[k + 1]:
            return k
    return len(_BUCKETS) - 2


def size_classes(level):
    """Patch indices grouped by (x bucket, y bucket, periodic, frozen ghosts)."""
    cls = defaultdict(list)
    for k, (mx, my) in enumerate(level.shapes):
        cls[(_bucket(mx), _bucket(my), level.bcs[k] == "periodic", level.bcs[k] is None)].append(k)
    return dict(cls)


def candidates(mx, my, periodic, medium=False, frozen=False):
    """Tilings worth timing for patches of about mx x my cells: DIRECT and
    MARCH tiles (DIRECT only for periodic patches), and PACKED tiles for
    patches with frozen ghosts in a homogeneous medium.  In a heterogeneous
    medium DIRECT threads march up their column, so taller runs of rows per
    thread are tried too."""
    out = []
    rows = (1, 2, 4, 8, 16, 32, 64) if medium else (1, 2, 4, 8)
    for tw in (8, 16, 32, 64, 128):
        if tw > 2 * mx and tw > 8:
            continue
        nty = 256 // tw
        for r in rows:
            if nty * r > 2 * my and r > 1:
                continue
            out.append((DIRECT, tw, nty * r))
    if not periodic:
        for r in (4, 8, 12, 16, 18, 20, 24, 32, 48, 64):  # rows per one-wavefront segment
            if 4 * r > 2 * my and r > 4:
                continue
            out.append((MARCH, 64, 4 * r))
        if frozen and not medium:
            for r in (4, 8, 12, 16, 24, 32, 48, 64):  # rows per wavefront
                if 4 * r > 2 * my and r > 4:
                    continue
                out.append((PACKED, 64, 4 * r))
    return out


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tilings.json")


# The sources that decide how fast a tiling steps: the step kernels, the
# tables they read and the host code that builds the tile lists.
TILING_SOURCES = ("ws_api.hip", "ws_device.h", "ws_internal.h", "ws_kernels.hip", "ws_pack.h",
                  "ws_tables.h")


def _library_version():
    """SHA-1 of the library's step-kernel and tiling sources (TILING_SOURCES
    in name order): the same sources give the same kernels and tile lists,
    whichever build."""
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha1()
    for name in sorted(TILING_SOURCES):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:12]


def _key(level):
    arch = torch.cuda.get_device_properties(level.device).gcnArchName
    hist = sorted({(mx, my, str(level.bcs[k])) for k, (mx, my) in enumerate(level.shapes)})
    h = hashlib.sha1(json.dumps([hist, len(level.shapes)]).encode()).hexdigest()[:16]
    lim = level.limiter + ("+tc" if getattr(level, "transverse_corr", False) else "")
    lim += "+medium" if getattr(level, "medium", None) is not None else ""
    return f"{arch}|{_library_version()}|{level.dtype}|{lim}|{h}"


def _default_cache():
    return os.path.join(os.path.expanduser("~"), ".cache", "wavestep", "tiling.json")


def _apply(level, classes, choice, wg):
    var = np.zeros(level.n, dtype=object)
    tw = np.zeros(level.n, np.int32)
    th = np.zeros(level.n, np.int32)
    for c, idx in classes.items():
        v, w, h = choice[c]
        for k in idx:
            var[k], tw[k], th[k] = v, w, h
    level.set_tiling(tw, th, wg_per_cu=wg, variant=list(var))


def autotune(level, *, launches=40, use_cache=True, cache_path=None, verbose=False):
    """Pick a tiling for ``level`` and apply it.  Returns the choice as a dict
    {"classes": {class: (variant, tile_w, tile_h)}, "wg_per_cu": n, "ms": t}."""
    launches += launches % 2  # even: the state returns to its pool
    classes = size_classes(level)
    cache_path = cache_path or _default_cache()
    key = _key(level)
    cache = {}
    if use_cache and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    shipped = {}
    if use_cache and os.path.exists(SHIPPED):
        try:
            shipped = json.load(open(SHIPPED))
        except (OSError, ValueError):
            shipped = {}
    ent = shipped.get(key) if use_cache else None
    if ent is None and use_cache:
        ent = cache.get(key)
    if ent is not None:
        choice = {tuple(json.loads(c)): tuple(v) for c, v in ent["classes"].items()}
        if set(choice) == set(classes):
            _apply(level, classes, choice, ent["wg_per_cu"])
            return {"classes": choice, "wg_per_cu": ent["wg_per_cu"], "ms": ent["ms"],
                    "cached": True}

    # The timed steps run with the level's device dt: give it a stable one
    # for the duration (an unset dt steps garbage, whose timings mislead and
    # whose values need not even be finite), and keep the state to restore.
    dt_saved = level.read_dt_cfl()[0]
    dt_safe = level.stable_dt(0.5)
    level.set_dt(dt_safe)
    # saved and restored on the level's own stream, in order with its kernels
    torch.cuda.synchronize(level.device)
    with torch.cuda.stream(level.stream):
        saved = [p.clone() for p in level.pools]
    torch.cuda.synchronize(level.device)

    dt_step = float(min(dt_safe))

    def run(n):
        # n level steps back to back on the level's stream, as a captured
        # step loop runs them (an event pair around each launch would time
        # every launch from an idle GPU, which ranks close tilings otherwise)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(level.stream)
        for _ in range(n):
            level.step(dt_step, read_cfl=False)
        e1.record(level.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    seen = {}  # (choice, wg) -> best time

    def timed(choice, wg):
        # the faster of two timings: candidates a few percent apart would
        # otherwise trade places from run to run
        _apply(level, classes, choice, wg)
        run(2)
        t = min(run(launches), run(launches))
        k = (json.dumps(sorted((json.dumps(list(c)), list(v)) for c, v in choice.items())), wg)
        seen[k] = (min(t, seen[k][0]) if k in seen else t, dict(choice), wg)
        return t

    # start from the library's default tiling (the class's first patch)
    var0, tw0, th0, _wg0, _grid0 = level.get_tiling()
    choice = {c: (var0[idx[0]], int(tw0[idx[0]]), int(th0[idx[0]])) for c, idx in classes.items()}
    wg = 0
    best = timed(choice, wg)
    medium = getattr(level, "medium", None) is not None
    # Level-wide starts: every non-periodic class MARCH, or every class of
    # frozen-ghost patches PACKED (they share wavefronts only when packed
    # together, and a level of one tile kind runs a kernel of that kind
    # alone), over a few segment heights and workgroups per CU; then refine
    # class by class.
    nonper = [c for c in classes if not c[2]]
    frozen = [c for c in nonper if c[3]] if not medium else []
    starts = []
    for r in (4, 8, 16, 32, 64):
        if nonper:
            starts.append({c: (MARCH, 64, 4 * r) for c in nonper})
        if frozen:
            starts.append({c: (PACKED, 64, 4 * r) for c in frozen})
    for st in starts:
        trial = dict(choice)
        trial.update(st)
        for w in (0, 8, 16):
            try:
                t = timed(trial, w)
            except WaveStepError:  # a tiling some patch cannot take
                break
            if verbose:
                print(f"level-wide {sorted(set(st.values()))} wg {w}: {t:.4f} ms", flush=True)
            if t < best:
                best, choice, wg = t, trial, w
    order = sorted(classes, key=lambda c: -sum(level.shapes[k][0] * level.shapes[k][1]
                                                for k in classes[c]))
    for c in order:
        idx = classes[c]
        mx = int(np.median([level.shapes[k][0] for k in idx]))
        my = int(np.median([level.shapes[k][1] for k in idx]))
        for cand in candidates(mx, my, c[2], medium, c[3] and not medium):
            if cand == choice[c]:
                continue
            trial = dict(choice)
            trial[c] = cand
            try:
                t = timed(trial, wg)
            except WaveStepError:
                continue
            if verbose:
                print(f"class {c} {cand}: {t:.4f} ms", flush=True)
            if t < best:
                best, choice = t, trial
    for w in _WG_CHOICES:
        if w == wg:
            continue
        t = timed(choice, w)
        if verbose:
            print(f"wg_per_cu {w}: {t:.4f} ms", flush=True)
        if t < best:
            best, wg = t, w
    # a play-off of the four fastest configurations seen, timed in turns
    # with twice the launches, so that a timing a percent or two off does not
    # decide between near-equal candidates
    top = sorted(seen.values(), key=lambda e: e[0])[:4]
    if len(top) > 1:
        scores = [[] for _ in top]
        for _ in range(3):
            for k, (_, ch, w) in enumerate(top):
                _apply(level, classes, ch, w)
                run(2)
                scores[k].append(run(2 * launches))
        k = min(range(len(top)), key=lambda k: min(scores[k]))
        choice, wg, best = top[k][1], top[k][2], min(scores[k])
        if verbose:
            print("play-off:", [(round(min(sc), 4), e[2]) for sc, e in zip(scores, top)], flush=True)
    else:
        best = timed(choice, wg)
    _apply(level, classes, choice, wg)
    torch.cuda.synchronize(level.device)
    with torch.cuda.stream(level.stream):
        for p, s in zip(level.pools, saved):
            p.copy_(s)
    torch.cuda.synchronize(level.device)
    del saved
    level.set_dt([d if np.isfinite(d) and d > 0 else s for d, s in zip(dt_saved, dt_safe)])
    if use_cache:
        cache[key] = {"classes": {json.dumps(list(c)): list(v) for c, v in choice.items()},
                      "wg_per_cu": wg, "ms": best}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return {"classes": choice, "wg_per_cu": wg, "ms": best, "cached": False}
