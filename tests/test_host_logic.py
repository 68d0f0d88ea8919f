"""Host-side logic that needs no GPU: the autotuner's candidate tilings and
the benchmark layouts' agreement with the layout rules of the composite step
and the tiled level (checked by the oracle's own layout checks)."""

import numpy as np

import workloads
from oracle import amr as oamr
from oracle import tiled as otiled
from paper_1808_02638_amd.autotune import DIRECT, MARCH, PACKED, candidates


def test_candidates_cover_the_tile_kinds_each_level_may_take():
    plain = candidates(120, 120, periodic=False)
    assert any(v == MARCH for v, _, _ in plain) and any(v == DIRECT for v, _, _ in plain)
    # DIRECT tiles: at most 8 rows per thread unless the medium marches columns
    assert max(th // (256 // tw) for v, tw, th in plain if v == DIRECT) == 8
    direct_only = candidates(120, 120, periodic=True)
    assert all(v == DIRECT for v, _, _ in direct_only)
    medium = candidates(2048, 2048, periodic=True, medium=True)
    assert all(v == DIRECT for v, _, _ in medium)
    assert max(th // (256 // tw) for _, tw, th in medium) == 64
    # PACKED tiles for patches with frozen ghosts only, 4..64 rows per wavefront
    assert not any(v == PACKED for v, _, _ in plain)
    frozen = candidates(40, 40, periodic=False, frozen=True)
    packed = [th for v, _, th in frozen if v == PACKED]
    assert packed and min(packed) >= 16 and max(packed) <= 256
    # every candidate is a whole number of rows per thread / per segment
    for v, tw, th in plain + medium + frozen:
        assert th % (256 // tw) == 0


def test_benchmark_hierarchies_satisfy_the_composite_layout_rules():
    n, r = 1024, 4
    rects = workloads.two_level_layout(n)
    fines = [oamr.FinePatch(ci0, cj0, w, h, np.zeros((3, r * h + 4, r * w + 4)))
             for (ci0, cj0, w, h) in rects]
    oamr.check_layout(n, n, fines, r)
    l1, l2 = workloads.three_level_layout(512)
    by_parent = {}
    for (p, ci0, cj0, w, h) in l2:
        by_parent.setdefault(p, []).append(oamr.FinePatch(ci0, cj0, w, h,
                                                          np.zeros((3, r * h + 4, r * w + 4)), p))
    for p, kids in by_parent.items():
        _, _, w, h = l1[p]
        oamr.check_layout(r * w, r * h, kids, r)


def test_benchmark_tiling_covers_its_domain():
    n, t = 2048, 4
    w = n // t
    origins = [(w * a, w * b) for b in range(t) for a in range(t)]
    own = otiled.owner_map([(w, w)] * len(origins), origins, (n, n))
    assert own.min() == 0 and own.max() == len(origins) - 1
