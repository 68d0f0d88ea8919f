"""CPU checks of the tile lists the library builds for a level (no GPU).

The library's builders (``csrc/ws_pack.h``: PACKED tiles and conservation-sum
tiles) are compiled with g++ into a small driver that prints the tables; the
tests replay on them the lane arithmetic of the step kernel's PACKED branch
and the index arithmetic of the sum kernel, and check what the kernels
assume:

* every interior cell of every PACKED patch is updated by exactly one lane
  and row of one wavefront, and the lanes within two of an updating lane
  (the stencil's reach through the lane shifts) hold the neighbouring
  columns of the same patch;
* the byte offsets a lane forms from its piece's entries (column read,
  column stored, row and plane strides) are those of its patch's column in
  the pool layout; every column a lane reads lies in the patch's padded
  storage, and the rows a wavefront marches over lie in every one of its
  patches;
* the blocks of a wavefront sit side by side from lane 0, at most four, within
  64 lanes; all patches of a tile share instance and cell sizes (the tile's
  one Courant number and coefficients); a tile's wavefronts are stacked row
  segments of the same blocks (so the rows two of them share are read by one
  workgroup); a patch's tile_begin names a tile that holds it;
* the wavefront list stays within the bound the workspace is sized by;
* every cell of every patch lies in exactly one sum tile.
"""

import os
import subprocess

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "native", "pack_dump.cpp")
DIRECT, MARCH, PACKED = 0, 1, 2
LANES = 64


@pytest.fixture(scope="module")
def dump(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("pack") / "pack_dump")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", exe, DRIVER],
                   check=True)

    def run(patches):
        """patches: list of (mx, my, inst, dx, dy, variant, th)."""
        text = f"{len(patches)}\n" + "".join(
            f"{mx} {my} {inst} {dx!r} {dy!r} {v} {th}\n"
            for mx, my, inst, dx, dy, v, th in patches)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        P, T, S, W, bound = {}, [], [], [], None
        for line in out.splitlines():
            f = line.split()
            if f[0] == "P":
                P[int(f[1])] = tuple(int(x) for x in f[2:])  # tile_begin, n, sum_begin, n, layout
            elif f[0] == "T":
                T.append(tuple(int(x) for x in f[1:]))
            elif f[0] == "S":
                S.append(tuple(int(x) for x in f[1:]))
            elif f[0] == "W":
                v = [int(x) for x in f[1:]]
                W.append(dict(r0=v[0], r1=v[1], n=v[2], patch=v[3:7], c0=v[7:11], w=v[11:15],
                              lane0=v[15:19], org=v[19:23], ldb=v[23:27], plb=v[27:31],
                              lim=v[31:35]))
            elif f[0] == "BOUND":
                bound = int(f[1])
        return P, T, S, W, bound

    return run


ES = 8  # the dump program lays out FP64 pools


def lane_map(pw, shapes, P):
    """The PACKED branch's per-lane piece and its byte offsets as the kernel
    forms them from the piece's entries, checked against the column the lane
    holds (i) and reads (ic) in its patch's layout."""
    out = []
    for lx in range(LANES):
        pc = 0
        for n in range(1, pw["n"]):
            if lx >= pw["lane0"][n]:
                pc = n
        off = lx - pw["lane0"][pc]
        colb = pw["org"][pc] + min(off, pw["lim"][pc]) * ES
        ocolb = pw["org"][pc] + off * ES
        upd = 2 <= off < pw["w"][pc] + 2
        k = pw["patch"][pc]
        mx, _my = shapes[k]
        q_off, col0, ld, plane = P[k][4:8]
        i = pw["c0"][pc] - 2 + off
        ic = min(i, mx + 1)
        assert colb == (q_off + col0 + ic) * ES
        assert pw["ldb"][pc] == ld * ES and pw["plb"][pc] == plane * ES
        if upd:
            assert i < mx and ocolb == (q_off + col0 + i) * ES
        out.append((pc, k, i, ic, upd))
    return out


def check_level(dump, patches):
    P, T, S, W, bound = dump(patches)
    n = len(patches)
    shapes = [(p[0], p[1]) for p in patches]
    key = [(p[2], p[3], p[4]) for p in patches]
    packed = [k for k in range(n) if patches[k][5] == PACKED]
    cover = {k: np.zeros((shapes[k][1], shapes[k][0]), np.int32) for k in packed}

    assert len(W) <= bound
    assert len(W) % 4 == 0
    seen_waves = np.zeros(len(W), np.int32)
    tile_patches = {}
    for t, (tp, _tx, _ty) in enumerate(T):
        assert tp < 0, "only PACKED tiles come from the packer"
        g = -1 - tp
        assert 4 * g + 3 < len(W)
        keys = set()
        members = set()
        for q in range(4 * g, 4 * g + 4):
            seen_waves[q] += 1
            pw = W[q]
            keys.add(key[pw["patch"][0]])
            assert 0 <= pw["n"] <= 4
            if pw["n"] == 0:
                continue
            # blocks side by side from lane 0, within the wavefront
            assert pw["lane0"][0] == 0
            for m in range(1, pw["n"]):
                assert pw["lane0"][m] == pw["lane0"][m - 1] + pw["w"][m - 1] + 4
            last = pw["n"] - 1
            assert pw["lane0"][last] + pw["w"][last] + 4 <= LANES
            for m in range(pw["n"]):
                k = pw["patch"][m]
                assert patches[k][5] == PACKED
                keys.add(key[k])
                members.add(k)
                mx, my = shapes[k]
                assert 1 <= pw["w"][m] <= 60
                assert 0 <= pw["c0"][m] and pw["c0"][m] + pw["w"][m] <= mx
                # the march's rows (and the two above and below it) exist
                assert 0 <= pw["r0"] < pw["r1"] <= my
            lm = lane_map(pw, shapes, P)
            for lx, (pc, k, i, ic, upd) in enumerate(lm):
                mx, my = shapes[k]
                assert -2 <= ic <= mx + 1  # the column read lies in the padded patch
                if not upd:
                    continue
                for d in (-2, -1, 1, 2):  # the stencil's reach through lane shifts
                    assert 0 <= lx + d < LANES
                    pc2, k2, i2, _, _ = lm[lx + d]
                    assert (pc2, k2, i2) == (pc, k, i + d)
                cover[k][pw["r0"]:pw["r1"], i] += 1
        assert len(keys) == 1, "a tile's patches share instance, dx and dy"
        # the tile's wavefronts: stacked segments of one lane column
        full = [W[q] for q in range(4 * g, 4 * g + 4) if W[q]["n"] > 0]
        assert full and full == [W[q] for q in range(4 * g, 4 * g + len(full))]
        for a, b in zip(full, full[1:]):
            assert a["r1"] == b["r0"]
            assert all(a[f] == b[f] for f in ("n", "patch", "c0", "w", "lane0", "org"))
        tile_patches[t] = members
    assert (seen_waves == 1).all()
    for k in packed:
        assert (cover[k] == 1).all(), f"patch {k}: cells updated {cover[k].min()}..{cover[k].max()}"
        tb, nt = P[k][0], P[k][1]
        assert nt == 1 and k in tile_patches[tb]

    # sum tiles: the sum kernel's mapping (64 columns, 4 x 16 rows per tile)
    for k in range(n):
        mx, my = shapes[k]
        sb, sn = P[k][2], P[k][3]
        cnt = np.zeros((my, mx), np.int32)
        for (sp, tx, ty) in S[sb:sb + sn]:
            assert sp == k
            for ly in range(4):
                j0 = ty * 64 + ly * 16
                j1 = min(j0 + 16, my)
                i0, i1 = tx * 64, min(tx * 64 + 64, mx)
                if j0 < j1 and i0 < i1:
                    cnt[j0:j1, i0:i1] += 1
        assert (cnt == 1).all()
    assert sum(P[k][3] for k in range(n)) == len(S)
    return P, T, W


@pytest.mark.parametrize("th", [16, 32, 64, 128, 256])
def test_amr_level_batch_all_packed(dump, th):
    """The benchmark's three AMR levels, every patch PACKED."""
    for specs in workloads.amr_level_batch():
        patches = [(p.mx, p.my, 0, p.dx, p.dy, PACKED, th) for p in specs]
        _, _, W = check_level(dump, patches)
        # lanes that update cells: far more than one MARCH segment per patch gives
        busy = sum(sum(pw["w"][:pw["n"]]) for pw in W)
        segs = [-(-p.my // -(-p.my // (4 * -(-p.my // th)))) for p in specs]  # rows spread evenly
        assert busy == sum(p.mx * s for p, s in zip(specs, segs))
        # a patch no taller than its tile spreads its rows over the four
        # wavefronts: none idles (the benchmark's patches are >= 16 rows tall)
        if th >= 64:
            assert all(pw["n"] > 0 for pw in W)


def test_mixed_variants_instances_and_sizes(dump):
    rng = np.random.default_rng(5)
    patches = []
    for _ in range(300):
        mx, my = int(rng.integers(1, 200)), int(rng.integers(1, 150))
        v = int(rng.choice([DIRECT, MARCH, PACKED, PACKED]))
        th = int(rng.choice([16, 20, 24, 64, 100, 256])) if v == PACKED else 64
        patches.append((mx, my, int(rng.integers(0, 3)), float(rng.choice([0.5, 0.25])),
                        float(rng.choice([0.5, 0.125])), v, th))
    check_level(dump, patches)


def test_degenerate_shapes(dump):
    shapes = [(1, 1), (1, 5), (5, 1), (60, 4), (61, 5), (64, 64), (300, 7), (7, 300), (8, 3),
              (59, 1), (2, 2), (121, 17)]
    for th in (16, 28, 256):
        check_level(dump, [(mx, my, 0, 1.0, 1.0, PACKED, th) for mx, my in shapes])


def test_wavefront_fill(dump):
    """Next-fit packing leaves few lanes idle: on the finest benchmark level
    at least 80% of the lanes update a cell (one MARCH segment per 16..64-wide
    patch averages about 60%)."""
    specs = workloads.amr_level_batch()[-1]
    patches = [(p.mx, p.my, 0, p.dx, p.dy, PACKED, 64) for p in specs]
    _, _, W = check_level(dump, patches)
    work = [pw for pw in W if pw["n"] > 0]
    busy = sum(sum(pw["w"][:pw["n"]]) for pw in work)
    assert busy / (LANES * len(work)) >= 0.80
