"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side validation rejects bad arguments before touching a GPU."""

import ctypes
import os

import pytest

from helpers import ROOT, header_symbols

LIB = os.path.join(ROOT, "paper_1808_02638_amd", "libwavestep.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libwavestep.so is not built (run __graft_entry__.build())")
    from paper_1808_02638_amd import _lib
    return _lib.lib()


def test_every_header_symbol_is_exported(L):
    from paper_1808_02638_amd import _lib
    declared = header_symbols()
    assert declared, "no declarations parsed"
    assert sorted(declared) == sorted(_lib.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_symbols_have_c_linkage():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    names = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in header_symbols():
        assert name in names, f"{name} missing or mangled"


def _descs(C, shapes, bc=0):
    d = (C.PatchDesc * len(shapes))()
    for k, (mx, my) in enumerate(shapes):
        d[k].mx, d[k].my, d[k].dx, d[k].dy, d[k].instance, d[k].bc = mx, my, 1 / mx, 1 / my, 0, bc
    return d


def test_layout_sizes(L):
    from paper_1808_02638_amd import _lib as C
    pool, ws = ctypes.c_int64(), ctypes.c_int64()
    d = _descs(C, [(2048, 2048)])
    assert L.ws_layout(d, 1, 1, C.WS_F64, ctypes.byref(pool), ctypes.byref(ws)) == 0
    # at least the padded cells, at most a few per cent above (row alignment)
    assert 3 * 2052 * 2052 * 8 <= pool.value <= 1.05 * 3 * 2052 * 2052 * 8
    pool32 = ctypes.c_int64()
    assert L.ws_layout(d, 1, 1, C.WS_F32, ctypes.byref(pool32), None) == 0
    assert abs(pool32.value * 2 - pool.value) <= 0.05 * pool.value
    d2 = _descs(C, [(16, 64), (64, 16), (33, 17)])
    assert L.ws_layout(d2, 3, 1, C.WS_F64, ctypes.byref(pool), ctypes.byref(ws)) == 0
    assert pool.value % 256 == 0 and ws.value % 256 == 0


@pytest.mark.parametrize("case", ["zero_size", "bad_dx", "bad_instance", "bad_bc", "periodic_1",
                                  "no_patches", "bad_dtype"])
def test_layout_rejects_bad_descriptors(L, case):
    from paper_1808_02638_amd import _lib as C
    d = _descs(C, [(8, 8)])
    n, n_inst, dtype = 1, 1, C.WS_F64
    if case == "zero_size":
        d[0].mx = 0
    elif case == "bad_dx":
        d[0].dx = -1.0
    elif case == "bad_instance":
        d[0].instance = 3
    elif case == "bad_bc":
        d[0].bc = 9
    elif case == "periodic_1":
        d[0].mx, d[0].bc = 1, C.WS_BC_PERIODIC
    elif case == "no_patches":
        n = 0
    elif case == "bad_dtype":
        dtype = 7
    rc = L.ws_layout(d, n, n_inst, dtype, None, None)
    assert rc == C.WS_EINVAL
    assert L.ws_last_error().decode()


def test_init_validates_before_touching_the_gpu(L):
    from paper_1808_02638_amd import _lib as C
    d = _descs(C, [(8, 8)], bc=C.WS_BC_EXTRAP)
    m = (C.Material * 1)()
    m[0].rho, m[0].K = 1.0, 4.0
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    fake2 = ctypes.c_void_p(0x2000)
    # mbc must be 2
    assert L.ws_init_patches(ctypes.byref(ctx), d, 1, m, 1, 3, 0, 0, fake, fake2, 1 << 20, fake,
                             1 << 20, None) == C.WS_EINVAL
    assert "mbc" in L.ws_last_error().decode()
    # unknown limiter
    assert L.ws_init_patches(ctypes.byref(ctx), d, 1, m, 1, 2, 0, 5, fake, fake2, 1 << 20, fake,
                             1 << 20, None) == C.WS_EINVAL
    # bad material
    m[0].rho = 0.0
    assert L.ws_init_patches(ctypes.byref(ctx), d, 1, m, 1, 2, 0, 0, fake, fake2, 1 << 20, fake,
                             1 << 20, None) == C.WS_EINVAL
    m[0].rho = 1.0
    # same pool twice
    assert L.ws_init_patches(ctypes.byref(ctx), d, 1, m, 1, 2, 0, 0, fake, fake, 1 << 20, fake,
                             1 << 20, None) == C.WS_EINVAL
    # undersized pool / workspace
    assert L.ws_init_patches(ctypes.byref(ctx), d, 1, m, 1, 2, 0, 0, fake, fake2, 64, fake,
                             1 << 20, None) == C.WS_ENOMEM
    assert L.ws_init_patches(ctypes.byref(ctx), d, 1, m, 1, 2, 0, 0, fake, fake2, 1 << 20, fake,
                             64, None) == C.WS_ENOMEM
    assert not ctx.value


def test_null_context_is_rejected(L):
    from paper_1808_02638_amd import _lib as C
    cfl = ctypes.c_double()
    assert L.ws_step_level(None, 0.1, ctypes.byref(cfl)) == C.WS_EINVAL
    assert L.ws_graph_launch(None) == C.WS_EINVAL
    assert L.ws_fill_ghosts(None) == C.WS_EINVAL
    assert L.ws_destroy(None) == C.WS_OK


def test_product_package_never_imports_the_oracle():
    """The library path must not reach the test oracle (nor any CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_1808_02638_amd")
    for dirpath, _dirs, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("oracle is the oracle", ""), f
