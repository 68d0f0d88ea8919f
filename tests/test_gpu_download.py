"""Downloads of patches: ws_download_patch into pageable host memory (staged
through the context's pinned buffer a block of rows at a time) and into a
device buffer give, bitwise, the current state as the device holds it (read
back through torch from the pool itself), for patches smaller and larger
than the staging buffer, in FP64 and FP32."""

import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_download_equals_device_state(dtype):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1808_02638_amd as ws
    from paper_1808_02638_amd import _lib as C

    shapes = [(1100, 1050), (37, 20), (1, 1), (300, 2)]
    lev = ws.Level([dict(mx=mx, my=my, dx=1 / mx, dy=1 / my, bc="extrap") for mx, my in shapes],
                   [(1.0, 4.0)], dtype=dtype)
    rng = np.random.default_rng(7)
    for k, (mx, my) in enumerate(shapes):
        lev.upload(k, 1.0 + 0.1 * rng.standard_normal((3, my + 4, mx + 4)))
    lev.fill_ghosts()
    dt = 0.4 * min(lev.stable_dt(1.0))
    for _ in range(3):
        lev.step(dt)
    torch.cuda.synchronize()
    pool = lev.pools[lev.current_pool()].view(dtype)
    for k, (mx, my) in enumerate(shapes):
        ref = lev.patch_view(pool, k).cpu().numpy()
        got = lev.download(k)
        assert got.dtype == ref.dtype and got.shape == ref.shape
        assert np.array_equal(got.view(np.uint8), np.ascontiguousarray(ref).view(np.uint8)), k
        dev = torch.empty((3, my + 4, mx + 4), dtype=dtype, device="cuda")
        C.check(lev._L.ws_download_patch(lev._ctx, k, ctypes.c_void_p(dev.data_ptr())))
        assert torch.equal(dev.cpu(), torch.from_numpy(np.ascontiguousarray(ref))), k
    lev.close()
