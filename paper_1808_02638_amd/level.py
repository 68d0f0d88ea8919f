"""``Level``: one AMR level (or ensemble) of ghost-padded acoustics patches on
one GPU, advanced by the HIP library through its C ABI.

PyTorch provides the device memory (two q pools and a workspace, raw bytes)
and the stream; all arithmetic happens in the library's kernels.
"""

from __future__ import annotations

import ctypes
from typing import Iterable, Sequence

import numpy as np
import torch

from . import _lib as C

_LIMITERS = {"mc": C.WS_LIM_MC, "none": C.WS_LIM_NONE, "vanleer": C.WS_LIM_VANLEER}
_BCS = {None: C.WS_BC_NONE, "none": C.WS_BC_NONE, "extrap": C.WS_BC_EXTRAP,
        "periodic": C.WS_BC_PERIODIC}


def poisoned(nbytes: int, device) -> torch.Tensor:
    """Raw device bytes, every byte 0xFF: as FP64 or FP32 values that is a NaN.
    Pools and workspaces start out this way, so a kernel that read memory the
    library had not written would turn the result non-finite every time,
    instead of depending on what the allocator last held there."""
    return torch.full((max(int(nbytes), 1),), 0xFF, dtype=torch.uint8, device=device)


def _get(p, name, default=None):
    if isinstance(p, dict):
        return p.get(name, default)
    return getattr(p, name, default)


class Level:
    """Patches of one level, resident in HBM, stepped by one fused launch.

    patches: sequence of objects or dicts with mx, my, dx, dy and optionally
        instance (default 0) and bc ("extrap", "periodic" or None = frozen
        ghosts; default None).
    materials: sequence of (rho, K), one per instance.
    dtype: torch.float64 or torch.float32 (arithmetic and storage).
    limiter: "mc", "vanleer" or "none".
    transverse_corr: the variant whose transverse solver also splits the
        limited second-order correction (no branch recording or adjoint).
    """

    def __init__(self, patches: Sequence, materials: Sequence, *, dtype=torch.float64,
                 limiter: str = "mc", transverse_corr: bool = False, device="cuda",
                 stream: torch.cuda.Stream | None = None):
        self._L = C.lib()
        self._ctx = None
        self.dtype = dtype
        self.np_dtype = np.float64 if dtype == torch.float64 else np.float32
        if dtype not in (torch.float64, torch.float32):
            raise ValueError("dtype must be torch.float64 or torch.float32")
        self.n = len(patches)
        self.n_inst = len(materials)
        self.shapes = [(int(_get(p, "mx")), int(_get(p, "my"))) for p in patches]
        self.bcs = [_get(p, "bc", None) for p in patches]
        self.limiter = limiter
        self.transverse_corr = bool(transverse_corr)
        lim_code = _LIMITERS[limiter] | (C.WS_TRANSVERSE_CORR if transverse_corr else 0)
        descs = (C.PatchDesc * self.n)()
        for k, p in enumerate(patches):
            descs[k].mx, descs[k].my = self.shapes[k]
            descs[k].dx = float(_get(p, "dx"))
            descs[k].dy = float(_get(p, "dy"))
            descs[k].instance = int(_get(p, "instance", 0) or 0)
            descs[k].bc = _BCS[_get(p, "bc", None)]
        mats = (C.Material * self.n_inst)()
        for k, (rho, K) in enumerate(materials):
            mats[k].rho, mats[k].K = float(rho), float(K)
        # per patch: instance, cell sizes and the largest sound speed (for a
        # stable dt where none has been set, e.g. while timing tilings)
        self.instances = [int(descs[k].instance) for k in range(self.n)]
        self.cell_sizes = [(float(descs[k].dx), float(descs[k].dy)) for k in range(self.n)]
        self._cmax = [float(np.sqrt(float(materials[i][1]) / float(materials[i][0])))
                      for i in self.instances]
        code = C.WS_F64 if dtype == torch.float64 else C.WS_F32
        pool_b, ws_b = ctypes.c_int64(0), ctypes.c_int64(0)
        C.check(self._L.ws_layout(descs, self.n, self.n_inst, code, ctypes.byref(pool_b),
                                  ctypes.byref(ws_b)))
        self.device = torch.device(device)
        self.pool_bytes = pool_b.value
        self.pools = [poisoned(pool_b.value, self.device) for _ in range(2)]
        self.workspace = poisoned(ws_b.value, self.device)
        # A stream of our own (default priority): graph capture cannot use the
        # legacy null stream.  Allocation above ran on torch's stream.
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        ctx = ctypes.c_void_p()
        C.check(self._L.ws_init_patches(
            ctypes.byref(ctx), descs, self.n, mats, self.n_inst, 2, code, lim_code,
            ctypes.c_void_p(self.pools[0].data_ptr()), ctypes.c_void_p(self.pools[1].data_ptr()),
            pool_b.value, ctypes.c_void_p(self.workspace.data_ptr()), ws_b.value,
            ctypes.c_void_p(self.stream.cuda_stream)))
        self._ctx = ctx

    # ------------------------------------------------------------ medium
    def set_medium(self, k: int, rho, K) -> None:
        """Heterogeneous medium of patch k: rho, K as (my+4, mx+4) arrays (ghost
        cells included).  The first call attaches a medium buffer to the level
        and resets every patch to its default DIRECT tiles (set_tiling or the
        autotuner may then choose MARCH tiles); patches never given a medium
        keep whatever the buffer holds, so give every patch one."""
        mx, my = self.shapes[k]
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        if rho.shape != (my + 4, mx + 4) or K.shape != rho.shape:
            raise ValueError(f"patch {k}: rho and K must have shape {(my + 4, mx + 4)}")
        if getattr(self, "medium", None) is None:
            self.medium = poisoned(self.pool_bytes, self.device)
            torch.cuda.synchronize(self.device)
            C.check(self._L.ws_attach_medium(self._ctx, ctypes.c_void_p(self.medium.data_ptr()),
                                             self.pool_bytes))
        dp = ctypes.POINTER(ctypes.c_double)
        C.check(self._L.ws_upload_medium(self._ctx, k, rho.ctypes.data_as(dp),
                                         K.ctypes.data_as(dp)))
        self._cmax[k] = float(np.sqrt(K / rho).max())

    def link(self, origins, domain, periodic=(True, True)) -> None:
        """Make the level a tiled domain: patch k's interior cell (0, 0) sits at
        global cell origins[k] = (x0, y0) of a domain of domain = (DX, DY)
        cells, which the patches cover exactly; periodic per direction.  From
        now on every step refreshes the ghosts from the neighbouring patches
        (and the domain's physical condition), and fill_ghosts does too."""
        if len(origins) != self.n:
            raise ValueError("one origin per patch")
        org = np.ascontiguousarray(np.asarray(origins, dtype=np.int32).reshape(self.n, 2))
        nbytes = ctypes.c_int64(0)
        C.check(self._L.ws_link_layout(self._ctx, ctypes.byref(nbytes)))
        self.links = poisoned(nbytes.value, self.device)
        torch.cuda.synchronize(self.device)
        bits = (1 if periodic[0] else 0) | (2 if periodic[1] else 0)
        C.check(self._L.ws_link_level(self._ctx, org.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      int(domain[0]), int(domain[1]), bits,
                                      ctypes.c_void_p(self.links.data_ptr()), nbytes.value))

    # ------------------------------------------------------------------ data
    def upload(self, k: int, q) -> None:
        """Patch k's state in host layout (3, my+4, mx+4): a numpy array, or a
        torch tensor on the CPU or this GPU; written into both pools."""
        mx, my = self.shapes[k]
        if isinstance(q, torch.Tensor):
            t = q.detach().to(self.dtype).contiguous()
            if t.shape != (3, my + 4, mx + 4):
                raise ValueError(f"patch {k}: expected shape {(3, my + 4, mx + 4)}")
            if t.is_cuda:
                self.stream.wait_stream(torch.cuda.current_stream(self.device))
            C.check(self._L.ws_upload_patch(self._ctx, k, ctypes.c_void_p(t.data_ptr())))
            return
        a = np.ascontiguousarray(q, dtype=self.np_dtype)
        if a.shape != (3, my + 4, mx + 4):
            raise ValueError(f"patch {k}: expected shape {(3, my + 4, mx + 4)}")
        C.check(self._L.ws_upload_patch(self._ctx, k, a.ctypes.data_as(ctypes.c_void_p)))

    def download(self, k: int) -> np.ndarray:
        mx, my = self.shapes[k]
        a = np.empty((3, my + 4, mx + 4), dtype=self.np_dtype)
        C.check(self._L.ws_download_patch(self._ctx, k, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def fill_ghosts(self) -> None:
        C.check(self._L.ws_fill_ghosts(self._ctx))

    # ----------------------------------------------------------------- steps
    def step(self, dt: float, read_cfl: bool = True):
        """One level step with fixed dt; returns the level's Courant number
        (read_cfl=False: asynchronous, returns None)."""
        if not read_cfl:
            C.check(self._L.ws_step_level(self._ctx, float(dt), None))
            return None
        cfl = ctypes.c_double(0.0)
        C.check(self._L.ws_step_level(self._ctx, float(dt), ctypes.byref(cfl)))
        return cfl.value

    def step_per_patch(self, dt: float) -> float:
        cfl = ctypes.c_double(0.0)
        C.check(self._L.ws_step_level_per_patch(self._ctx, float(dt), ctypes.byref(cfl)))
        return cfl.value

    def stable_dt(self, cfl: float = 0.5) -> list:
        """Per instance, cfl times the smallest min(dx, dy) / c over its patches
        (c the largest sound speed of the patch's medium)."""
        dts = [float("inf")] * self.n_inst
        for k in range(self.n):
            i = self.instances[k]
            dts[i] = min(dts[i], cfl * min(self.cell_sizes[k]) / self._cmax[k])
        return [d if np.isfinite(d) else 1.0 for d in dts]

    def set_dt(self, dts: Iterable[float]) -> None:
        arr = (ctypes.c_double * self.n_inst)(*[float(v) for v in dts])
        C.check(self._L.ws_set_dt(self._ctx, arr))

    def step_auto(self, cfl_desired: float) -> None:
        C.check(self._L.ws_step_auto(self._ctx, float(cfl_desired)))

    def capture(self, n_steps: int, cfl_desired: float) -> None:
        C.check(self._L.ws_capture_steps(self._ctx, int(n_steps), float(cfl_desired)))

    def graph_launch(self) -> None:
        C.check(self._L.ws_graph_launch(self._ctx))

    def read_dt_cfl(self):
        n = self.n_inst
        dt, last, mx = (ctypes.c_double * n)(), (ctypes.c_double * n)(), (ctypes.c_double * n)()
        C.check(self._L.ws_read_dt_cfl(self._ctx, dt, last, mx))
        return np.array(dt), np.array(last), np.array(mx)

    def patch_cfl(self) -> np.ndarray:
        out = (ctypes.c_double * self.n)()
        C.check(self._L.ws_read_patch_cfl(self._ctx, out))
        return np.array(out)

    def conservation_sums(self) -> np.ndarray:
        out = (ctypes.c_double * (3 * self.n_inst))()
        C.check(self._L.ws_conservation_sums(self._ctx, out))
        return np.array(out).reshape(self.n_inst, 3)

    def set_tiling(self, tile_w=None, tile_h=None, wg_per_cu: int = 0, variant="direct") -> None:
        """Tiling per patch (scalars broadcast): variant "direct", "march" or
        "packed" (or 0/1/2 codes), tile width and height; and persistent
        workgroups per CU (0: as many as the kernel's occupancy allows).
        Without tile sizes the tiling in use is kept."""
        if tile_w is None:
            C.check(self._L.ws_set_tiling(self._ctx, None, None, None, int(wg_per_cu)))
            return
        codes = {"direct": C.WS_TILE_DIRECT, "march": C.WS_TILE_MARCH,
                 "packed": C.WS_TILE_PACKED}
        var = np.asarray([codes.get(v, v) if isinstance(v, str) else v
                          for v in np.broadcast_to(np.asarray(variant, dtype=object), (self.n,))],
                         np.int32)
        tw = np.broadcast_to(np.asarray(tile_w, np.int32), (self.n,)).copy()
        th = np.broadcast_to(np.asarray(tile_h, np.int32), (self.n,)).copy()
        P = ctypes.POINTER(ctypes.c_int32)
        C.check(self._L.ws_set_tiling(self._ctx, var.ctypes.data_as(P), tw.ctypes.data_as(P),
                                      th.ctypes.data_as(P), int(wg_per_cu)))

    # --------------------------------------------------------------- adjoint
    # Buffers passed in come from torch's current stream: the level's stream
    # waits for it before the library reads them, and torch's stream waits
    # for the level's stream before it reads what the library wrote.
    def _on_level_stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream == self.stream.cuda_stream

    def _sync_in(self):
        if not self._on_level_stream():
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _sync_out(self):
        if not self._on_level_stream():
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def mask_bytes(self) -> int:
        b = ctypes.c_int64(0)
        C.check(self._L.ws_mask_bytes(self._ctx, ctypes.byref(b)))
        return b.value

    def new_masks(self) -> torch.Tensor:
        """A device buffer for the branches of one step."""
        return poisoned(self.mask_bytes(), self.device)

    def new_buffer(self) -> torch.Tensor:
        """A zeroed FP64 device buffer in the pools' layout (for cotangents)."""
        if self.dtype != torch.float64:
            raise ValueError("cotangent buffers are FP64")
        return torch.zeros(self.pool_bytes // 8, dtype=torch.float64, device=self.device)

    def patch_view(self, buf: torch.Tensor, k: int) -> torch.Tensor:
        """Patch k of a pool-layout buffer as a (3, my+4, mx+4) strided view
        (ghost-padded; interior is [:, 2:-2, 2:-2])."""
        off, ld, plane = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        C.check(self._L.ws_patch_layout(self._ctx, int(k), ctypes.byref(off), ctypes.byref(ld),
                                        ctypes.byref(plane)))
        mx, my = self.shapes[k]
        return buf.as_strided((3, my + 4, mx + 4), (plane.value, ld.value, 1), off.value)

    def state_view(self, k: int) -> torch.Tensor:
        """Patch k of the current state (a view into the live pool)."""
        pool = self.pools[self.current_pool()].view(self.dtype)
        return self.patch_view(pool, k)

    def step_record_masks(self, dt: float, masks: torch.Tensor) -> None:
        """One level step with fixed dt that records its MC branches."""
        self._check_masks(masks)
        self._sync_in()
        C.check(self._L.ws_step_record_masks(self._ctx, float(dt),
                                             ctypes.c_void_p(masks.data_ptr()), None))
        self._sync_out()

    def adjoint_step(self, dt: float, masks: torch.Tensor, lam_in: torch.Tensor,
                     lam_out: torch.Tensor) -> None:
        """lam_out <- S^T lam_in for the step recorded in ``masks``."""
        self._check_masks(masks)
        for b in (lam_in, lam_out):
            self._check_buffer(b)
        self._sync_in()
        C.check(self._L.ws_adjoint_step(self._ctx, float(dt), ctypes.c_void_p(masks.data_ptr()),
                                        ctypes.c_void_p(lam_in.data_ptr()),
                                        ctypes.c_void_p(lam_out.data_ptr())))
        self._sync_out()

    def _cells(self, k, ij):
        mx, my = self.shapes[k]
        if not (isinstance(ij, torch.Tensor) and ij.dtype == torch.int32 and ij.is_cuda
                and ij.is_contiguous() and ij.dim() == 2 and ij.shape[1] == 2):
            raise ValueError("ij must be a contiguous int32 device tensor of shape (n, 2)")
        return ij.shape[0]

    def gather(self, k: int, comp: int, ij: torch.Tensor, out: torch.Tensor,
               buf: torch.Tensor | None = None) -> None:
        """out[n] = buf(comp, i_n, j_n) of patch k (buf None: the current state)."""
        n = self._cells(k, ij)
        if out.dtype != torch.float64 or not out.is_contiguous() or out.numel() < n:
            raise ValueError("out must be a contiguous FP64 device tensor of n values")
        if buf is not None:
            self._check_buffer(buf)
        self._sync_in()
        C.check(self._L.ws_gather(self._ctx, None if buf is None else ctypes.c_void_p(buf.data_ptr()),
                                  int(k), int(comp), n, ctypes.c_void_p(ij.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr())))
        self._sync_out()

    def add_at(self, k: int, comp: int, ij: torch.Tensor, val: torch.Tensor,
               buf: torch.Tensor | None = None) -> None:
        """buf(comp, i_n, j_n) += val[n] of patch k (buf None: the current state)."""
        n = self._cells(k, ij)
        if val.dtype != torch.float64 or not val.is_contiguous() or val.numel() < n:
            raise ValueError("val must be a contiguous FP64 device tensor of n values")
        if buf is not None:
            self._check_buffer(buf)
        self._sync_in()
        C.check(self._L.ws_add_at(self._ctx, None if buf is None else ctypes.c_void_p(buf.data_ptr()),
                                  int(k), int(comp), n, ctypes.c_void_p(ij.data_ptr()),
                                  ctypes.c_void_p(val.data_ptr())))
        self._sync_out()

    def _check_masks(self, masks):
        if not (isinstance(masks, torch.Tensor) and masks.dtype == torch.uint8 and masks.is_cuda
                and masks.is_contiguous() and masks.numel() >= self.mask_bytes()):
            raise ValueError("masks must be a contiguous uint8 device tensor of mask_bytes()")

    def _check_buffer(self, b):
        if not (isinstance(b, torch.Tensor) and b.dtype == torch.float64 and b.is_cuda
                and b.is_contiguous() and b.numel() * 8 >= self.pool_bytes):
            raise ValueError("buffers must be contiguous FP64 device tensors of pool_bytes")

    def get_tiling(self):
        """(variants, tile_w, tile_h, wg_per_cu, grid) in use; variants as
        "direct"/"march"/"packed" strings."""
        P = ctypes.POINTER(ctypes.c_int32)
        var = np.zeros(self.n, np.int32)
        tw = np.zeros(self.n, np.int32)
        th = np.zeros(self.n, np.int32)
        wg, grid = ctypes.c_int32(0), ctypes.c_int32(0)
        C.check(self._L.ws_get_tiling(self._ctx, var.ctypes.data_as(P), tw.ctypes.data_as(P),
                                      th.ctypes.data_as(P), ctypes.byref(wg), ctypes.byref(grid)))
        names = {C.WS_TILE_DIRECT: "direct", C.WS_TILE_MARCH: "march",
                 C.WS_TILE_PACKED: "packed"}
        return [names[int(v)] for v in var], tw, th, wg.value, grid.value

    def time_step_kernel(self, n_launches: int, per_patch: bool = False) -> float:
        """Mean milliseconds per level step of n back-to-back step launches
        (HIP events on the level's stream; fixed device dt, no dt update)."""
        ms = ctypes.c_double(0.0)
        C.check(self._L.ws_time_step_kernel(self._ctx, int(n_launches), int(bool(per_patch)),
                                            ctypes.byref(ms)))
        return ms.value

    def current_pool(self) -> int:
        w = ctypes.c_int32(0)
        C.check(self._L.ws_current_pool(self._ctx, ctypes.byref(w)))
        return w.value

    def close(self) -> None:
        if self._ctx is not None:
            self._L.ws_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _tables(patches: Sequence, materials: Sequence):
    """The C patch-descriptor and material arrays of a patch list."""
    descs = (C.PatchDesc * len(patches))()
    for k, p in enumerate(patches):
        descs[k].mx, descs[k].my = int(_get(p, "mx")), int(_get(p, "my"))
        descs[k].dx = float(_get(p, "dx"))
        descs[k].dy = float(_get(p, "dy"))
        descs[k].instance = int(_get(p, "instance", 0) or 0)
        descs[k].bc = _BCS[_get(p, "bc", None)]
    mats = (C.Material * len(materials))()
    for k, (rho, K) in enumerate(materials):
        mats[k].rho, mats[k].K = float(rho), float(K)
    return descs, mats


def step_level_noalloc(patches: Sequence, materials: Sequence, q_in: torch.Tensor,
                       q_out: torch.Tensor, dt: float, *, dtype=torch.float64,
                       limiter: str = "mc", transverse_corr: bool = False,
                       stream: torch.cuda.Stream | None = None) -> float:
    """``ws_step_level_noalloc``: one level step from the pool-layout buffer
    q_in into q_out (device tensors of the pool size ``ws_layout`` gives for
    this patch list) with the library's own scratch array in place of a
    workspace; returns the level's Courant number.  Synchronises ``stream``
    (default: torch's current stream)."""
    L = C.lib()
    descs, mats = _tables(patches, materials)
    code = C.WS_F64 if dtype == torch.float64 else C.WS_F32
    lim = _LIMITERS[limiter] | (C.WS_TRANSVERSE_CORR if transverse_corr else 0)
    nbytes = min(q_in.numel() * q_in.element_size(), q_out.numel() * q_out.element_size())
    s = stream if stream is not None else torch.cuda.current_stream(q_in.device)
    cfl = ctypes.c_double(0.0)
    C.check(L.ws_step_level_noalloc(descs, len(patches), mats, len(materials), code, lim,
                                    ctypes.c_void_p(q_in.data_ptr()),
                                    ctypes.c_void_p(q_out.data_ptr()), int(nbytes), float(dt),
                                    ctypes.byref(cfl), ctypes.c_void_p(s.cuda_stream)))
    return cfl.value
