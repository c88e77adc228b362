"""polyrecon: polyline-array near-field MMW imaging on an AMD MI355X (gfx950).

A thin ctypes binding over ``libpolyrecon.so`` (declared in
``include/polyrecon.h``).  Every computation runs in the library's HIP
kernels; this module only marshals arguments, and uses PyTorch for device
memory and the current stream.  There is no CPU fallback: if the library is
missing, loading fails loudly.

Entry points keep the C names: make_geometry, simulate_echo,
reconstruct_hybrid, reconstruct_bp, plus the plan queries and the four
steps of the hybrid method (scan_fft, range_compress, backproject, kz_ifft).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpolyrecon.so")

PL_OK, PL_EINVAL, PL_EGEOM, PL_EDEVICE, PL_EWORKSPACE, PL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PL_MONO, PL_MULTI = 0, 1
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
INTERPS = {"bspline4": 0, "lagrange4": 1, "linear": 2}
BP_KERNELS = {0: "kz-lanes", 1: "pixel-lanes", 2: "mfma", 3: "mfma-1pass"}
RANGE_METHODS = {"nufft": 0, "resample": 1}
REF_MODES = {"band-centre": 0, "min-k": 1}
WARN_ELEMENT_SPACING, WARN_SCAN_STEP = 1, 2

_ERRNAMES = {PL_EINVAL: "PL_EINVAL", PL_EGEOM: "PL_EGEOM", PL_EDEVICE: "PL_EDEVICE",
             PL_EWORKSPACE: "PL_EWORKSPACE", PL_EUNSUPPORTED: "PL_EUNSUPPORTED"}


class PolyreconError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class GeometryDesc(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_chords", C.c_int32), ("radius_m", C.c_double),
                ("arc_center_rad", C.c_double), ("n_elem", C.c_int32), ("n_tx", C.c_int32),
                ("spacing_m", C.c_double), ("tx_offsets_m", C.POINTER(C.c_double)),
                ("n_scan", C.c_int32), ("n_freq", C.c_int32), ("scan_step_m", C.c_double),
                ("scan_z0_m", C.c_double), ("f_start_hz", C.c_double), ("f_stop_hz", C.c_double)]


class GeometryInfo(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("mode", "n_chords", "n_channels", "n_scan", "n_freq",
                                         "n_tx", "n_elem", "reserved")]


class ImageGridC(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("x0", C.c_double), ("y0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double)]


class HybridOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("interp", C.c_int32), ("l_oversample", C.c_double),
                ("nufft_tol", C.c_double), ("tile", C.c_int32), ("kz_per_lane", C.c_int32),
                ("waves", C.c_int32), ("mfma_backprojection", C.c_int32), ("tile_y", C.c_int32),
                ("kz_block", C.c_int32), ("range_method", C.c_int32), ("ref_mode", C.c_int32)]


class HybridPlanInfo(C.Structure):
    _fields_ = [("n_kz", C.c_int32), ("n_l", C.c_int32), ("n_fine", C.c_int32),
                ("kernel_width", C.c_int32), ("n_blocks", C.c_int32), ("block", C.c_int32),
                ("window", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32),
                ("bp_kernel", C.c_int32), ("waves", C.c_int32), ("du", C.c_double), ("beta", C.c_double),
                ("workspace_bytes", C.c_size_t), ("range_method", C.c_int32), ("dk_uniform", C.c_double),
                ("scan_fft_len", C.c_int32), ("reserved_", C.c_int32)]


_P = C.c_void_p
_SIGNATURES = {
    "make_geometry": (C.c_int, [C.POINTER(GeometryDesc), C.POINTER(_P)]),
    "destroy_geometry": (C.c_int, [_P]),
    "geometry_upload": (C.c_int, [_P, _P]),
    "geometry_info": (C.c_int, [_P, C.POINTER(GeometryInfo), _P, _P, _P, _P, _P]),
    "check_sampling": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(C.c_uint32)]),
    "simulate_echo": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
    "hybrid_plan_info": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts),
                                   C.POINTER(HybridPlanInfo), _P]),
    "hybrid_workspace_bytes": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts),
                                         C.POINTER(C.c_size_t)]),
    "reconstruct_hybrid": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P, _P,
                                     C.c_size_t, _P]),
    "reconstruct_hybrid_prepared": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P, _P,
                                              C.c_size_t, _P]),
    "hybrid_prepare": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, C.c_size_t, _P]),
    "reconstruct_hybrid_static": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P, _P]),
    "adjoint_hybrid": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P, _P,
                                 C.c_size_t, _P]),
    "reconstruct_hybrid_events": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P,
                                            _P, C.c_size_t, _P, _P]),
    "fft_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "scan_fft": (C.c_int, [_P, _P, _P, _P, C.c_size_t, _P]),
    "range_compress": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P, _P, _P,
                                 C.c_size_t, _P]),
    "backproject": (C.c_int, [_P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), _P, _P, _P,
                              C.c_size_t, _P]),
    "kz_ifft": (C.c_int, [_P, C.POINTER(ImageGridC), _P, _P, _P, C.c_size_t, _P]),
    "bp_workspace_bytes": (C.c_int, [_P, C.POINTER(ImageGridC), C.c_int32, C.POINTER(C.c_size_t)]),
    "reconstruct_bp": (C.c_int, [_P, C.POINTER(ImageGridC), C.c_int32, C.c_int32, _P, _P, _P,
                                 C.c_size_t, _P]),
    "make_hybrid_batch": (C.c_int, [C.c_int32, _P, C.POINTER(ImageGridC), C.POINTER(HybridOpts), C.POINTER(_P)]),
    "destroy_hybrid_batch": (C.c_int, [_P]),
    "hybrid_batch_info": (C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "reconstruct_hybrid_batch": (C.c_int, [_P, _P, _P, _P, C.c_size_t, _P]),
    "hybrid_batch_prepare": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "reconstruct_hybrid_batch_prepared": (C.c_int, [_P, _P, _P, _P, C.c_size_t, _P]),
    "last_error": (C.c_char_p, []),
}
EXPORTED = tuple(_SIGNATURES)

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2109_02842_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().last_error().decode()


def _check(code: int) -> None:
    if code != PL_OK:
        raise PolyreconError(code, last_error())


# ------------------------------------------------------------------ geometry
class Geometry:
    """Owning wrapper of a ``pl_geometry*`` handle."""

    def __init__(self, desc):
        self.desc = desc
        d = GeometryDesc()
        d.mode = PL_MONO if desc.mode == "mono" else PL_MULTI if desc.mode == "multi" else -1
        d.n_chords = desc.n_chords
        d.radius_m = desc.radius
        d.arc_center_rad = getattr(desc, "arc_center", -math.pi / 2)
        d.n_elem = desc.n_elem
        d.n_tx = getattr(desc, "n_tx", 0) or 0
        d.spacing_m = desc.spacing
        offs = getattr(desc, "tx_offsets", None)
        self._offs = None
        if offs is not None:
            self._offs = (C.c_double * len(offs))(*offs)
            d.tx_offsets_m = C.cast(self._offs, C.POINTER(C.c_double))
        d.n_scan = desc.n_scan
        d.n_freq = desc.n_freq
        d.scan_step_m = desc.scan_step
        z0 = getattr(desc, "z0", None)
        d.scan_z0_m = z0 if z0 is not None else -(desc.n_scan - 1) * desc.scan_step / 2.0
        d.f_start_hz = desc.f_start
        d.f_stop_hz = desc.f_stop
        h = _P()
        _check(lib().make_geometry(C.byref(d), C.byref(h)))
        self.handle = h
        if _torch().cuda.is_available():
            # the device tables on the current device, stream-ordered: later
            # calls then allocate nothing (graph capture, timing)
            _check(lib().geometry_upload(h, _stream()))
        info = GeometryInfo()
        _check(lib().geometry_info(h, C.byref(info), None, None, None, None, None))
        self.mode = "mono" if info.mode == PL_MONO else "multi"
        self.n_chords, self.n_channels = info.n_chords, info.n_channels
        self.n_scan, self.n_freq = info.n_scan, info.n_freq

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().destroy_geometry(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def echo_shape(self):
        return (self.n_channels, self.n_scan, self.n_freq)

    def info(self) -> dict:
        """Channel phase centres, scan heights, frequencies, chord ends (numpy)."""
        import numpy as np
        tx = np.zeros((self.n_channels, 2))
        rx = np.zeros((self.n_channels, 2))
        z = np.zeros(self.n_scan)
        f = np.zeros(self.n_freq)
        ends = np.zeros((self.n_chords, 2, 2))
        _check(lib().geometry_info(self.handle, None, tx.ctypes.data, rx.ctypes.data, z.ctypes.data,
                                   f.ctypes.data, ends.ctypes.data))
        return {"tx": tx, "rx": rx, "z_scan": z, "freq": f, "chord_ends": ends}


def make_geometry(desc) -> Geometry:
    return Geometry(desc)


def geometry_info(geom: Geometry) -> dict:
    return geom.info()


def _grid(grid) -> ImageGridC:
    return ImageGridC(int(grid.nx), int(grid.ny), float(grid.x0), float(grid.y0), float(grid.dx),
                      float(grid.dy))


def _opts(precision="fp32", interp="bspline4", l_oversample=6.0, nufft_tol=1e-6, tile=0, kz_per_lane=0,
          waves=0, mfma_backprojection=0, tile_y=0, kz_block=0, range_method="nufft",
          ref_mode="band-centre") -> HybridOpts:
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {list(PRECISIONS)}")
    if interp not in INTERPS:
        raise ValueError(f"interp must be one of {list(INTERPS)}")
    if range_method not in RANGE_METHODS:
        raise ValueError(f"range_method must be one of {list(RANGE_METHODS)}")
    if ref_mode not in REF_MODES:
        raise ValueError(f"ref_mode must be one of {list(REF_MODES)}")
    return HybridOpts(PRECISIONS[precision], INTERPS[interp], float(l_oversample), float(nufft_tol),
                      int(tile), int(kz_per_lane), int(waves), int(mfma_backprojection), int(tile_y),
                      int(kz_block), RANGE_METHODS[range_method], REF_MODES[ref_mode])


def check_sampling(geom: Geometry, grid) -> int:
    w = C.c_uint32()
    _check(lib().check_sampling(geom.handle, C.byref(_grid(grid)), C.byref(w)))
    return w.value


@dataclass
class PlanInfo:
    n_kz: int
    n_l: int
    n_fine: int
    kernel_width: int
    n_blocks: int
    block: int
    window: int
    tile: tuple
    du: float
    beta: float
    workspace_bytes: int
    k_ref: list
    bp_kernel: str = "kz-lanes"
    waves: int = 4
    range_method: str = "nufft"
    dk_uniform: float = 0.0         # resampling method: step of the uniform k_L grid (rad/m)
    scan_fft_len: int = 0           # length the scan / k_z transforms run through (chirp-z if > n_kz)

    @property
    def mfma_backprojection(self) -> bool:
        return self.bp_kernel in ("mfma", "mfma-1pass")


def hybrid_plan_info(geom: Geometry, grid, **opts) -> PlanInfo:
    info = HybridPlanInfo()
    _check(lib().hybrid_plan_info(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                  C.byref(info), None))
    kref = (C.c_double * max(1, info.n_blocks))()
    _check(lib().hybrid_plan_info(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                  C.byref(info), C.cast(kref, _P)))
    return PlanInfo(info.n_kz, info.n_l, info.n_fine, info.kernel_width, info.n_blocks, info.block,
                    info.window, (info.tile_x, info.tile_y), info.du, info.beta,
                    int(info.workspace_bytes), list(kref[: info.n_blocks]), BP_KERNELS[info.bp_kernel],
                    int(info.waves), {v: k for k, v in RANGE_METHODS.items()}[info.range_method],
                    float(info.dk_uniform), int(info.scan_fft_len))


def hybrid_workspace_bytes(geom: Geometry, grid, **opts) -> int:
    n = C.c_size_t()
    _check(lib().hybrid_workspace_bytes(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                        C.byref(n)))
    return int(n.value)


# ------------------------------------------------------- device-side helpers
def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_c64(t, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.complex64:
        raise TypeError(f"{name} must be complex64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def workspace(nbytes: int, device=None):
    """A 256-byte aligned device buffer of at least ``nbytes`` bytes."""
    torch = _torch()
    buf = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(int(nbytes), 1)]


def _ws(ws, need):
    if ws is None:
        ws = workspace(need)
    if ws.numel() < need:
        raise ValueError(f"workspace of {ws.numel()} bytes, {need} needed")
    return ws


# ------------------------------------------------------------- entry points
def simulate_echo(geom: Geometry, xyz, refl, out=None):
    """Echo cube s[c][m][f] (complex64, device) of point scatterers, eqs. (1)/(10).

    ``xyz``: (n, 3) float64 CUDA tensor; ``refl``: (n,) complex128 or (n, 2)
    float64 CUDA tensor.
    """
    torch = _torch()
    if refl.dtype == torch.complex128:
        refl = torch.view_as_real(refl)
    xyz = xyz.contiguous()
    refl = refl.contiguous()
    if xyz.dtype != torch.float64 or refl.dtype != torch.float64 or not xyz.is_cuda or not refl.is_cuda:
        raise TypeError("xyz and refl must be float64 CUDA tensors")
    n = xyz.shape[0]
    if tuple(xyz.shape) != (n, 3) or tuple(refl.shape) != (n, 2):
        raise ValueError("xyz must be (n, 3) and refl (n,) complex / (n, 2) real")
    if out is None:
        out = torch.empty(geom.echo_shape, dtype=torch.complex64, device=xyz.device)
    p = _dev_c64(out, geom.echo_shape, "out")
    _check(lib().simulate_echo(geom.handle, n, C.c_void_p(xyz.data_ptr()), C.c_void_p(refl.data_ptr()),
                               p, _stream()))
    return out


def reconstruct_hybrid(geom: Geometry, grid, echo, out=None, ws=None, prepared=False, **opts):
    """Image g[z][y][x] (complex64) by the hybrid method of Sec. II.

    prepared=True skips the plan tables: ``ws`` must hold them from
    ``hybrid_prepare`` with the same geometry, grid and options."""
    torch = _torch()
    need = hybrid_workspace_bytes(geom, grid, **opts)
    if prepared and ws is None:
        raise ValueError("prepared=True needs the workspace hybrid_prepare filled")
    ws = _ws(ws, need)
    shape = (geom.n_scan, grid.ny, grid.nx)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=echo.device)
    fn = lib().reconstruct_hybrid_prepared if prepared else lib().reconstruct_hybrid
    _check(fn(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
              _dev_c64(echo, geom.echo_shape, "echo"), _dev_c64(out, shape, "out"),
              C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


STATIC_SCRATCH_BYTES = 64 << 20


def reconstruct_hybrid_static(geom: Geometry, grid, echo, out=None, **opts):
    """reconstruct_hybrid on the library's static per-device scratch: no
    workspace and no device allocation inside the call (problems whose
    workspace fits STATIC_SCRATCH_BYTES; calls on one device must not
    overlap)."""
    torch = _torch()
    shape = (geom.n_scan, grid.ny, grid.nx)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=echo.device)
    _check(lib().reconstruct_hybrid_static(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                           _dev_c64(echo, geom.echo_shape, "echo"), _dev_c64(out, shape, "out"),
                                           _stream()))
    return out


def hybrid_prepare(geom: Geometry, grid, ws=None, **opts):
    """Write the plan's device tables into a workspace (returned) for
    reconstruct_hybrid(..., prepared=True)."""
    need = hybrid_workspace_bytes(geom, grid, **opts)
    ws = _ws(ws, need)
    _check(lib().hybrid_prepare(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return ws


# ------------------------------------------------------------------ batches
class HybridBatch:
    """Owning wrapper of a ``pl_hybrid_batch*``: several scans reconstructed by
    one call, their back-projections in one persistent launch.

    ``opts`` is one dict of options for every scan or a list of dicts."""

    def __init__(self, geoms, grids, opts=None):
        n = len(geoms)
        if len(grids) != n:
            raise ValueError("one grid per geometry")
        if opts is None or isinstance(opts, dict):
            opts = [dict(opts or {})] * n
        if len(opts) != n:
            raise ValueError("one options dict per geometry")
        self.geoms, self.grids, self.opts = list(geoms), list(grids), [dict(o) for o in opts]
        handles = (_P * n)(*[g.handle for g in geoms])
        cgrids = (ImageGridC * n)(*[_grid(g) for g in grids])
        copts = (HybridOpts * n)(*[_opts(**o) for o in opts])
        h = _P()
        _check(lib().make_hybrid_batch(n, C.cast(handles, _P), cgrids, copts, C.byref(h)))
        self.handle = h
        ws, queued, items, wgs = C.c_size_t(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().hybrid_batch_info(h, C.byref(ws), C.byref(queued), C.byref(items), C.byref(wgs)))
        self.workspace_bytes = int(ws.value)
        self.queued_scans, self.work_items, self.workgroups = queued.value, items.value, wgs.value

    @classmethod
    def autotuned(cls, geoms, grids, precision: str = "fp32", echoes=None, cache: Optional[str] = None,
                  repeats: int = 5, **fixed) -> "HybridBatch":
        """A batch whose scans take the launch shapes the autotuner finds
        fastest for each (timed per scan on the device, cached in ``cache``);
        ``fixed`` options (e.g. the interpolation) apply to every scan."""
        from .autotune import autotune_batch
        opts = autotune_batch(geoms, grids, precision, echoes=echoes, cache=cache, repeats=repeats, **fixed)
        return cls(geoms, grids, opts)

    def __len__(self):
        return len(self.geoms)

    def image_shape(self, i):
        return (self.geoms[i].n_scan, self.grids[i].ny, self.grids[i].nx)

    def close(self) -> None:
        if getattr(self, "handle", None):
            lib().destroy_hybrid_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hybrid_batch_prepare(batch: HybridBatch, ws):
    """Write every scan's plan tables into ``ws`` (for
    ``reconstruct_hybrid_batch(..., prepared=True)`` with the same ``ws``)."""
    ws = _ws(ws, batch.workspace_bytes)
    _check(lib().hybrid_batch_prepare(batch.handle, C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return ws


def reconstruct_hybrid_batch(batch: HybridBatch, echoes, outs=None, ws=None, prepared: bool = False):
    """Images of every scan of ``batch`` (list of complex64 device tensors).
    ``prepared``: ``ws`` holds the plan tables (hybrid_batch_prepare)."""
    torch = _torch()
    n = len(batch)
    if len(echoes) != n:
        raise ValueError(f"{n} echoes expected")
    if prepared and ws is None:
        raise ValueError("a prepared call needs the prepared workspace")
    ws = _ws(ws, batch.workspace_bytes)
    if outs is None:
        outs = [torch.empty(batch.image_shape(i), dtype=torch.complex64, device=echoes[i].device) for i in range(n)]
    e_ptrs = (_P * n)(*[_dev_c64(echoes[i], batch.geoms[i].echo_shape, f"echo {i}") for i in range(n)])
    o_ptrs = (_P * n)(*[_dev_c64(outs[i], batch.image_shape(i), f"out {i}") for i in range(n)])
    fn = lib().reconstruct_hybrid_batch_prepared if prepared else lib().reconstruct_hybrid_batch
    _check(fn(batch.handle, C.cast(e_ptrs, _P), C.cast(o_ptrs, _P), C.c_void_p(ws.data_ptr()), ws.numel(),
              _stream()))
    return outs


class CapturedBatch:
    """A batch call captured once in a graph (torch.cuda.CUDAGraph) and
    replayed: the echo and image tensors and the workspace are fixed at
    capture; copy new echoes into ``echoes`` before ``replay()``.  The
    workspace is prepared once (plan tables) and the graph holds the
    prepared call, so a replay runs no table kernels."""

    def __init__(self, batch: HybridBatch, echoes):
        torch = _torch()
        self.batch = batch
        self.echoes = [e.clone() for e in echoes]
        self.ws = workspace(batch.workspace_bytes)
        self.outs = [torch.empty(batch.image_shape(i), dtype=torch.complex64, device="cuda")
                     for i in range(len(batch))]
        # the tables, then one eager call (kernel attributes set on first use)
        hybrid_batch_prepare(batch, self.ws)
        reconstruct_hybrid_batch(batch, self.echoes, self.outs, self.ws, prepared=True)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            reconstruct_hybrid_batch(batch, self.echoes, self.outs, self.ws, prepared=True)

    def replay(self):
        self.graph.replay()
        return self.outs


def adjoint_hybrid(geom: Geometry, grid, image, out=None, ws=None, **opts):
    """Echo-shaped s~[c][m][f] = H^H g: the adjoint of reconstruct_hybrid's
    linear map (FP32 pixel-per-lane plans)."""
    torch = _torch()
    need = hybrid_workspace_bytes(geom, grid, **opts)
    ws = _ws(ws, need)
    shape = (geom.n_scan, grid.ny, grid.nx)
    if out is None:
        out = torch.empty(geom.echo_shape, dtype=torch.complex64, device=image.device)
    _check(lib().adjoint_hybrid(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                _dev_c64(image, shape, "image"), _dev_c64(out, geom.echo_shape, "out"),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


STAGES = ("plan_tables", "scan_fft", "range_compress", "backproject", "kz_ifft")


def reconstruct_hybrid_events(geom: Geometry, grid, echo, events, out=None, ws=None, **opts):
    """reconstruct_hybrid that records six torch.cuda.Events (created with
    enable_timing=True and recorded once beforehand) around its five stages."""
    torch = _torch()
    need = hybrid_workspace_bytes(geom, grid, **opts)
    ws = _ws(ws, need)
    shape = (geom.n_scan, grid.ny, grid.nx)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=echo.device)
    if len(events) != 6:
        raise ValueError("six events are needed")
    arr = (C.c_void_p * 6)(*[e.cuda_event for e in events])
    _check(lib().reconstruct_hybrid_events(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                           _dev_c64(echo, geom.echo_shape, "echo"),
                                           _dev_c64(out, shape, "out"), C.c_void_p(ws.data_ptr()),
                                           ws.numel(), C.cast(arr, _P), _stream()))
    return out


def fft_workspace_bytes(geom: Geometry) -> int:
    n = C.c_size_t()
    _check(lib().fft_workspace_bytes(geom.handle, C.byref(n)))
    return int(n.value)


def scan_fft(geom: Geometry, echo, out=None, ws=None):
    """Spectrum S[c][kz][f] = FFT over the scan axis, eq. (2)/(12)."""
    torch = _torch()
    if out is None:
        out = torch.empty(geom.echo_shape, dtype=torch.complex64, device=echo.device)
    ws = _ws(ws, fft_workspace_bytes(geom))
    _check(lib().scan_fft(geom.handle, _dev_c64(echo, geom.echo_shape, "echo"),
                          _dev_c64(out, geom.echo_shape, "out"), C.c_void_p(ws.data_ptr()), ws.numel(),
                          _stream()))
    return out


def _stage_opts(opts: dict) -> dict:
    """Options of a single-stage call: complex64 profiles, so the plan never
    takes the matrix-core back-projection."""
    if opts.get("mfma_backprojection", 0) > 0:
        raise ValueError("the MFMA back-projection runs only inside reconstruct_hybrid")
    return dict(opts, mfma_backprojection=-1)


def range_compress(geom: Geometry, grid, spec, out=None, ws=None, **opts):
    """Range profiles q[c][kz][n_l] and the range-grid origins l_lo[c] (numpy).
    The plan is that of hybrid_plan_info(..., mfma_backprojection=-1)."""
    import numpy as np
    torch = _torch()
    opts = _stage_opts(opts)
    pi = hybrid_plan_info(geom, grid, **opts)
    ws = _ws(ws, pi.workspace_bytes)
    shape = (geom.n_channels, geom.n_scan, pi.n_l)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=spec.device)
    llo = np.zeros(geom.n_channels)
    _check(lib().range_compress(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                                _dev_c64(spec, geom.echo_shape, "spec"), _dev_c64(out, shape, "out"),
                                llo.ctypes.data, C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out, llo


def backproject(geom: Geometry, grid, q, out=None, ws=None, **opts):
    """Spectrum G[p][kz] (p = iy*nx + ix) from range profiles, eq. (8b)/(19b).
    The plan is that of hybrid_plan_info(..., mfma_backprojection=-1)."""
    torch = _torch()
    opts = _stage_opts(opts)
    pi = hybrid_plan_info(geom, grid, **opts)
    ws = _ws(ws, pi.workspace_bytes)
    shape = (grid.ny * grid.nx, geom.n_scan)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=q.device)
    _check(lib().backproject(geom.handle, C.byref(_grid(grid)), C.byref(_opts(**opts)),
                             _dev_c64(q, (geom.n_channels, geom.n_scan, pi.n_l), "q"),
                             _dev_c64(out, shape, "out"), C.c_void_p(ws.data_ptr()), ws.numel(),
                             _stream()))
    return out


def kz_ifft(geom: Geometry, grid, spectrum, out=None, ws=None):
    """Image g[z][y][x] = inverse FFT over k_z (1/n), eq. (9)."""
    torch = _torch()
    shape = (geom.n_scan, grid.ny, grid.nx)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=spectrum.device)
    ws = _ws(ws, fft_workspace_bytes(geom))
    _check(lib().kz_ifft(geom.handle, C.byref(_grid(grid)),
                         _dev_c64(spectrum, (grid.ny * grid.nx, geom.n_scan), "spectrum"),
                         _dev_c64(out, shape, "out"), C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


def bp_workspace_bytes(geom: Geometry, grid, nz: Optional[int] = None) -> int:
    n = C.c_size_t()
    nz = geom.n_scan if nz is None else nz
    _check(lib().bp_workspace_bytes(geom.handle, C.byref(_grid(grid)), int(nz), C.byref(n)))
    return int(n.value)


def reconstruct_bp(geom: Geometry, grid, echo, iz0: int = 0, nz: Optional[int] = None, out=None, ws=None):
    """Brute-force back-projection image [nz][ny][nx] for scan planes [iz0, iz0+nz)."""
    torch = _torch()
    nz = geom.n_scan - iz0 if nz is None else nz
    ws = _ws(ws, bp_workspace_bytes(geom, grid, nz))
    shape = (nz, grid.ny, grid.nx)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=echo.device)
    _check(lib().reconstruct_bp(geom.handle, C.byref(_grid(grid)), int(iz0), int(nz),
                                _dev_c64(echo, geom.echo_shape, "echo"), _dev_c64(out, shape, "out"),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out
