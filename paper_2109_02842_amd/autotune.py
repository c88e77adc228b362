"""Autotuner for the hybrid reconstruction's launch shapes.

For one (geometry, image grid, precision) it times every back-projection
configuration the planner accepts -- the pixel-per-lane kernel with 32 or 64
k_z bins per workgroup, the k_z-per-lane kernel with 4 or 8 wavefronts, and in
the BF16 / FP16 modes the matrix-core kernel on 16x16, 16x8 and 8x8 tiles
with 64 or 128 k_z bins and 4 or 8 wavefronts -- on the device with hipEvents
around whole reconstructions, and returns the fastest.  Results are kept in
a JSON cache keyed by the problem's shape and the device name, so a shape is
tuned once per device.

Every candidate computes the same image to the method's tolerance (the
options only change launch shapes and, through the k_z block size, the
range-grid step), so the choice is a pure speed decision.  The single-pass
FP16 matrix-core form (``mfma_backprojection=2``) is a precision choice, not
a launch shape: asked for, it is tuned over its own tilings only.
"""
from __future__ import annotations

import json
import os
import statistics
from typing import Dict, List, Optional, Tuple

from . import (PolyreconError, Geometry, hybrid_plan_info, reconstruct_hybrid, workspace, _torch)

VALU_CANDIDATES = (
    {},                                  # pixel per lane, 32 k_z bins
    {"kz_block": 64},                    # pixel per lane, 64 k_z bins
    {"kz_per_lane": 1},                  # k_z per lane, 4 wavefronts
    {"kz_per_lane": 1, "waves": 8},      # k_z per lane, 8 wavefronts
)
MFMA_CANDIDATES = tuple(
    {"mfma_backprojection": 1, "tile": tx, "tile_y": ty, "kz_block": kb, "waves": nw}
    for tx, ty, kb, nw in ((16, 16, 64, 8), (16, 16, 64, 4), (16, 8, 64, 8), (16, 8, 128, 8), (16, 16, 128, 4),
                           (8, 8, 64, 4), (8, 8, 128, 4)))


def candidates(geom: Geometry, grid, precision: str = "fp32", **fixed) -> List[dict]:
    """Option sets the planner accepts for this problem (``fixed`` options,
    e.g. the interpolation, are added to each)."""
    if fixed.get("mfma_backprojection") == 2:
        pool = tuple(dict(c, mfma_backprojection=2) for c in MFMA_CANDIDATES)
    else:
        pool = VALU_CANDIDATES + (MFMA_CANDIDATES if precision != "fp32" else ())
    out, seen = [], set()
    for c in pool:
        opts = dict(fixed, precision=precision, **c)
        try:
            plan = hybrid_plan_info(geom, grid, **opts)
        except PolyreconError:
            continue
        key = (plan.bp_kernel, plan.tile, plan.block, plan.waves)
        if key in seen:        # the planner mapped two requests to one shape
            continue
        seen.add(key)
        out.append(opts)
    return out


def signature(geom: Geometry, grid, precision: str, fixed: dict) -> str:
    d = geom.desc
    parts = [d.mode, d.n_chords, round(d.radius, 9), d.n_elem, round(d.spacing, 9), getattr(d, "n_tx", 0),
             d.n_scan, round(d.scan_step, 9), d.n_freq, round(d.f_start), round(d.f_stop), grid.nx, grid.ny,
             round(grid.dx, 9), round(grid.dy, 9), precision, sorted(fixed.items())]
    return json.dumps(parts)


def _device_name() -> str:
    torch = _torch()
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def _load(path: Optional[str]) -> dict:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path: Optional[str], cache: dict) -> None:
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_opts(geom: Geometry, grid, echo, opts: dict, repeats: int = 5, warmup: int = 2) -> float:
    """Median device time (ms) of reconstruct_hybrid with these options."""
    torch = _torch()
    plan = hybrid_plan_info(geom, grid, **opts)
    ws = workspace(plan.workspace_bytes)
    out = torch.empty((geom.n_scan, grid.ny, grid.nx), dtype=torch.complex64, device="cuda")
    for _ in range(warmup):
        reconstruct_hybrid(geom, grid, echo, out=out, ws=ws, **opts)
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        reconstruct_hybrid(geom, grid, echo, out=out, ws=ws, **opts)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(statistics.median(times))


def autotune(geom: Geometry, grid, precision: str = "fp32", echo=None, cache: Optional[str] = None,
             repeats: int = 5, **fixed) -> Tuple[dict, Dict[str, float]]:
    """Fastest options for this problem and the timing table (ms per
    reconstruction, keyed by the options as JSON).  ``echo``: a device echo
    cube to time with (zeros if None; the kernels' work does not depend on
    the data).  ``cache``: JSON file read and updated (None: no cache)."""
    torch = _torch()
    key = signature(geom, grid, precision, fixed) + "|" + _device_name()
    store = _load(cache)
    if key in store:
        hit = store[key]
        return dict(hit["best"]), dict(hit["times"])
    if echo is None:
        echo = torch.zeros(geom.echo_shape, dtype=torch.complex64, device="cuda")
    times: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for opts in candidates(geom, grid, precision, **fixed):
        ms = time_opts(geom, grid, echo, opts, repeats=repeats)
        times[json.dumps(opts, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = opts, ms
    if best is None:
        raise PolyreconError(-1, "no back-projection configuration fits this problem")
    store = _load(cache)          # another process may have added entries meanwhile
    store[key] = {"best": best, "times": times}
    _store(cache, store)
    return dict(best), times


def autotune_batch(geoms, grids, precision: str = "fp32", echoes=None, cache: Optional[str] = None,
                   repeats: int = 5, **fixed) -> List[dict]:
    """Per-scan options for a batch: each scan tuned on its own.  Scans whose
    best options share the pixel-per-lane kernel and k_z block size run in
    the batch's persistent back-projection launch together."""
    out = []
    for i, (g, grid) in enumerate(zip(geoms, grids)):
        best, _ = autotune(g, grid, precision, echo=None if echoes is None else echoes[i], cache=cache,
                           repeats=repeats, **fixed)
        out.append(best)
    return out
