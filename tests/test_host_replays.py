"""Host replays of the kernels' index arithmetic (CPU only).

Each test recomputes, in float64 from the plan the library reports, the
indices a kernel derives on the device, and checks that every access stays
inside the buffer the kernel stages or owns:

* matrix-core back-projection: a 4x4 pixel group's taps lie in its 16-sample
  window (start aligned to 4 samples, clamped to the staged row) and the
  staged row holds every tap of the tile, with slack for the float32 range
  offsets the kernel forms (positions perturbed by 1e-3 samples);
* adjoint back-projection: the tiles a (channel, range segment) workgroup
  lists include every pixel whose taps reach the segment;
* NUFFT spreading: the fine-grid cells a (channel, k_z) pair fills lie within
  one period of the grid on either side and number at most one period;
* matrix-core back-projection tail split: the pieces of a split work item
  cover its channels exactly once in runs that start at multiples of four,
  and the split fills at most the resident workgroups and the workspace.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import geometry as ogeom

pr = pytest.importorskip("paper_2109_02842_amd")

DELTA = 1e-3   # samples: far above the float32 error of the kernels' range positions


def _multi_small():
    arr = W.ArrayDesc(mode="multi", n_chords=3, radius=0.5, n_elem=16, spacing=W._D_MULTI, n_tx=4,
                      n_scan=24, scan_step=0.005, n_freq=16, f_start=26e9, f_stop=34e9)
    return W.Workload(name="multi-small", array=arr, grid=W.ImageGrid.centred(32, 0.30),
                      scene=W.Scene(n=4, kind="box", half=(0.12, 0.12, 0.04), seed=21, min_sep=0.06))


def _fine(wl, nx, ny, d):
    return replace(wl, grid=W.ImageGrid(nx=nx, ny=ny, x0=-d * (nx - 1) / 2 + 0.004, y0=-d * (ny - 1) / 2 - 0.003,
                                        dx=d, dy=d))


def _channels(g):
    gi = pr.geometry_info(g)
    return np.asarray(gi["tx"]).reshape(-1, 2), np.asarray(gi["rx"]).reshape(-1, 2)


def _range_origin(p, grid, du):
    """l_lo of a channel: its lowest range over the pixel-centre rectangle minus two samples."""
    X1 = grid.x0 + (grid.nx - 1) * grid.dx
    Y1 = grid.y0 + (grid.ny - 1) * grid.dy

    def to_rect(q):
        return math.hypot(q[0] - min(max(q[0], grid.x0), X1), q[1] - min(max(q[1], grid.y0), Y1))
    return to_rect(p[0]) + to_rect(p[1]) - 2 * du


# ---------------------------------------------------- matrix-core windows
@pytest.mark.parametrize("case,opts", [
    ("C2", dict(precision="fp16", mfma_backprojection=2)),
    ("C2", dict(precision="bf16", mfma_backprojection=1)),
    ("C2", dict(precision="fp16", mfma_backprojection=2, tile=16, tile_y=8, kz_block=128, waves=8)),
    ("C3", dict(precision="fp16", mfma_backprojection=2)),
    ("C1-fine", dict(precision="fp16", mfma_backprojection=2, tile=8, tile_y=8)),
    ("multi-fine", dict(precision="bf16", mfma_backprojection=1, tile=16, tile_y=8)),
])
def test_mfma_group_windows_hold_every_tap(case, opts):
    wl = {"C2": W.C2, "C3": W.C3, "C1-fine": _fine(W.C1, 45, 37, 0.0015),
          "multi-fine": _fine(_multi_small(), 61, 45, 0.0015)}[case]
    g = pr.make_geometry(wl.array)
    plan = pr.hybrid_plan_info(g, wl.grid, **opts)
    assert plan.mfma_backprojection
    TX, TY = plan.tile
    gr, du, n_l, wpl = wl.grid, plan.du, plan.n_l, plan.window
    tiles_x, tiles_y = -(-gr.nx // TX), -(-gr.ny // TY)
    NX, NY = tiles_x * TX, tiles_y * TY
    X = gr.x0 + np.arange(NX) * gr.dx
    Y = gr.y0 + np.arange(NY) * gr.dy
    valid = (np.arange(NY)[:, None] < gr.ny) & (np.arange(NX)[None, :] < gr.nx)
    cx = gr.x0 + (np.arange(tiles_x) * TX + 0.5 * (TX - 1)) * gr.dx
    cy = gr.y0 + (np.arange(tiles_y) * TY + 0.5 * (TY - 1)) * gr.dy
    reach = math.hypot((TX - 1) * gr.dx, (TY - 1) * gr.dy)
    tx, rx = _channels(g)
    worst_span, worst_row = 0, -1
    for c in range(tx.shape[0]):
        def rng(px, py):
            return (np.hypot(px[None, :] - tx[c, 0], py[:, None] - tx[c, 1]) +
                    np.hypot(px[None, :] - rx[c, 0], py[:, None] - rx[c, 1]))
        llo = _range_origin((tx[c], rx[c]), gr, du)
        s = np.floor((rng(cx, cy) - reach - llo) / du).astype(np.int64) - 2
        s = np.clip(s, 0, n_l - wpl) & ~1
        s_pix = np.repeat(np.repeat(s, TY, axis=0), TX, axis=1)
        u = (rng(X, Y) - llo) / du
        lo = np.floor(u - DELTA).astype(np.int64) - 1 - s_pix     # first taps, rounding down
        hi = np.floor(u + DELTA).astype(np.int64) - 1 - s_pix     # first taps, rounding up
        lo = np.where(valid, lo, 1 << 40)
        hi = np.where(valid, hi, -(1 << 40))
        # groups of 4x4 pixels
        glo = lo.reshape(NY // 4, 4, NX // 4, 4).min(axis=(1, 3))
        ghi = hi.reshape(NY // 4, 4, NX // 4, 4).max(axis=(1, 3))
        gval = valid.reshape(NY // 4, 4, NX // 4, 4).any(axis=(1, 3))
        sr = np.clip(glo & ~3, 0, wpl - 16)
        assert (glo[gval] >= 0).all(), (c, "a first tap before the staged window")
        span = (ghi - sr)[gval]          # last first-tap from the group window start
        worst_span = max(worst_span, int(span.max()))
        worst_row = max(worst_row, int(ghi[gval].max()))
    assert worst_span + 3 <= 15, (case, worst_span)          # four taps inside the 16-sample window
    assert worst_row + 3 <= wpl - 1, (case, worst_row, wpl)  # and inside the staged row


# ---------------------------------------------------- adjoint tile lists
@pytest.mark.parametrize("case,kz_block", [("C1", 32), ("multi-small", 32), ("C2", 32), ("C2", 64)])
def test_adjoint_segment_lists_cover_every_tap(case, kz_block):
    wl = {"C1": W.C1, "multi-small": _multi_small(), "C2": W.C2}[case]
    g = pr.make_geometry(wl.array)
    plan = pr.hybrid_plan_info(g, wl.grid, kz_block=kz_block)
    if plan.bp_kernel != "pixel-lanes":
        pytest.skip("the adjoint runs on pixel-per-lane plans")
    gr, du, n_l = wl.grid, plan.du, plan.n_l
    S = 32                               # range samples per adjoint workgroup
    n_seg = -(-n_l // S)
    tiles_x, tiles_y = -(-gr.nx // 8), -(-gr.ny // 8)
    X = gr.x0 + np.arange(gr.nx) * gr.dx
    Y = gr.y0 + np.arange(gr.ny) * gr.dy
    tx, rx = _channels(g)
    xa = gr.x0 + np.arange(tiles_x) * 8 * gr.dx
    xb = gr.x0 + np.minimum(np.arange(tiles_x) * 8 + 7, gr.nx - 1) * gr.dx
    ya = gr.y0 + np.arange(tiles_y) * 8 * gr.dy
    yb = gr.y0 + np.minimum(np.arange(tiles_y) * 8 + 7, gr.ny - 1) * gr.dy
    for c in range(tx.shape[0]):
        def dist_rect(p):
            dx = np.maximum(np.maximum(xa - p[0], p[0] - xb), 0)[None, :]
            dy = np.maximum(np.maximum(ya - p[1], p[1] - yb), 0)[:, None]
            return np.hypot(dx, dy)
        llo = _range_origin((tx[c], rx[c]), gr, du)
        lmin = dist_rect(tx[c]) + dist_rect(rx[c])
        lmax = np.zeros_like(lmin)
        for xs in (xa, xb):
            for ys in (ya, yb):
                lmax = np.maximum(lmax, np.hypot(xs[None, :] - tx[c, 0], ys[:, None] - tx[c, 1]) +
                                  np.hypot(xs[None, :] - rx[c, 0], ys[:, None] - rx[c, 1]))
        umin, umax = (lmin - llo) / du, (lmax - llo) / du
        u = (np.hypot(X[None, :] - tx[c, 0], Y[:, None] - tx[c, 1]) +
             np.hypot(X[None, :] - rx[c, 0], Y[:, None] - rx[c, 1]) - llo) / du
        f = np.floor(u).astype(np.int64)
        assert (f - 1 >= 0).all() and (f + 2 <= n_l - 1).all(), c      # taps on the range grid
        ti = (np.arange(gr.ny) // 8)[:, None] * np.ones(gr.nx, dtype=np.int64)[None, :]
        tj = np.ones(gr.ny, dtype=np.int64)[:, None] * (np.arange(gr.nx) // 8)[None, :]
        for seg in (0, 1):   # the (at most two) segments a pixel's four taps reach
            k = (f - 1) // S + seg
            reach = ((f - 1) <= k * S + S - 1) & ((f + 2) >= k * S) & (k < n_seg)
            s0 = k * S
            listed = (umax[ti, tj] >= s0 - 3.0) & (umin[ti, tj] <= s0 + S + 1.0)
            assert (listed | ~reach).all(), (c, seg)


# ---------------------------------------------------- NUFFT cell wrap
@pytest.mark.parametrize("case,opts", [("C1", {}), ("C2", {}), ("C3", {}), ("C5", {}), ("C2", dict(ref_mode="min-k")),
                                       ("C3", dict(ref_mode="min-k")), ("evanescent", {}),
                                       ("evanescent", dict(ref_mode="min-k"))])
def test_nufft_cells_stay_within_one_period(case, opts):
    ev = W.ArrayDesc(mode="multi", n_chords=2, radius=0.4, n_elem=6, spacing=W._D_MULTI, n_tx=2,
                     n_scan=30, scan_step=0.002, n_freq=12, f_start=26e9, f_stop=34e9)
    if case == "C5":
        wls = W.batch_c5()
    elif case == "evanescent":
        wls = [W.Workload(name="ev", array=ev, grid=W.ImageGrid.centred(20, 0.16), scene=W.C1.scene)]
    else:
        wls = [getattr(W, case)]
    for wl in wls:
        a = wl.array
        g = pr.make_geometry(a)
        plan = pr.hybrid_plan_info(g, wl.grid, **opts)
        N, h = plan.n_fine, 0.5 * plan.kernel_width
        kz = 2 * np.pi * np.fft.fftfreq(a.n_scan, a.scan_step) if a.n_scan > 1 else np.zeros(1)
        k = ogeom.build(a).k
        arg = k[None, :] ** 2 - kz[:, None] ** 2 / 4
        prop = arg > 0
        kr = np.sqrt(np.where(prop, arg, 0))
        if opts.get("ref_mode") == "min-k":
            first = np.where(prop.any(axis=1), prop.argmax(axis=1), 0)
            kref = np.where(prop.any(axis=1), kr[np.arange(a.n_scan), first], 0.0)
        else:
            kref = np.asarray(plan.k_ref)[np.arange(a.n_scan) // plan.block]
        py = (kr - kref[:, None]) * plan.du * N / (2 * np.pi)
        for kap in range(a.n_scan):
            p = py[kap][prop[kap]]
            if p.size == 0:
                continue
            assert (np.diff(p) > 0).all()                 # sorted: the binary search's premise
            klo = math.floor(p[0] - h) + 1
            khi = math.floor(p[-1] + h)
            assert -N <= klo and khi < 2 * N, (wl.name, kap, klo, khi, N)
            assert khi - klo + 1 <= N, (wl.name, kap)        # no cell is filled twice


# ------------------------------------------- matrix-core tail split pieces
def _tail_split(n_work, slots, n_ch, cap_pieces):
    """The launcher's choice: (whole items, pieces per tail item)."""
    n_ch4 = (n_ch + 3) // 4
    tail = n_work % slots
    if tail > 0 and 2 * tail <= slots:
        k = min(slots // tail, n_ch4, cap_pieces // tail)
        if k >= 2:
            return n_work - tail, k
    return n_work, 1


def _piece_channels(part, k, n_ch):
    n_ch4 = (n_ch + 3) // 4
    return 4 * (part * n_ch4 // k), min(n_ch, 4 * ((part + 1) * n_ch4 // k))


@pytest.mark.parametrize("n_work,slots,n_ch", [(676, 512, 320), (256, 512, 320), (768, 512, 896), (2048, 512, 896),
                                                (8, 512, 48), (3, 512, 5), (1300, 512, 320), (5, 1024, 7)])
def test_tail_split_pieces_cover_channels_once(n_work, slots, n_ch):
    cap = min(1024, n_work * ((n_ch + 3) // 4))      # pieces the workspace holds
    n_whole, k = _tail_split(n_work, slots, n_ch, cap)
    tail = n_work - n_whole
    if k > 1:
        assert n_whole % slots == 0 and 0 < tail < slots    # whole rounds, then the split tail
        assert tail * k <= slots and tail * k <= cap    # one round, within the workspace
        assert 2 * tail <= slots
    else:
        assert n_whole == n_work
    for part in range(k):
        cb, ce = _piece_channels(part, k, n_ch)
        assert cb % 4 == 0 and cb < ce <= n_ch
    covered = [c for part in range(k) for c in range(*_piece_channels(part, k, n_ch))]
    assert covered == list(range(n_ch))
    # the tail's workgroups: XCD b % 8 takes a contiguous share of the pieces
    n_pieces = tail * k if k > 1 else 0
    per_xcd_tail = (n_pieces + 7) // 8
    pieces = [(b & 7) * per_xcd_tail + (b >> 3) for b in range(8 * per_xcd_tail)]
    assert sorted(q for q in pieces if q < n_pieces) == list(range(n_pieces))
