"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/polyrecon.h declares, builds the same array geometry as
the oracle, plans the hybrid method sensibly and rejects bad arguments."""
import math
import os
import re
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import geometry as ogeom

pr = pytest.importorskip("paper_2109_02842_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

if not os.path.exists(pr.LIB_PATH):
    pytest.skip("libpolyrecon.so not built", allow_module_level=True)


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "polyrecon.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    decl = _declared_functions()
    assert len(decl) >= 15
    lib = pr.lib()
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(pr.EXPORTED)


@pytest.mark.parametrize("wl", [W.C1, W.C2, W.C3], ids=["C1", "C2", "C3"])
def test_geometry_matches_oracle(wl):
    g = pr.make_geometry(wl.array)
    info = g.info()
    arr = ogeom.build(wl.array)
    assert g.n_channels == arr.n_channels
    assert np.allclose(info["tx"], arr.tx, rtol=0, atol=1e-12)
    assert np.allclose(info["rx"], arr.rx, rtol=0, atol=1e-12)
    assert np.allclose(info["z_scan"], arr.z_scan, rtol=0, atol=1e-12)
    assert np.array_equal(info["freq"], arr.freq)
    assert np.allclose(info["chord_ends"], arr.chord_ends, rtol=0, atol=1e-12)


def test_geometry_errors():
    a = W.C1.array
    with pytest.raises(pr.PolyreconError) as e:
        pr.make_geometry(replace(a, n_elem=400))          # chord longer than the diameter
    assert e.value.code == pr.PL_EGEOM
    for bad in (dict(n_chords=0), dict(spacing=-1.0), dict(f_stop=20e9), dict(n_scan=0),
                dict(n_freq=5000), dict(mode="bistatic")):
        with pytest.raises(pr.PolyreconError) as e:
            pr.make_geometry(replace(a, **bad))
        assert e.value.code == pr.PL_EINVAL
    with pytest.raises(pr.PolyreconError):
        pr.make_geometry(replace(W.C3.array, n_tx=3))       # no default placement for 3 Tx
    g = pr.make_geometry(replace(W.C3.array, n_tx=3, tx_offsets=(-0.1, 0.0, 0.1)))
    assert g.n_channels == 7 * 3 * 32
    # null pointers through the raw ABI
    assert pr.lib().make_geometry(None, None) == pr.PL_EINVAL
    assert "null" in pr.last_error()
    assert pr.lib().destroy_geometry(None) == pr.PL_OK


@pytest.mark.parametrize("wl", [W.C1, W.C2, W.C3], ids=["C1", "C2", "C3"])
def test_plan_is_consistent(wl):
    g = pr.make_geometry(wl.array)
    p = pr.hybrid_plan_info(g, wl.grid)
    assert p.n_kz == wl.array.n_scan
    # FP32 NUFFT fine grid: at least 1.25 n_l points, 2,3,5-smooth, kernel
    # width from the error estimate exp(-pi W sqrt(1 - 1/s)) <= 1e-6
    ups = p.n_fine / p.n_l
    assert ups >= 1.25 and p.n_l % 4 == 0 and _smooth(p.n_fine)
    assert p.kernel_width == math.ceil(math.log(1e6) / (math.pi * math.sqrt(1 - 1 / ups)))
    assert math.isclose(p.beta, 0.97 * math.pi * p.kernel_width * (1 - 0.5 / ups), rel_tol=1e-12)
    assert p.block % 32 == 0
    assert p.n_blocks == math.ceil(wl.array.n_scan / p.block)
    # the range grid covers every channel's range span at the requested step
    arr = ogeom.build(wl.array)
    x = wl.grid.x0 + wl.grid.dx * np.array([0, wl.grid.nx - 1])
    y = wl.grid.y0 + wl.grid.dy * np.array([0, wl.grid.ny - 1])
    xx, yy = np.meshgrid(np.linspace(x[0], x[1], 41), np.linspace(y[0], y[1], 41))
    l = (np.hypot(xx.ravel()[None] - arr.tx[:, :1], yy.ravel()[None] - arr.tx[:, 1:]) +
         np.hypot(xx.ravel()[None] - arr.rx[:, :1], yy.ravel()[None] - arr.rx[:, 1:]))
    assert (l.max(1) - l.min(1)).max() + 4 * p.du < p.n_l * p.du
    # reference wavenumbers lie inside the propagating band k_rho in (0, k_max]
    kmax = 2 * math.pi * wl.array.f_stop / W.SPEED_OF_LIGHT
    assert all(0 < k <= kmax for k in p.k_ref)
    # step: l_oversample samples per Nyquist interval of the widest block band
    kz = 2 * np.pi * np.fft.fftfreq(wl.array.n_scan, wl.array.scan_step)
    kf = 2 * np.pi * np.linspace(wl.array.f_start, wl.array.f_stop, wl.array.n_freq) / W.SPEED_OF_LIGHT
    half = 0.0
    for b in range(p.n_blocks):
        kk = kz[b * p.block:(b + 1) * p.block]
        kr = np.sqrt(np.maximum(kf[None] ** 2 - kk[:, None] ** 2 / 4, 0))
        kr = kr[kr > 0]
        half = max(half, (kr.max() - kr.min()) / 2)
    assert math.isclose(p.du, math.pi / (6 * half), rel_tol=1e-12)   # default l_oversample 6
    assert pr.hybrid_workspace_bytes(g, wl.grid) == p.workspace_bytes
    assert p.workspace_bytes >= 8 * (arr.n_channels * wl.array.n_scan * (wl.array.n_freq + p.n_l))


def test_plan_errors():
    g = pr.make_geometry(W.C1.array)
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, replace(W.C1.grid, nx=0))
    assert e.value.code == pr.PL_EINVAL
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, W.C1.grid, l_oversample=1.0)
    assert e.value.code == pr.PL_EINVAL
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, W.C1.grid, nufft_tol=0.5)
    assert e.value.code == pr.PL_EINVAL
    with pytest.raises(ValueError):
        pr.hybrid_plan_info(g, W.C1.grid, precision="fp64")


def _stages(m):
    """Radix stages of a 2,3,5-smooth length: factors of 8, then 4, 2, 3, 5."""
    count = 0
    for r in (8, 4, 2, 3, 5):
        while m % r == 0:
            m //= r
            count += 1
    return count


def _smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("n_scan", [7, 37, 131, 226, 389, 509, 1000, 1100, 2304, 2310, 4096, 4093])
def test_plan_blocks_and_transform_length_at_any_scan_length(n_scan):
    # Every k_z block gets its band-centre reference wavenumber, also past
    # 64 blocks (scans longer than 2048 with 32-bin blocks), and the scan
    # transform runs through n_scan itself when it is 2,3,5-smooth, else
    # through a smooth chirp-z length >= 2 n_scan - 1.
    a = replace(W.C1.array, n_scan=n_scan)
    g = pr.make_geometry(a)
    for opts in ({}, dict(kz_per_lane=1)):
        p = pr.hybrid_plan_info(g, W.C1.grid, **opts)
        assert p.n_blocks == -(-n_scan // p.block) and len(p.k_ref) == p.n_blocks
        kz = 2 * np.pi * np.fft.fftfreq(n_scan, a.scan_step)
        kf = 2 * np.pi * np.linspace(a.f_start, a.f_stop, a.n_freq) / W.SPEED_OF_LIGHT
        for b in range(p.n_blocks):
            kr2 = kf[None] ** 2 - kz[b * p.block:(b + 1) * p.block, None] ** 2 / 4
            kr = np.sqrt(kr2[kr2 > 0])
            want = 0.5 * (kr.min() + kr.max()) if kr.size else 0.0
            assert math.isclose(p.k_ref[b], want, rel_tol=1e-12, abs_tol=1e-9)
        # smooth lengths run as they are; any other through a chirp-z length
        # m >= 2n - 1: from n = 64 on the smallest m = 64 R with R smooth and
        # at most 32 (the wavefront kernel), else the m up to twice the
        # smallest with the fewest length x stages
        lo = 2 * n_scan - 1
        wave = [64 * r for r in range(2, 33) if _smooth(r) and 64 * r >= lo] if n_scan >= 64 else []
        if _smooth(n_scan):
            want_len = n_scan
        elif wave:
            want_len = wave[0]
        else:
            want_len = min((m for m in range(lo, 2 * lo + 1) if _smooth(m)), key=lambda m: (m * _stages(m), m))
        assert p.scan_fft_len == want_len
    assert pr.fft_workspace_bytes(g) >= 8 * want_len * (1 if _smooth(n_scan) else 3)
    assert _smooth(want_len) and want_len >= (n_scan if _smooth(n_scan) else 2 * n_scan - 1)


def test_reference_mode_plans():
    # PL_REF_MIN_K: the paper's per-k_z reference k_rho0 = k_rho(k_0): every
    # k' lies in [0, max k_rho - k_rho0], so the range step follows the
    # widest such band at the requested oversampling, on the k_z-per-lane
    # kernel; options it cannot run are refused
    for wl in (W.C1, W.C2, W.C3):
        a = wl.array
        g = pr.make_geometry(a)
        p = pr.hybrid_plan_info(g, wl.grid, ref_mode="min-k")
        assert p.bp_kernel == "kz-lanes" and p.block == 64
        kz = 2 * np.pi * np.fft.fftfreq(a.n_scan, a.scan_step)
        kf = 2 * np.pi * np.linspace(a.f_start, a.f_stop, a.n_freq) / W.SPEED_OF_LIGHT
        kr2 = kf[None] ** 2 - kz[:, None] ** 2 / 4
        band = max(np.sqrt(r[r > 0]).max() - np.sqrt(r[r > 0]).min() for r in kr2 if (r > 0).any())
        assert math.isclose(p.du, math.pi / (6 * band), rel_tol=1e-12)
    g = pr.make_geometry(W.C1.array)
    for bad in (dict(range_method="resample"), dict(precision="bf16", mfma_backprojection=1),
                dict(kz_per_lane=2), dict(kz_block=32), dict(waves=8)):
        with pytest.raises(pr.PolyreconError) as e:
            pr.hybrid_plan_info(g, W.C1.grid, ref_mode="min-k", **bad)
        assert e.value.code == pr.PL_EUNSUPPORTED, bad
    with pytest.raises(ValueError):
        pr.hybrid_plan_info(g, W.C1.grid, ref_mode="centre")


def test_sampling_criteria():
    # C1's half-wavelength transceivers satisfy eq. (21)/2; doubling the
    # spacing or the scan step beyond eq. (22) raises the warnings.
    g = pr.make_geometry(W.C1.array)
    assert pr.check_sampling(g, W.C1.grid) == 0
    g2 = pr.make_geometry(replace(W.C1.array, spacing=3 * W.C1.array.spacing))
    assert pr.check_sampling(g2, W.C1.grid) & pr.WARN_ELEMENT_SPACING
    g3 = pr.make_geometry(replace(W.C1.array, scan_step=0.05))
    assert pr.check_sampling(g3, W.C1.grid) & pr.WARN_SCAN_STEP


def test_raw_abi_argument_errors_before_device_use():
    # These paths return before any device access, so dummy pointers suffice.
    import ctypes as C
    L = pr.lib()
    g = pr.make_geometry(W.C1.array)
    grid = C.byref(pr._grid(W.C1.grid))
    opts = C.byref(pr._opts())
    fake = C.c_void_p(1 << 20)
    need = pr.hybrid_workspace_bytes(g, W.C1.grid)
    assert L.reconstruct_hybrid(g.handle, grid, opts, None, fake, fake, need, None) == pr.PL_EINVAL
    assert L.reconstruct_hybrid(g.handle, grid, opts, fake, fake, None, need, None) == pr.PL_EWORKSPACE
    assert L.reconstruct_hybrid(g.handle, grid, opts, fake, fake, fake, need - 1, None) == pr.PL_EWORKSPACE
    assert "needed" in pr.last_error()
    assert L.reconstruct_hybrid(g.handle, grid, opts, fake, fake, C.c_void_p((1 << 20) + 8), need,
                                None) == pr.PL_EWORKSPACE
    assert "aligned" in pr.last_error()
    bad_opts = pr.HybridOpts(7, 0, 8.0, 1e-6)
    assert L.reconstruct_hybrid(g.handle, grid, C.byref(bad_opts), fake, fake, fake, need, None) == pr.PL_EINVAL
    assert L.reconstruct_bp(g.handle, grid, 0, 0, fake, fake, fake, 1 << 30, None) == pr.PL_EINVAL
    assert L.reconstruct_bp(g.handle, grid, 20, 10, fake, fake, fake, 1 << 30, None) == pr.PL_EINVAL
    assert L.reconstruct_bp(g.handle, grid, 0, 1, fake, fake, fake, 16, None) == pr.PL_EWORKSPACE
    bneed = pr.bp_workspace_bytes(g, W.C1.grid, 2)
    assert bneed >= 8 * W.C1.array.n_channels * W.C1.array.n_scan * W.C1.array.n_freq
    assert L.reconstruct_bp(g.handle, grid, 0, 2, fake, fake, fake, bneed - 1, None) == pr.PL_EWORKSPACE
    assert L.reconstruct_bp(g.handle, grid, 0, 2, fake, fake, C.c_void_p((1 << 20) + 8), bneed, None) == pr.PL_EWORKSPACE
    assert L.simulate_echo(g.handle, -1, fake, fake, fake, None) == pr.PL_EINVAL
    assert L.simulate_echo(g.handle, 3, None, fake, fake, None) == pr.PL_EINVAL
    assert L.scan_fft(None, fake, fake, fake, 1 << 20, None) == pr.PL_EINVAL
    fneed = pr.fft_workspace_bytes(g)
    assert L.scan_fft(g.handle, fake, fake, None, fneed, None) == pr.PL_EWORKSPACE
    assert L.scan_fft(g.handle, fake, fake, fake, fneed - 1, None) == pr.PL_EWORKSPACE
    assert L.kz_ifft(g.handle, grid, fake, fake, C.c_void_p((1 << 20) + 8), fneed, None) == pr.PL_EWORKSPACE


def _fine_grid(nx, ny, d):
    return W.ImageGrid(nx=nx, ny=ny, x0=-d * (nx - 1) / 2 + 0.004, y0=-d * (ny - 1) / 2 - 0.003, dx=d, dy=d)


def test_mfma_backprojection_plan_rules():
    g = pr.make_geometry(W.C1.array)
    fine = _fine_grid(40, 40, 0.0015)
    p = pr.hybrid_plan_info(g, fine, precision="bf16", mfma_backprojection=1)
    assert p.mfma_backprojection and p.tile == (16, 16) and p.block == 64 and p.window % 8 == 0
    # every 4x4 group's taps fit a 16-sample window that starts on a multiple
    # of 4: up to 3 samples of alignment, 2 x group diagonal / du, 4 taps
    assert 3 + math.ceil(2 * math.hypot(3 * fine.dx, 3 * fine.dy) / p.du) + 3 <= 15
    for tile, tile_y, kb in [(8, 8, 64), (16, 8, 128), (16, 16, 128)]:
        q = pr.hybrid_plan_info(g, fine, precision="bf16", mfma_backprojection=1, tile=tile, tile_y=tile_y,
                                kz_block=kb)
        assert q.tile == (tile, tile_y) and q.block == kb
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, fine, precision="bf16", mfma_backprojection=1, tile=8, tile_y=16)
    assert e.value.code == pr.PL_EINVAL
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, fine, precision="bf16", tile=16)          # 16 is a matrix-core tile
    assert e.value.code == pr.PL_EINVAL
    with pytest.raises(pr.PolyreconError):
        pr.hybrid_plan_info(g, fine, precision="bf16", mfma_backprojection=1, kz_block=96)
    assert not pr.hybrid_plan_info(g, fine, precision="fp32").mfma_backprojection
    q = pr.hybrid_plan_info(g, fine, precision="bf16", mfma_backprojection=-1)
    assert not q.mfma_backprojection and q.bp_kernel == "pixel-lanes"
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, fine, precision="fp32", mfma_backprojection=1)
    assert e.value.code == pr.PL_EUNSUPPORTED
    with pytest.raises(pr.PolyreconError):
        pr.hybrid_plan_info(g, W.C1.grid, precision="bf16", mfma_backprojection=1)   # pixels too coarse
    assert not pr.hybrid_plan_info(g, fine, precision="bf16").mfma_backprojection   # opt-in
    # the full-size workloads allow it in the BF16 / FP16 modes
    for wl in (W.C2, W.C3):
        assert pr.hybrid_plan_info(pr.make_geometry(wl.array), wl.grid, precision="fp16",
                                   mfma_backprojection=1).mfma_backprojection
    # the single-stage calls exchange complex64 profiles
    with pytest.raises(ValueError):
        pr.range_compress(g, fine, None, precision="bf16", mfma_backprojection=1)
    import ctypes as C
    fake = C.c_void_p(1 << 20)
    opts = pr._opts(precision="bf16", mfma_backprojection=1)
    assert pr.lib().range_compress(g.handle, C.byref(pr._grid(fine)), C.byref(opts), fake, fake, None, fake,
                                   1 << 40, None) == pr.PL_EUNSUPPORTED
    assert "reconstruct_hybrid" in pr.last_error()


def test_mfma_single_pass_plan_rules():
    g = pr.make_geometry(W.C1.array)
    fine = _fine_grid(40, 40, 0.0015)
    p = pr.hybrid_plan_info(g, fine, precision="fp16", mfma_backprojection=2)
    assert p.bp_kernel == "mfma-1pass" and p.mfma_backprojection and p.tile == (16, 16)
    split = pr.hybrid_plan_info(g, fine, precision="fp16", mfma_backprojection=1)
    assert split.bp_kernel == "mfma" and split.window == p.window and split.n_l == p.n_l
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, fine, precision="bf16", mfma_backprojection=2)   # FP16 operands only
    assert e.value.code == pr.PL_EUNSUPPORTED
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, fine, precision="fp32", mfma_backprojection=2)
    assert e.value.code == pr.PL_EUNSUPPORTED
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, fine, precision="fp16", mfma_backprojection=3)
    assert e.value.code == pr.PL_EINVAL
    assert pr.hybrid_plan_info(pr.make_geometry(W.C2.array), W.C2.grid, precision="fp16",
                               mfma_backprojection=2).bp_kernel == "mfma-1pass"


def test_valu_backprojection_plan_rules():
    g = pr.make_geometry(W.C2.array)
    p = pr.hybrid_plan_info(g, W.C2.grid)
    assert p.bp_kernel == "pixel-lanes" and p.tile == (8, 8) and p.block == 32 and p.waves == 4
    assert pr.hybrid_plan_info(g, W.C2.grid, kz_block=64).block == 64
    assert p.window % 2 == 0 and p.window <= 64
    assert pr.hybrid_plan_info(g, W.C2.grid, waves=8).bp_kernel == "kz-lanes"
    assert pr.hybrid_plan_info(g, W.C2.grid, kz_per_lane=1).bp_kernel == "kz-lanes"
    assert pr.hybrid_plan_info(g, W.C2.grid, tile=4).bp_kernel == "kz-lanes"
    # pixels too coarse for 64 staged samples: the k_z-per-lane kernel on smaller tiles
    p1 = pr.hybrid_plan_info(pr.make_geometry(W.C1.array), W.ImageGrid.centred(16, 0.30))
    assert p1.bp_kernel == "kz-lanes" and p1.tile == (4, 4)


def _gather_window_margins(wl):
    """Tap margins of the pixel-per-lane back-projection's staged window.

    Replays, in float64, where the planner and the tile table put a tile's
    window (start s: the tile centre's range minus its reach, two samples
    lower, clamped to the range grid, even; length: the plan's window) and
    returns the smallest distance of any pixel's range position u (in
    samples from s) to the two limits that keep its reads inside the
    window: u >= 1 (first tap floor(u) - 1 >= 0) and u < window - 3 (first
    tap at most window - 5; the four-sample reads need window - 4).
    The range grid starts at each channel's lowest range over the pixel
    rectangle minus two samples.
    """
    g = pr.make_geometry(wl.array)
    info = pr.hybrid_plan_info(g, wl.grid)
    assert info.bp_kernel == "pixel-lanes"
    gi = pr.geometry_info(g)
    tx, rx = np.asarray(gi["tx"]).reshape(-1, 2), np.asarray(gi["rx"]).reshape(-1, 2)
    gr = wl.grid
    du, n_l, wpl = info.du, info.n_l, info.window
    reach = math.hypot(7 * gr.dx, 7 * gr.dy)
    X = gr.x0 + np.arange(gr.nx) * gr.dx
    Y = gr.y0 + np.arange(gr.ny) * gr.dy
    tiles_x, tiles_y = (gr.nx + 7) // 8, (gr.ny + 7) // 8
    cx = gr.x0 + (np.arange(tiles_x) * 8 + 3.5) * gr.dx
    cy = gr.y0 + (np.arange(tiles_y) * 8 + 3.5) * gr.dy
    lo, hi = np.inf, np.inf
    for c in range(tx.shape[0]):
        def rng(px, py):
            return (np.hypot(px[None, :] - tx[c, 0], py[:, None] - tx[c, 1]) +
                    np.hypot(px[None, :] - rx[c, 0], py[:, None] - rx[c, 1]))
        def to_rect(p):
            return math.hypot(p[0] - min(max(p[0], X[0]), X[-1]), p[1] - min(max(p[1], Y[0]), Y[-1]))
        llo = to_rect(tx[c]) + to_rect(rx[c]) - 2 * du
        s = np.floor((rng(cx, cy) - reach - llo) / du).astype(np.int64) - 2
        s = np.clip(s, 0, n_l - wpl) & ~1
        s_pix = np.repeat(np.repeat(s, 8, axis=0), 8, axis=1)[: gr.ny, : gr.nx]
        u = (rng(X, Y) - llo) / du - s_pix
        lo = min(lo, float((u - 1).min()))
        hi = min(hi, float(((wpl - 3) - u).min()))
    return lo, hi


@pytest.mark.parametrize("which", ["C1", "C2", "C3", "C5"])
def test_gather_window_holds_every_tap(which):
    """Every pixel's taps (and the aligned read past them) lie inside the
    staged window with room to spare for float32 rounding of the range."""
    wls = W.batch_c5() if which == "C5" else [getattr(W, which)]
    for wl in wls:
        lo, hi = _gather_window_margins(wl)
        assert lo >= 0.5 and hi >= 0.5, (wl.name, lo, hi)


def test_resample_range_method_plan_rules():
    g = pr.make_geometry(W.C2.array)
    base = pr.hybrid_plan_info(g, W.C2.grid)
    assert base.range_method == "nufft" and base.dk_uniform == 0.0
    p = pr.hybrid_plan_info(g, W.C2.grid, range_method="resample")
    assert p.range_method == "resample"
    # the inverse FFT of the uniform grid lands on the range grid
    assert p.dk_uniform == pytest.approx(2 * math.pi / (p.n_fine * p.du), rel=1e-12)
    # same range step and back-projection as the NUFFT plan; its range grid
    # is rounded up to a 2,3,5-smooth fine grid of 2 n_l points
    assert (p.du, p.bp_kernel, p.block) == (base.du, base.bp_kernel, base.block)
    assert p.n_l >= base.n_l and p.n_fine == 2 * p.n_l and _smooth(p.n_fine)
    # reference wavenumbers moved onto the grid (by at most half a step)
    for kr, kb in zip(p.k_ref, base.k_ref):
        assert abs(kr / p.dk_uniform - round(kr / p.dk_uniform)) < 1e-9
        assert abs(kr - kb) <= 0.5 * p.dk_uniform + 1e-9
    # a block's propagating band fits the transform: at most n_fine / 8 + 1 grid points
    k = ogeom.build(W.C2.array).k
    assert (k[-1] - k[0]) / p.dk_uniform + 1 <= p.n_fine
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(g, W.C2.grid, range_method="resample", precision="bf16")
    assert e.value.code == pr.PL_EUNSUPPORTED
    with pytest.raises(pr.PolyreconError) as e:
        pr.hybrid_plan_info(pr.make_geometry(replace(W.C1.array, n_freq=1)), W.C1.grid, range_method="resample")
    assert e.value.code == pr.PL_EUNSUPPORTED
    with pytest.raises(ValueError):
        pr.hybrid_plan_info(g, W.C2.grid, range_method="stolt")


def test_batch_argument_errors_before_device_use():
    import ctypes as C
    L = pr.lib()
    h = C.c_void_p()
    assert L.make_hybrid_batch(0, None, None, None, C.byref(h)) == pr.PL_EINVAL
    assert L.make_hybrid_batch(2, None, None, None, C.byref(h)) == pr.PL_EINVAL
    assert L.make_hybrid_batch(1, None, None, None, None) == pr.PL_EINVAL
    assert L.hybrid_batch_info(None, None, None, None, None) == pr.PL_EINVAL
    assert L.reconstruct_hybrid_batch(None, None, None, None, 0, None) == pr.PL_EINVAL
    assert L.destroy_hybrid_batch(None) == pr.PL_OK


def test_batch_c5_workload():
    wls = W.batch_c5()
    assert len(wls) == 16 and len({w.name for w in wls}) == 16
    for w in wls:
        a = w.array
        assert 3 <= a.n_chords <= 7 and 32 <= a.n_elem <= 64 and 32 <= a.n_freq <= 128
        assert 128 <= a.n_scan <= 512 and pr.hybrid_plan_info(pr.make_geometry(a), w.grid).bp_kernel == "pixel-lanes"
    assert W.batch_c5()[3] == wls[3]           # seeded


def test_autotune_candidates_and_cache(tmp_path):
    from paper_2109_02842_amd import autotune as at
    g = pr.make_geometry(W.C2.array)
    c32 = at.candidates(g, W.C2.grid, "fp32")
    kernels = {(pr.hybrid_plan_info(g, W.C2.grid, **o).bp_kernel, pr.hybrid_plan_info(g, W.C2.grid, **o).block)
               for o in c32}
    assert ("pixel-lanes", 32) in kernels and ("pixel-lanes", 64) in kernels and ("kz-lanes", 64) in kernels
    assert not any(o.get("mfma_backprojection") for o in c32)
    cb = at.candidates(g, W.C2.grid, "bf16")
    assert any(o.get("mfma_backprojection") for o in cb) and len(cb) > len(c32)
    # the single-pass form, once asked for, is tuned over its own tilings
    c1p = at.candidates(g, W.C2.grid, "fp16", mfma_backprojection=2)
    assert c1p and all(pr.hybrid_plan_info(g, W.C2.grid, **o).bp_kernel == "mfma-1pass" for o in c1p)
    assert len({(o["tile"], o["tile_y"], o["kz_block"], o["waves"]) for o in c1p}) == len(c1p)
    # coarse pixels: every request maps to the k_z-per-lane kernel, listed once per shape
    g1, coarse = pr.make_geometry(W.C1.array), W.ImageGrid.centred(16, 0.30)
    c1 = at.candidates(g1, coarse, "fp32")
    shapes = [(p.bp_kernel, p.tile, p.block, p.waves) for p in (pr.hybrid_plan_info(g1, coarse, **o) for o in c1)]
    assert len(shapes) == len(set(shapes)) and all(s[0] == "kz-lanes" for s in shapes)
    # a cached entry is returned without timing anything
    cache = str(tmp_path / "tune.json")
    key = at.signature(g, W.C2.grid, "fp32", {}) + "|" + at._device_name()
    at._store(cache, {key: {"best": {"precision": "fp32", "kz_block": 64}, "times": {"x": 1.0}}})
    best, times = at.autotune(g, W.C2.grid, "fp32", cache=cache)
    assert best == {"precision": "fp32", "kz_block": 64} and times == {"x": 1.0}
