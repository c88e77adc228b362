"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (relative L2 unless noted):
  * hybrid reconstruction, FP32:  1e-4 (the target stated for the FP32 path);
  * brute-force BP, FP32:          1e-4;
  * echo simulator:                1e-5 -- float64 path lengths and phase
    reduction, float32 sin/cos (|err| ~ 1e-7) and a 16-step phasor
    recurrence (~16 * 6e-8), summed over scatterers in float32;
  * FFT steps:                     2e-6 -- float32 butterflies over
    log2(N) <= 11 stages (~ 11 * 6e-8 rms growth, twiddles rounded from
    float64);
  * range compression vs the direct NUDFT: 2e-5 -- NUFFT tolerance 1e-6 plus
    float32 spreading, transform and deapodisation;
  * range compression on the matrix cores (BF16 / FP16, operands split into
    hi + lo, three products, FP32 accumulation): 5e-5 -- the dropped lo*lo
    term and the rounding of the lo parts are ~2^-16 (BF16) or ~2^-22 (FP16)
    of each product, accumulated over n_f terms in FP32;
  * hybrid reconstruction with the MFMA range compression: 1e-3 (the target
    stated for the BF16 path); the split operands keep it near the FP32 path.
  * the resampling range method (omega-K variant) against the oracle of the
    same method: 1e-4, the FP32 bar -- its FP32 Lagrange weights and phases
    add ~1e-6 to the FP32 path's error.
"""
import math
import os
import sys
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import bp as obp
from oracle import geometry as ogeom
from oracle import hybrid as ohyb
from oracle import nudft as onudft
from oracle import omegak as oomk
from oracle import simulate as osim

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2109_02842_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(pr.LIB_PATH):
        pytest.fail("libpolyrecon.so is not built")
    yield
    torch.cuda.synchronize()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def multi_small():
    arr = W.ArrayDesc(mode="multi", n_chords=3, radius=0.5, n_elem=16, spacing=W._D_MULTI, n_tx=4,
                      n_scan=24, scan_step=0.005, n_freq=16, f_start=26e9, f_stop=34e9)
    return W.Workload(name="multi-small", array=arr, grid=W.ImageGrid.centred(32, 0.30),
                      scene=W.Scene(n=4, kind="box", half=(0.12, 0.12, 0.04), seed=21, min_sep=0.06))


# ------------------------------------------------------------------ FFTs
@pytest.mark.parametrize("n_scan", [1, 7, 10, 24, 127, 128, 131, 192, 251, 256, 320, 384, 448, 509, 512, 2310, 4093])
def test_scan_fft_and_kz_ifft(n_scan):
    # 64 R points (R = 2, 3, 4, 5, 6, 8) take the wavefront FFT, other
    # 2,3,5-smooth lengths the Stockham stages, the rest (primes, 7 | n) the
    # chirp-z transform (4093: through 8192 points, one transform per
    # workgroup); 9 frequencies and 15 pixels leave partial workgroups and
    # transforms that straddle channels
    a = replace(W.tiny("mono").array, n_scan=n_scan, n_freq=9)
    g = pr.make_geometry(a)
    say("scan_fft", n_scan)
    s = W.random_echo(a, 3)
    spec = host(pr.scan_fft(g, dev(s)))
    ref = np.fft.fft(s.astype(np.complex128), axis=1)
    assert rel(spec, ref) < 2e-6
    grid = W.ImageGrid(nx=5, ny=3, x0=0, y0=0, dx=1e-3, dy=1e-3)
    G = W.complex_normal(np.random.default_rng(1), (15, n_scan)).astype(np.complex64)
    img = host(pr.kz_ifft(g, grid, dev(G)))
    ref = np.fft.ifft(G.astype(np.complex128), axis=1).T.reshape(n_scan, 3, 5)
    assert rel(img, ref) < 2e-6


# ------------------------------------------------------------- simulator
@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_simulate_echo_tiny_full(mode):
    wl = W.tiny(mode)
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    pos, refl = W.scatterers(wl.scene)
    say("simulate", mode)
    s = host(pr.simulate_echo(g, dev(pos), dev(refl)))
    ref = osim.echo(arr, pos, refl)
    assert rel(s, ref) < 1e-5
    # no scatterers: a zero echo
    z = host(pr.simulate_echo(g, dev(np.zeros((0, 3))), dev(np.zeros(0, complex))))
    assert not np.any(z)


def test_simulate_echo_c1_and_c2_samples():
    for wl in (W.C1, W.C2):
        g = pr.make_geometry(wl.array)
        arr = ogeom.build(wl.array)
        pos, refl = W.scatterers(wl.scene)
        say("simulate", wl.name)
        s = host(pr.simulate_echo(g, dev(pos), dev(refl)))
        if wl is W.C1:
            assert rel(s, osim.echo(arr, pos, refl)) < 1e-5
        else:
            rng = np.random.default_rng(5)
            n = 300
            ci, mi, fi = (rng.integers(0, s.shape[i], n) for i in range(3))
            ref = osim.echo_samples(arr, pos, refl, ci, mi, fi)
            assert rel(s[ci, mi, fi], ref) < 1e-5


# --------------------------------------------------------- hybrid steps
def _kprime(wl, plan, kap):
    """k' = sqrt(k^2 - k_z^2/4) - k_ref(block) (the library's range unit is
    rho_T + rho_R, for which the multistatic relation (18) holds in both modes)."""
    arr = ogeom.build(wl.array)
    kz = ohyb.kz_grid(arr.z_scan.size, arr.scan_step)[kap]
    krho, valid = ohyb.dispersion("multi", arr.k, kz)
    return krho - plan.k_ref[kap // plan.block], valid, arr


@pytest.mark.parametrize("interp", ["lagrange4", "bspline4"])
@pytest.mark.parametrize("wlname", ["tiny-mono", "multi-small", "C1", "evanescent-small"])
def test_range_compress_matches_direct_nudft(interp, wlname):
    # fine grids of 192 (tiny), 384 (C1) and 512 (evanescent) points take the
    # wavefront-per-pair kernel, 432 (multi-small) the workgroup kernel; the
    # evanescent case has rows with no and with 1-3 propagating frequencies
    wl = {"tiny-mono": W.tiny("mono"), "multi-small": multi_small(), "C1": W.C1,
          "evanescent-small": evanescent_small()}[wlname]
    g = pr.make_geometry(wl.array)
    plan = pr.hybrid_plan_info(g, wl.grid, interp=interp)
    s = W.random_echo(wl.array, 8)
    say("range_compress", wlname, interp, plan.n_l, plan.n_fine)
    spec = pr.scan_fft(g, dev(s))
    q, llo = pr.range_compress(g, wl.grid, spec, interp=interp)
    q = host(q)
    S = ohyb.scan_spectrum(s)
    kaps = {0, 1, wl.array.n_scan // 2, wl.array.n_scan - 1}
    if wlname == "evanescent-small":
        kaps = set(range(wl.array.n_scan))
    n_dead = 0
    for kap in sorted(kaps):
        kp, valid, arr = _kprime(wl, plan, kap)
        w = arr.k * valid
        if interp == "bspline4":
            x = 0.5 * kp * plan.du                 # B-spline prefilter 1/sinc^4, closed form
            w = w / np.where(valid, np.sinc(x / np.pi) ** 4, 1.0)
        for c in sorted({0, arr.n_channels // 2, arr.n_channels - 1}):
            if not valid.any():                    # nothing propagates: the row is zero
                n_dead += 1
                assert not np.any(q[c, kap]), (kap, c)
                continue
            l = llo[c] + plan.du * np.arange(plan.n_l)
            ref = onudft.nudft(w * S[c, kap], kp, l)
            assert rel(q[c, kap], ref) < 2e-5, (kap, c)
    if wlname == "evanescent-small":
        assert n_dead > 0


def _oversampling_for_fine_grid(g, grid, n_fine):
    """A range-grid oversampling whose plan has this fine-grid size."""
    for sig in np.arange(4.0, 60.0, 0.25):
        try:
            plan = pr.hybrid_plan_info(g, grid, l_oversample=float(sig))
        except RuntimeError:
            continue
        if plan.n_fine == n_fine:
            return float(sig), plan
    raise AssertionError(f"no oversampling gives a {n_fine}-point fine grid")


@pytest.mark.parametrize("n_fine", [64 * r for r in (3, 4, 5, 6, 9, 10, 16, 18, 20, 24, 25, 27, 30, 32)] + [2160])
def test_range_compress_every_wavefront_radix(n_fine):
    # C1 at the oversampling that makes the fine grid 64 R points: every
    # R-point register DFT the wavefront NUFFT is compiled for (2160 points
    # are past them: the workgroup kernel)
    wl = W.C1
    g = pr.make_geometry(wl.array)
    sig, plan = _oversampling_for_fine_grid(g, wl.grid, n_fine)
    radix = n_fine // 64
    say("range_compress radix", radix, "l_oversample", sig, "n_l", plan.n_l)
    s = W.random_echo(wl.array, 30 + radix)
    spec = pr.scan_fft(g, dev(s))
    q, llo = pr.range_compress(g, wl.grid, spec, l_oversample=sig)
    q = host(q)
    S = ohyb.scan_spectrum(s)
    for kap in (0, 7, wl.array.n_scan - 1):
        kp, valid, arr = _kprime(wl, plan, kap)
        x = 0.5 * kp * plan.du
        w = arr.k * valid / np.where(valid, np.sinc(x / np.pi) ** 4, 1.0)
        for c in (0, arr.n_channels - 1):
            l = llo[c] + plan.du * np.arange(plan.n_l)
            ref = onudft.nudft(w * S[c, kap], kp, l)
            assert rel(q[c, kap], ref) < 2e-5, (radix, kap, c)


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("wlname", ["tiny-mono", "multi-small", "C1", "C1-40f", "C1-100f"])
def test_mfma_range_compress_matches_direct_nudft(precision, wlname):
    # 40 and 100 frequencies pad to 48 and 112 (strength rows of 24 and 56
    # chunks: the 8-chunk swizzle), 16 and 64 to rows of 8 and 32 chunks;
    # the C1 range grid of these plans (n_l 192) leaves the last 128-row
    # block's third and fourth wavefronts without rows
    wl = {"tiny-mono": W.tiny("mono"), "multi-small": multi_small(), "C1": W.C1,
          "C1-40f": replace(W.C1, array=replace(W.C1.array, n_freq=40)),
          "C1-100f": replace(W.C1, array=replace(W.C1.array, n_freq=100))}[wlname]
    g = pr.make_geometry(wl.array)
    plan = pr.hybrid_plan_info(g, wl.grid, precision=precision, mfma_backprojection=-1)
    s = W.random_echo(wl.array, 9)
    say("mfma range_compress", wlname, precision)
    spec = pr.scan_fft(g, dev(s))
    q, llo = pr.range_compress(g, wl.grid, spec, precision=precision)
    q = host(q)
    S = ohyb.scan_spectrum(s)
    worst = 0.0
    for kap in sorted({0, 1, wl.array.n_scan // 2, wl.array.n_scan - 1}):
        kp, valid, arr = _kprime(wl, plan, kap)
        x = 0.5 * kp * plan.du
        w = arr.k * valid / np.where(valid, np.sinc(x / np.pi) ** 4, 1.0)
        for c in sorted({0, arr.n_channels // 2, arr.n_channels - 1}):
            l = llo[c] + plan.du * np.arange(plan.n_l)
            ref = onudft.nudft(w * S[c, kap], kp, l)
            worst = max(worst, rel(q[c, kap], ref))
    say("   worst rel L2", worst)
    assert worst < 5e-5


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("wlname", ["tiny-multi", "C1"])
def test_hybrid_mfma_end_to_end_small(precision, wlname):
    wl = {"tiny-multi": W.tiny("multi"), "C1": W.C1}[wlname]
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 17)
    img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), precision=precision))
    err = rel(img, ohyb.image(arr, wl.grid, s))
    say("hybrid", precision, wlname, "rel L2", err)
    assert err < 1e-3


def _fine_grid(nx, ny, d):
    """Off-centre ragged grid of d-spaced pixels (fine enough for the
    matrix-core back-projection's 16-sample pixel groups)."""
    return W.ImageGrid(nx=nx, ny=ny, x0=-d * (nx - 1) / 2 + 0.004, y0=-d * (ny - 1) / 2 - 0.003, dx=d, dy=d)


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("interp", ["bspline4", "lagrange4", "linear"])
@pytest.mark.parametrize("case", ["tiny-multi", "multi-small", "C1"])
def test_mfma_backprojection_matches_oracle(case, interp, precision):
    wl = {"tiny-multi": W.tiny("multi"), "multi-small": multi_small(), "C1": W.C1}[case]
    grid = {"tiny-multi": _fine_grid(21, 11, 0.0015), "multi-small": _fine_grid(27, 35, 0.0015),
            "C1": _fine_grid(44, 37, 0.0015)}[case]
    sigma = 16.0 if interp == "lagrange4" else 8.0
    g = pr.make_geometry(wl.array)
    plan = pr.hybrid_plan_info(g, grid, precision=precision, interp=interp, l_oversample=sigma,
                               mfma_backprojection=1)
    assert plan.mfma_backprojection and plan.tile == (16, 16) and plan.block == 64
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 41)
    say("mfma backprojection", case, interp, precision, "window", plan.window, "block", plan.block)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), precision=precision, interp=interp,
                                     l_oversample=sigma, mfma_backprojection=1))
    ref = ohyb.image(arr, grid, s)
    err = rel(img, ref)
    valu = host(pr.reconstruct_hybrid(g, grid, dev(s), precision=precision, interp=interp,
                                      l_oversample=sigma, mfma_backprojection=-1))
    err_valu = rel(valu, ref)
    say("   rel L2", err, "VALU back-projection", err_valu)
    # linear taps carry their own interpolation error; the matrix cores must
    # not add to it beyond the split-BF16 rounding
    assert err < (1e-3 if interp != "linear" else 1.2 * err_valu + 1e-3)


@pytest.mark.parametrize("tile,tile_y,kb,waves", [(8, 8, 64, 4), (8, 8, 128, 4), (16, 8, 64, 4), (16, 8, 128, 4),
                                                   (16, 16, 64, 4), (16, 16, 128, 4), (16, 8, 64, 8),
                                                   (16, 8, 128, 8), (16, 16, 64, 8)])
def test_mfma_backprojection_tilings(tile, tile_y, kb, waves):
    # every tiling of the workgroup gives the same image to the split-BF16 bar;
    # 300 k_z bins leave a ragged last k_z block, 61 x 45 pixels ragged tiles
    arr_desc = replace(W.C1.array, n_scan=300)
    grid = _fine_grid(61, 45, 0.0015)
    g = pr.make_geometry(arr_desc)
    arr = ogeom.build(arr_desc)
    s = W.random_echo(arr_desc, 43)
    say("mfma tiling", tile, tile_y, kb, waves)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), precision="bf16", mfma_backprojection=1, tile=tile,
                                     tile_y=tile_y, kz_block=kb, waves=waves))
    kap = sorted(set(W.random_subset(300, 6, 44).tolist() + [0, 63, 64, 127, 128, 299]))
    pix = np.unique(np.concatenate([W.random_subset(grid.nx * grid.ny, 200, 45), [0, grid.nx * grid.ny - 1]]))
    px, py = ohyb.pixel_grid(grid)
    ref = ohyb.spectrum_at(arr, ohyb.scan_spectrum(s), kap, px[pix], py[pix])
    err = rel(_spectrum_subset(img, kap, pix), ref)
    say("   rel L2", err)
    assert err < 1e-3


@pytest.mark.parametrize("interp", ["bspline4", "lagrange4", "linear"])
@pytest.mark.parametrize("case", ["tiny-multi", "multi-small", "C1"])
def test_mfma_single_pass_matches_oracle(case, interp):
    # one FP16 product per pair: two FP16 roundings (2^-11 relative) per
    # term, held to the reduced-precision bar of 1e-3 relative L2
    wl = {"tiny-multi": W.tiny("multi"), "multi-small": multi_small(), "C1": W.C1}[case]
    grid = {"tiny-multi": _fine_grid(21, 11, 0.0015), "multi-small": _fine_grid(27, 35, 0.0015),
            "C1": _fine_grid(44, 37, 0.0015)}[case]
    sigma = 16.0 if interp == "lagrange4" else 8.0
    g = pr.make_geometry(wl.array)
    kw = dict(precision="fp16", interp=interp, l_oversample=sigma)
    plan = pr.hybrid_plan_info(g, grid, mfma_backprojection=2, **kw)
    assert plan.bp_kernel == "mfma-1pass" and plan.tile == (16, 16) and plan.block == 64
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 51)
    say("mfma single pass", case, interp, "window", plan.window)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), mfma_backprojection=2, **kw))
    ref = ohyb.image(arr, grid, s)
    err = rel(img, ref)
    err_valu = rel(host(pr.reconstruct_hybrid(g, grid, dev(s), mfma_backprojection=-1, **kw)), ref)
    say("   rel L2", err, "VALU back-projection", err_valu)
    assert np.isfinite(img).all()
    assert err < (1e-3 if interp != "linear" else 1.2 * err_valu + 1e-3)


@pytest.mark.parametrize("tile,tile_y,kb,waves", [(8, 8, 64, 4), (8, 8, 128, 4), (16, 8, 64, 4), (16, 8, 128, 4),
                                                   (16, 16, 64, 4), (16, 16, 128, 4), (16, 8, 64, 8),
                                                   (16, 8, 128, 8), (16, 16, 64, 8)])
def test_mfma_single_pass_tilings(tile, tile_y, kb, waves):
    # ragged k_z blocks (300 bins) and ragged tiles (61 x 45 pixels)
    arr_desc = replace(W.C1.array, n_scan=300)
    grid = _fine_grid(61, 45, 0.0015)
    g = pr.make_geometry(arr_desc)
    arr = ogeom.build(arr_desc)
    s = W.random_echo(arr_desc, 53)
    say("mfma single-pass tiling", tile, tile_y, kb, waves)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), precision="fp16", mfma_backprojection=2, tile=tile,
                                     tile_y=tile_y, kz_block=kb, waves=waves))
    kap = sorted(set(W.random_subset(300, 6, 54).tolist() + [0, 63, 64, 127, 128, 299]))
    pix = np.unique(np.concatenate([W.random_subset(grid.nx * grid.ny, 200, 55), [0, grid.nx * grid.ny - 1]]))
    px, py = ohyb.pixel_grid(grid)
    ref = ohyb.spectrum_at(arr, ohyb.scan_spectrum(s), kap, px[pix], py[pix])
    err = rel(_spectrum_subset(img, kap, pix), ref)
    say("   rel L2", err)
    assert err < 1e-3


@pytest.mark.parametrize("precision,mbp", [("fp16", 2), ("bf16", 1)])
def test_mfma_tail_split_is_repeatable(precision, mbp):
    # 4 x 3 tiles x 5 k_z blocks = 60 work items, fewer than half the
    # resident workgroups: the launch splits every item over its channels
    # and adds the pieces' partial spectra in a fixed order, so two calls
    # give the same bits (and the result holds the oracle's bar)
    arr_desc = replace(W.C1.array, n_scan=300)
    grid = _fine_grid(61, 45, 0.0015)
    g = pr.make_geometry(arr_desc)
    s = W.random_echo(arr_desc, 57)
    say("mfma tail split repeatability", precision, mbp)
    a = pr.reconstruct_hybrid(g, grid, dev(s), precision=precision, mfma_backprojection=mbp)
    b = pr.reconstruct_hybrid(g, grid, dev(s), precision=precision, mfma_backprojection=mbp)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    kap = [0, 64, 150, 299]
    pix = np.unique(np.concatenate([W.random_subset(grid.nx * grid.ny, 120, 58), [0, grid.nx * grid.ny - 1]]))
    px, py = ohyb.pixel_grid(grid)
    ref = ohyb.spectrum_at(ogeom.build(arr_desc), ohyb.scan_spectrum(s), kap, px[pix], py[pix])
    err = rel(_spectrum_subset(host(a), kap, pix), ref)
    say("   rel L2", err)
    assert err < 1e-3


@pytest.mark.parametrize("scale", [1e-15, 1.0, 1e15])
def test_mfma_single_pass_follows_the_data_scale(scale):
    # the FP16 profiles' power-of-two scale comes from the data: echoes 15
    # decades apart reconstruct to the same relative error, and a zero echo
    # to an exactly zero image
    wl = W.C1
    grid = _fine_grid(44, 37, 0.0015)
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 57) * scale
    say("mfma single pass, echo scale", scale)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), precision="fp16", mfma_backprojection=2))
    err = rel(img, ohyb.image(arr, grid, s))
    say("   rel L2", err)
    assert np.isfinite(img).all() and err < 1e-3
    if scale == 1.0:
        zero = host(pr.reconstruct_hybrid(g, grid, dev(np.zeros_like(s)), precision="fp16", mfma_backprojection=2))
        assert not np.any(zero)


@pytest.mark.parametrize("wlname", ["tiny-mono", "tiny-multi", "multi-small", "C1"])
@pytest.mark.parametrize("interp", ["bspline4", "lagrange4"])
def test_hybrid_end_to_end_small(wlname, interp):
    wl = {"tiny-mono": W.tiny("mono"), "tiny-multi": W.tiny("multi"), "multi-small": multi_small(),
          "C1": W.C1}[wlname]
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 11)
    say("hybrid", wlname, interp)
    img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), interp=interp))
    ref = ohyb.image(arr, wl.grid, s)
    # Lagrange taps need twice the oversampling for the same error
    tol = 1e-4
    err = rel(img, ref)
    say("   rel L2", err)
    if interp == "lagrange4":
        assert err < 1e-3
        img2 = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), interp=interp, l_oversample=16))
        assert rel(img2, ref) < tol
    else:
        assert err < tol
    # the separate steps give the same image
    spec = pr.scan_fft(g, dev(s))
    q, _ = pr.range_compress(g, wl.grid, spec, interp=interp)
    G = pr.backproject(g, wl.grid, q, interp=interp)
    img3 = host(pr.kz_ifft(g, wl.grid, G))
    assert rel(img3, img) < 1e-6


@pytest.mark.parametrize("case", ["multi-small", "C1"])
@pytest.mark.parametrize("kernel", ["pixel-lanes", "pixel-lanes-32", "kz-lanes", "kz-lanes-8"])
def test_valu_backprojection_kernels(case, kernel):
    # both VALU back-projection layouts on ragged 8x8-tiled grids, FP32 bar
    wl = {"multi-small": multi_small(), "C1": W.C1}[case]
    grid = _fine_grid(45, 29, 0.003) if case == "C1" else _fine_grid(27, 35, 0.004)
    opts = {"pixel-lanes": dict(), "pixel-lanes-32": dict(kz_block=32), "kz-lanes": dict(kz_per_lane=1),
            "kz-lanes-8": dict(waves=8)}[kernel]
    g = pr.make_geometry(wl.array)
    plan = pr.hybrid_plan_info(g, grid, **opts)
    assert plan.bp_kernel == kernel.replace("-8", "").replace("-32", "")
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 47)
    say("valu back-projection", case, kernel, plan.tile, plan.window)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), **opts))
    err = rel(img, ohyb.image(arr, grid, s))
    say("   rel L2", err)
    assert err < 1e-4


@pytest.mark.parametrize("case,n_scan", [("C1", 131), ("C1", 37), ("multi-small", 53), ("tiny-mono", 1)])
def test_hybrid_scan_lengths_that_are_not_smooth(case, n_scan):
    # eqs. (2), (9) and (12) hold for any number of scan positions: prime
    # lengths, 7 | n and a single position, end to end against the oracle
    base = {"C1": W.C1, "multi-small": multi_small(), "tiny-mono": W.tiny("mono")}[case]
    wl = replace(base, array=replace(base.array, n_scan=n_scan))
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 17)
    plan = pr.hybrid_plan_info(g, wl.grid)
    say("scan length", case, n_scan, "transform length", plan.scan_fft_len)
    img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s)))
    err = rel(img, ohyb.image(arr, wl.grid, s))
    say("   rel L2", err)
    assert err < 1e-4


@pytest.mark.parametrize("case", ["C1", "multi-small", "evanescent-small", "tiny-mono-fine"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reference_wavenumber_modes_give_the_same_image(case, precision):
    # eqs. (8a)/(8b) and (19a)/(19b): the reference wavenumber cancels, so the
    # paper's k_rho0 = k_rho at the lowest k (per k_z bin) and the band-centre
    # reference per block both reach the exact sum within the FP32 bar; in
    # "evanescent-small" k_0 is evanescent in some bins (the smallest real
    # k_rho of the bin is the reference there)
    wl = {"C1": W.C1, "multi-small": multi_small(), "evanescent-small": evanescent_small(),
          "tiny-mono-fine": W.tiny("mono")}[case]
    grid = _fine_grid(37, 29, 0.004) if case == "tiny-mono-fine" else wl.grid
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 23)
    ref = ohyb.image(arr, grid, s)
    assert pr.hybrid_plan_info(g, grid, precision=precision, ref_mode="min-k").bp_kernel == "kz-lanes"
    errs = []
    for mode in ("band-centre", "min-k"):
        img = host(pr.reconstruct_hybrid(g, grid, dev(s), precision=precision, ref_mode=mode))
        errs.append(rel(img, ref))
    say("reference modes", case, precision, "band-centre %.2e, min-k %.2e" % tuple(errs))
    assert max(errs) < 1e-4


@pytest.mark.parametrize("nx,ny", [(1, 1), (9, 13), (17, 5), (64, 40)])
def test_hybrid_ragged_grids(nx, ny):
    wl = W.tiny("multi")
    grid = W.ImageGrid(nx=nx, ny=ny, x0=-0.07, y0=-0.05, dx=0.15 / max(nx, 2), dy=0.11 / max(ny, 2))
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 12)
    say("ragged", nx, ny)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s)))
    assert rel(img, ohyb.image(arr, grid, s)) < 1e-4


def test_hybrid_c1_point_targets():
    wl = W.C1
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    pos, refl = W.scatterers(wl.scene)
    s = osim.echo(arr, pos, refl)
    s = osim.add_noise(s, wl.noise_db, W.noise(s.shape, wl.scene.seed)).astype(np.complex64)
    img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s)))
    ref = ohyb.image(arr, wl.grid, s)
    assert rel(img, ref) < 1e-4
    a, b = np.abs(img), np.abs(ref)
    assert np.unravel_index(np.argmax(a), a.shape) == np.unravel_index(np.argmax(b), b.shape)


@pytest.mark.parametrize("opts", [{}, dict(precision="bf16", mfma_backprojection=1), dict(range_method="resample")],
                         ids=["fp32", "bf16-mfma-bp", "resample"])
def test_prepared_plan_matches_plain_call(opts):
    # the plan tables written once by hybrid_prepare serve later calls; the
    # result is bitwise that of the call that builds them itself
    wl = W.C2
    g = pr.make_geometry(wl.array)
    s = dev(W.random_echo(wl.array, 31))
    ws = pr.hybrid_prepare(g, wl.grid, **opts)
    a = host(pr.reconstruct_hybrid(g, wl.grid, s, ws=ws, prepared=True, **opts))
    b = host(pr.reconstruct_hybrid(g, wl.grid, s, ws=ws, prepared=True, **opts))   # tables survive a call
    c = host(pr.reconstruct_hybrid(g, wl.grid, s, **opts))
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
    assert np.array_equal(b.view(np.uint32), c.view(np.uint32))


def test_hybrid_is_deterministic():
    wl = W.C1
    g = pr.make_geometry(wl.array)
    s = dev(W.random_echo(wl.array, 13))
    a = host(pr.reconstruct_hybrid(g, wl.grid, s))
    b = host(pr.reconstruct_hybrid(g, wl.grid, s))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def _spectrum_subset(img, kappas, pix):
    G = np.fft.fft(img.astype(np.complex128).reshape(img.shape[0], -1), axis=0)
    return G[np.ix_(kappas, pix)]


@pytest.mark.parametrize("wl,precision,mfma_bp", [(W.C2, "fp32", 0), (W.C3, "fp32", 0), (W.C2, "bf16", 0),
                                                 (W.C2, "fp16", 0), (W.C3, "bf16", 0), (W.C2, "bf16", 1),
                                                 (W.C2, "fp16", 1), (W.C3, "bf16", 1), (W.C2, "fp16", 2),
                                                 (W.C3, "fp16", 2)],
                         ids=["C2-fp32", "C3-fp32", "C2-bf16", "C2-fp16", "C3-bf16", "C2-bf16-mfma-bp",
                              "C2-fp16-mfma-bp", "C3-bf16-mfma-bp", "C2-fp16-mfma-bp-1pass",
                              "C3-fp16-mfma-bp-1pass"])
def test_hybrid_full_size_sampled(wl, precision, mfma_bp):
    # The full workload in the launch configuration the benchmark times;
    # the oracle evaluates sampled (k_z, pixel) pairs of the spectrum.
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 21)
    say("full size", wl.name, precision, "mfma back-projection" if mfma_bp else "")
    img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), precision=precision, mfma_backprojection=mfma_bp))
    assert np.all(np.isfinite(img))
    npix = wl.grid.nx * wl.grid.ny
    kap = W.random_subset(wl.array.n_scan, 3, 31).tolist()
    kap = sorted(set(kap + [0, wl.array.n_scan // 2]))
    pix = W.random_subset(npix, 192 if wl is W.C3 else 384, 32)
    pix = np.unique(np.concatenate([pix, [0, npix - 1, wl.grid.nx - 1]]))
    px, py = ohyb.pixel_grid(wl.grid)
    ref = ohyb.spectrum_at(arr, ohyb.scan_spectrum(s), kap, px[pix], py[pix])
    got = _spectrum_subset(img, kap, pix)
    err = rel(got, ref)
    say("   rel L2", err)
    assert err < (1e-4 if precision == "fp32" else 1e-3)


# ---------------------------------------------------------------- BP
@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_bp_tiny(mode):
    wl = W.tiny(mode)
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 14)
    say("bp", mode)
    img = host(pr.reconstruct_bp(g, wl.grid, dev(s)))
    ref = obp.bp_image(arr, wl.grid, s)
    assert rel(img, ref) < 1e-4
    part = host(pr.reconstruct_bp(g, wl.grid, dev(s), iz0=3, nz=4))
    assert rel(part, ref[3:7]) < 1e-4


def test_bp_c2_plane_samples():
    wl = W.C2
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 15)
    iz = 100
    say("bp C2 plane", iz)
    img = host(pr.reconstruct_bp(g, wl.grid, dev(s), iz0=iz, nz=1))[0]
    pix = W.random_subset(wl.grid.nx * wl.grid.ny, 12, 16)
    px, py = ohyb.pixel_grid(wl.grid)
    ref = obp.bp_voxels(arr, s, px[pix], py[pix], np.full(pix.size, arr.z_scan[iz]))
    assert rel(img.ravel()[pix], ref) < 1e-4


# ---------------------------------------------------------- error paths
def test_binding_rejects_bad_tensors():
    wl = W.tiny("mono")
    g = pr.make_geometry(wl.array)
    s = dev(W.random_echo(wl.array, 1))
    need = pr.hybrid_workspace_bytes(g, wl.grid)
    with pytest.raises(ValueError):
        pr.reconstruct_hybrid(g, wl.grid, s, ws=pr.workspace(need - 512))
    with pytest.raises(TypeError):
        pr.reconstruct_hybrid(g, wl.grid, s.to(torch.complex128))
    with pytest.raises(ValueError):
        pr.reconstruct_hybrid(g, wl.grid, s[:, :5].contiguous())
    with pytest.raises(TypeError):
        pr.reconstruct_hybrid(g, wl.grid, s.cpu())


# ------------------------------------------------------------------ batches
def _small_batch():
    """Uneven scans: pixel-per-lane scans of different sizes, one whose pixels
    are too coarse for it (k_z-per-lane kernel), one BF16 scan on the matrix
    cores and one FP16 scan in their single-pass form; every kind of
    back-projection the batch call launches."""
    c1 = W.C1
    ms = multi_small()
    scans = [
        (c1.array, _fine_grid(45, 29, 0.003), {}),
        (replace(c1.array, n_scan=30, n_freq=20), _fine_grid(21, 40, 0.004), {}),
        (ms.array, _fine_grid(27, 35, 0.004), {}),
        (c1.array, W.ImageGrid.centred(16, 0.30), {}),                        # coarse: k_z per lane
        (replace(c1.array, n_scan=32), _fine_grid(40, 40, 0.0015), dict(precision="bf16", mfma_backprojection=1)),
        (replace(c1.array, n_scan=40), _fine_grid(36, 44, 0.0015), dict(precision="fp16", mfma_backprojection=2)),
    ]
    return scans


def test_batch_matches_single_scans():
    scans = _small_batch()
    geoms = [pr.make_geometry(a) for a, _, _ in scans]
    batch = pr.HybridBatch(geoms, [g for _, g, _ in scans], [o for _, _, o in scans])
    say("batch", len(batch), "queued", batch.queued_scans, "items", batch.work_items, "workgroups", batch.workgroups)
    assert batch.queued_scans == 3
    echoes = [dev(W.random_echo(a, 60 + i)) for i, (a, _, _) in enumerate(scans)]
    outs = pr.reconstruct_hybrid_batch(batch, echoes)
    for i, ((a, grid, o), g) in enumerate(zip(scans, geoms)):
        single = host(pr.reconstruct_hybrid(g, grid, echoes[i], **o))
        got = host(outs[i])
        err = rel(got, single)
        say("   scan", i, "batch vs single", err)
        assert err == 0.0, i      # same kernels, same arithmetic
    # and the oracle for one queued scan
    a, grid, _ = scans[1]
    ref = ohyb.image(ogeom.build(a), grid, W.random_echo(a, 61))
    assert rel(host(outs[1]), ref) < 1e-4


def test_batch_c5_against_oracle():
    wls = W.batch_c5()
    geoms = [pr.make_geometry(w.array) for w in wls]
    batch = pr.HybridBatch(geoms, [w.grid for w in wls])
    say("C5 batch: queued", batch.queued_scans, "items", batch.work_items, "workgroups", batch.workgroups)
    assert batch.queued_scans == len(wls)
    echoes = [dev(W.random_echo(w.array, 70 + i)) for i, w in enumerate(wls)]
    outs = pr.reconstruct_hybrid_batch(batch, echoes)
    for i in (0, 7, 15):
        w = wls[i]
        img = host(outs[i])
        assert np.all(np.isfinite(img))
        npix = w.grid.nx * w.grid.ny
        kap = sorted(set(W.random_subset(w.array.n_scan, 2, 80 + i).tolist() + [0]))
        pix = W.random_subset(npix, 96, 90 + i)
        px, py = ohyb.pixel_grid(w.grid)
        ref = ohyb.spectrum_at(ogeom.build(w.array), ohyb.scan_spectrum(W.random_echo(w.array, 70 + i)), kap,
                               px[pix], py[pix])
        err = rel(_spectrum_subset(img, kap, pix), ref)
        say("   scan", i, w.name, "rel L2", err)
        assert err < 1e-4


def test_batch_graph_replays():
    scans = _small_batch()[:3]
    geoms = [pr.make_geometry(a) for a, _, _ in scans]
    batch = pr.HybridBatch(geoms, [g for _, g, _ in scans])
    e1 = [dev(W.random_echo(a, 100 + i)) for i, (a, _, _) in enumerate(scans)]
    e2 = [dev(W.random_echo(a, 200 + i)) for i, (a, _, _) in enumerate(scans)]
    eager1 = [host(t) for t in pr.reconstruct_hybrid_batch(batch, e1)]
    eager2 = [host(t) for t in pr.reconstruct_hybrid_batch(batch, e2)]
    cap = pr.CapturedBatch(batch, e1)
    for rep in range(4):
        src = e1 if rep % 2 == 0 else e2
        want = eager1 if rep % 2 == 0 else eager2
        for dst, e in zip(cap.echoes, src):
            dst.copy_(e)
        outs = cap.replay()
        got = [host(t) for t in outs]
        # eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        for i in range(len(scans)):
            assert rel(got[i], want[i]) == 0.0, (rep, i)
        del junk


def test_prepared_batch_matches_plain_call():
    # the plan-caching form: tables written once by hybrid_batch_prepare,
    # then calls without them give the plain call's images bit for bit
    scans = _small_batch()
    geoms = [pr.make_geometry(a) for a, _, _ in scans]
    batch = pr.HybridBatch(geoms, [g for _, g, _ in scans])
    echoes = [dev(W.random_echo(a, 300 + i)) for i, (a, _, _) in enumerate(scans)]
    plain = [host(t) for t in pr.reconstruct_hybrid_batch(batch, echoes)]
    ws = pr.workspace(batch.workspace_bytes)
    pr.hybrid_batch_prepare(batch, ws)
    for _ in range(2):
        got = [host(t) for t in pr.reconstruct_hybrid_batch(batch, echoes, ws=ws, prepared=True)]
        for i in range(len(scans)):
            assert rel(got[i], plain[i]) == 0.0, i
    with pytest.raises(ValueError):
        pr.reconstruct_hybrid_batch(batch, echoes, prepared=True)


def test_autotuned_batch_matches_single_scans(tmp_path):
    # per-scan tuned launch shapes (timed on the device, cached): the batch
    # call equals single-scan calls with the same options bit for bit and
    # the oracle within the FP32 bar
    scans = _small_batch()[:3]
    geoms = [pr.make_geometry(a) for a, _, _ in scans]
    grids = [g for _, g, _ in scans]
    cache = str(tmp_path / "tune.json")
    batch = pr.HybridBatch.autotuned(geoms, grids, cache=cache, repeats=2)
    say("autotuned batch options", batch.opts)
    assert os.path.exists(cache)
    echoes = [dev(W.random_echo(a, 300 + i)) for i, (a, _, _) in enumerate(scans)]
    outs = pr.reconstruct_hybrid_batch(batch, echoes)
    for i, g in enumerate(geoms):
        single = host(pr.reconstruct_hybrid(g, grids[i], echoes[i], **batch.opts[i]))
        assert np.array_equal(host(outs[i]).view(np.uint32), single.view(np.uint32)), i
    a, grid, _ = scans[0]
    ref = ohyb.image(ogeom.build(a), grid, W.random_echo(a, 300))
    assert rel(host(outs[0]), ref) < 1e-4


def test_autotune_picks_a_valid_configuration(tmp_path):
    from paper_2109_02842_amd import autotune as at
    wl = W.C1
    grid = _fine_grid(45, 29, 0.003)
    g = pr.make_geometry(wl.array)
    cache = str(tmp_path / "tune.json")
    best, times = at.autotune(g, grid, "bf16", cache=cache, repeats=2)
    say("autotune", best, "of", len(times), "candidates")
    assert len(times) == len(at.candidates(g, grid, "bf16")) and min(times.values()) > 0
    s = W.random_echo(wl.array, 48)
    img = host(pr.reconstruct_hybrid(g, grid, dev(s), **best))
    assert rel(img, ohyb.image(ogeom.build(wl.array), grid, s)) < 1e-3
    assert at.autotune(g, grid, "bf16", cache=cache) == (best, times)     # cached


# --------------------------------------------------- adjoint and autograd
def _adjoint_case(name):
    if name == "C1":
        return W.C1.array, _fine_grid(45, 29, 0.003)
    return multi_small().array, _fine_grid(27, 35, 0.004)


@pytest.mark.parametrize("case", ["C1", "multi-small"])
def test_adjoint_matches_oracle_and_dot_product(case):
    desc, grid = _adjoint_case(case)
    g = pr.make_geometry(desc)
    assert pr.hybrid_plan_info(g, grid).bp_kernel == "pixel-lanes"
    arr = ogeom.build(desc)
    rng = np.random.default_rng(7)
    img = W.complex_normal(rng, (desc.n_scan, grid.ny, grid.nx)).astype(np.complex64)
    s = W.random_echo(desc, 8)
    adj = host(pr.adjoint_hybrid(g, grid, dev(img)))
    ref = ohyb.image_adjoint(arr, grid, img)
    err = rel(adj, ref)
    fwd = host(pr.reconstruct_hybrid(g, grid, dev(s)))
    lhs = np.vdot(fwd.astype(np.complex128), img.astype(np.complex128))
    rhs = np.vdot(s.astype(np.complex128), adj.astype(np.complex128))
    dot = abs(lhs - rhs) / (np.linalg.norm(fwd) * np.linalg.norm(img))
    say("adjoint", case, "rel L2 vs oracle", err, "dot-product mismatch", dot)
    assert err < 1e-4
    assert dot < 2e-6
    # owner-computes adjoint: fixed summation order, bitwise repeatable
    adj2 = host(pr.adjoint_hybrid(g, grid, dev(img)))
    assert np.array_equal(adj.view(np.uint32), adj2.view(np.uint32))


def test_adjoint_ragged_grid_and_64_bin_blocks():
    # ragged tiles, both k_z block sizes of the pixel-per-lane plan, and
    # segments that end inside the range grid
    desc, _ = _adjoint_case("C1")
    grid = _fine_grid(37, 21, 0.0031)
    g = pr.make_geometry(desc)
    arr = ogeom.build(desc)
    rng = np.random.default_rng(9)
    img = W.complex_normal(rng, (desc.n_scan, grid.ny, grid.nx)).astype(np.complex64)
    ref = ohyb.image_adjoint(arr, grid, img)
    for kb in (32, 64):
        plan = pr.hybrid_plan_info(g, grid, kz_block=kb)
        assert plan.bp_kernel == "pixel-lanes" and plan.block == kb
        adj = host(pr.adjoint_hybrid(g, grid, dev(img), kz_block=kb))
        err = rel(adj, ref)
        say("adjoint ragged", kb, "k_z bins: rel L2", err, "n_l", plan.n_l)
        assert err < 1e-4


def test_autograd_gradients_against_oracle_and_finite_differences():
    from paper_2109_02842_amd import autograd as ag
    desc, grid = _adjoint_case("C1")
    g = pr.make_geometry(desc)
    arr = ogeom.build(desc)
    rng = np.random.default_rng(11)
    x = W.complex_normal(rng, (desc.n_scan, grid.ny, grid.nx)).astype(np.complex64)
    s = W.random_echo(desc, 12)
    xt = dev(x).requires_grad_(True)
    res = ag.echo_model(g, grid, xt) - dev(s)
    loss = torch.sum(res.real ** 2 + res.imag ** 2)
    loss.backward()
    grad = host(xt.grad)
    # the oracle's gradient of ||H^H x - s||^2: 2 H (H^H x - s)
    want = 2.0 * ohyb.image(arr, grid, ohyb.image_adjoint(arr, grid, x) - s)
    err = rel(grad, want)
    # central differences (the loss is quadratic: exact up to rounding)
    d = W.complex_normal(np.random.default_rng(13), x.shape).astype(np.complex64)
    eps = 1e-2 * np.linalg.norm(x) / np.linalg.norm(d)

    def loss_at(v):
        r = host(pr.adjoint_hybrid(g, grid, dev(v.astype(np.complex64)))).astype(np.complex128) - s
        return float(np.vdot(r, r).real)

    fd = (loss_at(x + eps * d) - loss_at(x - eps * d)) / (2 * eps)
    dd = float(np.vdot(grad.astype(np.complex128), d.astype(np.complex128)).real)
    say("autograd: grad vs oracle", err, "directional derivative", dd, "finite difference", fd)
    assert err < 1e-4
    assert abs(dd - fd) < 1e-4 * abs(fd)
    # the imaging operator's own backward is the adjoint
    st = dev(s).requires_grad_(True)
    out = ag.reconstruct(g, grid, st)
    (out.real.sum() + 2.0 * out.imag.sum()).backward()
    ones = np.ones(out.shape, dtype=np.complex128) * (1.0 + 2.0j)
    assert rel(host(st.grad), ohyb.image_adjoint(arr, grid, ones)) < 1e-4


@pytest.mark.parametrize("method", ["cg", "sd"])
def test_least_squares_refinement(method, tmp_path):
    from paper_2109_02842_amd import autograd as ag
    desc, grid = _adjoint_case("C1")
    g = pr.make_geometry(desc)
    # echo of a sparse scene through the echo model, plus 1 % noise
    rng = np.random.default_rng(21)
    truth = np.zeros((desc.n_scan, grid.ny, grid.nx), dtype=np.complex64)
    idx = rng.choice(truth.size, 12, replace=False)
    truth.reshape(-1)[idx] = W.complex_normal(rng, 12)
    s = host(pr.adjoint_hybrid(g, grid, dev(truth)))
    s = (s + 0.01 * np.linalg.norm(s) / np.sqrt(s.size) * W.complex_normal(rng, s.shape)).astype(np.complex64)
    x, hist = ag.refine(g, grid, dev(s), steps=10, method=method)
    say("refine", method, ["%.4g" % h for h in hist])
    assert len(hist) == 11
    assert all(b <= a * (1 + 1e-6) for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]
    # interrupted after 4 steps, resumed from the checkpoint: the same
    # iterate bit for bit (deterministic kernels, same operation order)
    ck = str(tmp_path / f"refine-{method}.pt")
    ag.refine(g, grid, dev(s), steps=4, method=method, checkpoint=ck)
    x2, hist2 = ag.refine(g, grid, dev(s), steps=10, method=method, checkpoint=ck, resume=True)
    assert hist2 == hist
    assert np.array_equal(host(x2).view(np.uint32), host(x).view(np.uint32))


# ------------------------------------------------ omega-K variant (resampling)
def evanescent_small():
    # a 2 mm scan step reaches k_z / 2 = 785 rad/m > k at 34 GHz: whole rows
    # evanescent, and rows with 1-3 propagating frequencies (short stencils)
    arr = W.ArrayDesc(mode="multi", n_chords=2, radius=0.4, n_elem=6, spacing=W._D_MULTI, n_tx=2,
                      n_scan=30, scan_step=0.002, n_freq=12, f_start=26e9, f_stop=34e9)
    return W.Workload(name="evanescent-small", array=arr, grid=W.ImageGrid.centred(20, 0.16),
                      scene=W.Scene(n=3, kind="box", half=(0.06, 0.06, 0.02), seed=8, min_sep=0.03))


@pytest.mark.parametrize("wlname", ["tiny-mono", "tiny-multi", "multi-small", "C1", "evanescent-small",
                                    "C1-fine", "multi-small-fine"])
def test_resample_range_method_matches_oracle(wlname):
    # random echoes fill the whole unambiguous range, so the method's own
    # error (interpolating the demodulated spectrum) is large here; the
    # oracle of the same method is the reference.  Each case runs the
    # automatic back-projection and the k_z-per-lane one.
    wl = {"tiny-mono": W.tiny("mono"), "tiny-multi": W.tiny("multi"), "multi-small": multi_small(),
          "C1": W.C1, "evanescent-small": evanescent_small(),
          "C1-fine": replace(W.C1, grid=_fine_grid(45, 29, 0.003)),
          "multi-small-fine": replace(multi_small(), grid=_fine_grid(27, 35, 0.004))}[wlname]
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    s = W.random_echo(wl.array, 71)
    ref, dkl = None, None
    for extra in ({}, {"kz_per_lane": 1}):      # the automatic back-projection, then k_z per lane
        opts = dict(range_method="resample", **extra)
        plan = pr.hybrid_plan_info(g, wl.grid, **opts)
        kernel = plan.bp_kernel
        assert plan.range_method == "resample" and (kernel == "kz-lanes" or not extra)
        assert plan.dk_uniform == pytest.approx(2 * math.pi / (plan.n_fine * plan.du), rel=1e-12)
        if dkl != plan.dk_uniform:
            dkl = plan.dk_uniform
            ref = oomk.image(arr, wl.grid, s, dkl)
        say("resample range method", wlname, kernel, "dk_uniform", dkl)
        img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), **opts))
        err = rel(img, ref)
        say("   rel L2 vs omega-K oracle", err)
        assert err < 1e-4
    if wlname == "C1":
        # the separate steps give the same image
        opts = dict(range_method="resample")
        img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), **opts))
        spec = pr.scan_fft(g, dev(s))
        q, _ = pr.range_compress(g, wl.grid, spec, **opts)
        G = pr.backproject(g, wl.grid, q, **opts)
        assert rel(host(pr.kz_ifft(g, wl.grid, G)), img) < 1e-6


def table1_small(mode):
    # the sampling of the paper's Table 1 (R = 1 m, 30-35 GHz in 51 steps,
    # 5 mm scan steps) on a smaller array: the sweep samples the scene's
    # range extent finely, the regime the interpolation is meant for
    if mode == "mono":
        arr = W.ArrayDesc(mode="mono", n_chords=3, radius=1.0, n_elem=40, spacing=0.0048, n_scan=32,
                          scan_step=0.005, n_freq=51, f_start=30e9, f_stop=35e9)
    else:
        arr = W.ArrayDesc(mode="multi", n_chords=3, radius=1.0, n_elem=20, spacing=0.0102, n_tx=2, n_scan=32,
                          scan_step=0.005, n_freq=51, f_start=30e9, f_stop=35e9)
    return W.Workload(name=f"table1-small-{mode}", array=arr, grid=W.ImageGrid.centred(32, 0.2),
                      scene=W.Scene(n=4, kind="box", half=(0.08, 0.08, 0.05), seed=5, min_sep=0.04))


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_resample_point_targets_focus_where_the_nufft_does(mode):
    # point targets inside the image on the Table 1 sampling: the resampled
    # image stays within a few percent of the NUFFT image (which is within
    # 1e-4 of the exact sum) and peaks at the same voxel; the FP64 oracles
    # of the two methods differ by 5.3% on this scene
    wl = table1_small(mode)
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    pos, refl = W.scatterers(wl.scene)
    s = osim.echo(arr, pos, refl).astype(np.complex64)
    a = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), range_method="resample"))
    b = host(pr.reconstruct_hybrid(g, wl.grid, dev(s)))
    ia, ib = np.unravel_index(np.argmax(np.abs(a)), a.shape), np.unravel_index(np.argmax(np.abs(b)), b.shape)
    assert ia == ib
    err = rel(a, b)
    say("resample vs NUFFT, point targets,", mode, ": rel L2", err, "peak", abs(a[ia]) / abs(b[ib]))
    assert err < 0.08


def test_resample_full_size_sampled():
    # the benchmark's monostatic workload with the resampling range method,
    # sampled (k_z, pixel) pairs against the oracle of the same method
    wl = W.C2
    g = pr.make_geometry(wl.array)
    arr = ogeom.build(wl.array)
    plan = pr.hybrid_plan_info(g, wl.grid, range_method="resample")
    s = W.random_echo(wl.array, 22)
    say("full size resample", wl.name, "dk_uniform", plan.dk_uniform)
    img = host(pr.reconstruct_hybrid(g, wl.grid, dev(s), range_method="resample"))
    assert np.all(np.isfinite(img))
    npix = wl.grid.nx * wl.grid.ny
    kap = sorted(set(W.random_subset(wl.array.n_scan, 3, 41).tolist() + [0, wl.array.n_scan // 2]))
    pix = np.unique(np.concatenate([W.random_subset(npix, 256, 42), [0, npix - 1, wl.grid.nx - 1]]))
    px, py = ohyb.pixel_grid(wl.grid)
    ref = oomk.spectrum_at(arr, ohyb.scan_spectrum(s), kap, px[pix], py[pix], plan.dk_uniform,
                           oomk.reference_lengths(arr, wl.grid))
    err = rel(_spectrum_subset(img, kap, pix), ref)
    say("   rel L2", err)
    assert err < 1e-4


def test_resample_in_a_batch_matches_single_scans():
    c1 = W.C1
    scans = [(c1.array, _fine_grid(45, 29, 0.003), dict(range_method="resample")),
             (replace(c1.array, n_scan=30, n_freq=20), _fine_grid(21, 40, 0.004), {})]
    geoms = [pr.make_geometry(a) for a, _, _ in scans]
    batch = pr.HybridBatch(geoms, [g for _, g, _ in scans], [o for _, _, o in scans])
    echoes = [dev(W.random_echo(a, 80 + i)) for i, (a, _, _) in enumerate(scans)]
    outs = pr.reconstruct_hybrid_batch(batch, echoes)
    for i, ((a, grid, o), g) in enumerate(zip(scans, geoms)):
        assert rel(host(outs[i]), host(pr.reconstruct_hybrid(g, grid, echoes[i], **o))) == 0.0, i
