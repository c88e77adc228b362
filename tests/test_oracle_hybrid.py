"""Pins of the oracle's hybrid inversion (eqs. 2-9, 12-19) against facts that
do not come from the oracle: brute-force DFTs, a numerical Fourier transform of
the Green's function (the stationary-phase dispersion relations (5) and (18)),
symmetries of the operator, focusing at known target positions, and the
paper's resolution formulas (23)-(26)."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import geometry, hybrid, nudft, simulate

C = W.SPEED_OF_LIGHT


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 24, 64])
def test_scan_transform_is_forward_dft(n):
    rng = np.random.default_rng(n)
    s = W.complex_normal(rng, (2, n, 3))
    m = np.arange(n)
    dft = np.exp(-2j * np.pi * np.outer(m, m) / n)     # brute-force DFT matrix
    ref = np.einsum("km,cmf->ckf", dft, s)
    assert np.allclose(hybrid.scan_spectrum(s), ref, atol=1e-10)
    back = np.fft.ifft(hybrid.scan_spectrum(s), axis=1)
    assert np.allclose(back, s, atol=1e-12)
    # spatial frequency grid: kappa-th bin is 2 pi kappa / (n dz), wrapped
    kz = hybrid.kz_grid(n, 0.004)
    for kap in range(n):
        assert np.isclose(np.exp(-1j * kz[kap] * 0.004 * m), dft[kap]).all()


# ------------------------------------------------------- dispersion relation
def _green_ft_phase(k, kz, rho_t, rho_r):
    """Phase of int exp(-j k (R_T + R_R)) exp(-j kz u) du by dense quadrature,
    with R = sqrt(rho^2 + u^2) and a smooth taper far from the stationary
    point (independent of any closed form)."""
    u = np.linspace(-4.0, 4.0, 400001)
    taper = np.ones_like(u)
    edge = np.abs(u) > 2.5
    taper[edge] = np.cos(0.5 * np.pi * (np.abs(u[edge]) - 2.5) / 1.5) ** 2
    ph = -k * (np.sqrt(rho_t ** 2 + u ** 2) + np.sqrt(rho_r ** 2 + u ** 2)) - kz * u
    val = np.sum(taper * np.exp(1j * ph)) * (u[1] - u[0])
    return np.angle(val)


@pytest.mark.parametrize("mode,k,kz", [("mono", 600.0, 0.0), ("mono", 600.0, 450.0),
                                       ("mono", 700.0, -800.0), ("multi", 650.0, 300.0),
                                       ("multi", 560.0, -900.0)])
def test_dispersion_matches_numerical_green_transform(mode, k, kz):
    # Phase slope of the transformed Green's function with respect to the
    # horizontal range is -k_rho (per unit of l = rho for mono, l = rho_T + rho_R
    # for multi with rho_T = rho_R), eqs. (3)-(5) and (16)-(18).
    r1, dr = 0.5, 0.0008
    if mode == "mono":
        p1 = _green_ft_phase(k, kz, r1, r1)
        p2 = _green_ft_phase(k, kz, r1 + dr, r1 + dr)
        dl = dr            # l = rho
    else:
        p1 = _green_ft_phase(k, kz, r1, r1)
        p2 = _green_ft_phase(k, kz, r1 + dr, r1 + dr)
        dl = 2 * dr        # l = rho_T + rho_R
    slope = -np.angle(np.exp(1j * (p2 - p1))) / dl
    krho, valid = hybrid.dispersion(mode, np.array([k]), kz)
    assert valid[0]
    assert abs(slope - krho[0]) / krho[0] < 2e-3
    # the alternatives a dropped factor would give are far off
    for wrong in (np.sqrt(k * k - kz * kz / 4), np.sqrt(4 * k * k - kz * kz)):
        if not np.isclose(wrong, krho[0]):
            assert abs(slope - wrong) / wrong > 0.05


def test_evanescent_terms_are_masked():
    krho, valid = hybrid.dispersion("mono", np.array([100.0, 400.0]), 300.0)
    assert not valid[0] and valid[1] and krho[0] == 0.0
    krho, valid = hybrid.dispersion("multi", np.array([100.0, 400.0]), 300.0)
    assert not valid[0] and valid[1]


# ---------------------------------------------------------- operator facts
def _tiny(mode):
    wl = W.tiny(mode)
    return wl, geometry.build(wl.array)


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_linearity(mode):
    wl, arr = _tiny(mode)
    s1 = W.random_echo(wl.array, 1, np.complex128)
    s2 = W.random_echo(wl.array, 2, np.complex128)
    a, b = 1.5 - 0.25j, -0.7 + 2j
    lhs = hybrid.image(arr, wl.grid, a * s1 + b * s2)
    rhs = a * hybrid.image(arr, wl.grid, s1) + b * hybrid.image(arr, wl.grid, s2)
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-9 * np.abs(rhs).max())


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_circular_scan_shift_is_image_shift(mode):
    wl, arr = _tiny(mode)
    s = W.random_echo(wl.array, 3, np.complex128)
    g = hybrid.image(arr, wl.grid, s)
    g_shift = hybrid.image(arr, wl.grid, np.roll(s, 1, axis=1))
    assert np.allclose(g_shift, np.roll(g, 1, axis=0), atol=1e-9 * np.abs(g).max())


def test_multistatic_with_coincident_tx_rx_equals_monostatic():
    # (18) with l = rho_T + rho_R = 2 rho must reproduce (5) with l = rho
    wl, arr = _tiny("mono")
    s = W.random_echo(wl.array, 4, np.complex128)
    g_mono = hybrid.image(arr, wl.grid, s)
    g_multi = hybrid.image(replace(arr, mode="multi"), wl.grid, s)
    assert np.allclose(g_multi, g_mono, atol=1e-9 * np.abs(g_mono).max())


def test_subset_evaluator_matches_full_spectrum():
    wl, arr = _tiny("multi")
    s = W.random_echo(wl.array, 5, np.complex128)
    G = hybrid.spectrum(arr, wl.grid, s)
    g = hybrid.image(arr, wl.grid, s)
    assert np.allclose(np.fft.fft(g, axis=0), G, atol=1e-9 * np.abs(G).max())
    px, py = hybrid.pixel_grid(wl.grid)
    sel = [3, 17, 40]
    sub = hybrid.spectrum_at(arr, hybrid.scan_spectrum(s), [2, 7], px[sel], py[sel])
    assert np.allclose(sub, G.reshape(G.shape[0], -1)[[2, 7]][:, sel], atol=1e-12 * np.abs(G).max())


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_two_step_form_equals_direct_sum_for_any_reference(mode):
    # (8a)+(8b): q evaluated exactly at l = l_c(p), times exp(+j k_rho0 l), summed
    # over channels, is the direct sum of (7) whatever k_rho0 is.
    wl, arr = _tiny(mode)
    s = W.random_echo(wl.array, 6, np.complex128)
    S = hybrid.scan_spectrum(s)
    px, py = hybrid.pixel_grid(wl.grid)
    l = hybrid.range_of(arr, px, py)
    kz = hybrid.kz_grid(arr.z_scan.size, arr.scan_step)
    for kap in (0, 3, 7):
        direct = hybrid.spectrum_at(arr, S, [kap], px, py)[0]
        krho0 = hybrid.dispersion(mode, arr.k[:1], kz[kap])[0][0]  # paper: k at k_0 = min k
        for kref in (krho0, 123.4):
            q = nudft.range_profiles(arr, S, kap, kref, l)      # q[c, p] at l = l_c(p)
            two_step = np.sum(q * np.exp(1j * kref * l), axis=0)
            assert np.allclose(two_step, direct, atol=1e-10 * np.abs(direct).max())


# -------------------------------------------------------- imaging behaviour
def _local_max_near(a, idx, radius=1):
    z, y, x = idx
    sl = a[max(z - radius, 0):z + radius + 1, max(y - radius, 0):y + radius + 1,
           max(x - radius, 0):x + radius + 1]
    loc = np.unravel_index(np.argmax(sl), sl.shape)
    pz, py, px = loc[0] + max(z - radius, 0), loc[1] + max(y - radius, 0), loc[2] + max(x - radius, 0)
    # a local maximum of the full image (3x3x3 neighbourhood)
    nb = a[max(pz - 1, 0):pz + 2, max(py - 1, 0):py + 2, max(px - 1, 0):px + 2]
    return a[pz, py, px] >= nb.max()


@pytest.fixture(scope="module")
def c1_noise_free():
    wl = W.C1
    arr = geometry.build(wl.array)
    pos, refl = W.scatterers(wl.scene)
    s = simulate.echo(arr, pos, refl)
    return wl, arr, pos, refl, s


def test_c1_point_targets_focus_at_true_positions(c1_noise_free):
    wl, arr, pos, refl, s = c1_noise_free
    a = np.abs(hybrid.image(arr, wl.grid, s))
    x, y = geometry.pixel_centres(wl.grid)
    strong = np.abs(refl) >= 0.2 * np.abs(refl).max()
    assert strong.sum() >= 3
    for p in pos[strong]:
        idx = (np.argmin(abs(arr.z_scan - p[2])), np.argmin(abs(y - p[1])), np.argmin(abs(x - p[0])))
        assert _local_max_near(a, idx), f"no focus near target {p}"


def test_c1_noise_does_not_move_peaks(c1_noise_free):
    wl, arr, pos, refl, s = c1_noise_free
    noisy = simulate.add_noise(s, wl.noise_db, W.noise(s.shape, wl.scene.seed))
    a0 = np.abs(hybrid.image(arr, wl.grid, s))
    a1 = np.abs(hybrid.image(arr, wl.grid, noisy))
    assert np.unravel_index(np.argmax(a0), a0.shape) == np.unravel_index(np.argmax(a1), a1.shape)
    assert np.linalg.norm(a1 - a0) / np.linalg.norm(a0) < 0.1


def _width_3db(profile, step):
    p = profile / profile.max()
    i = int(np.argmax(p))
    lo = i
    while lo > 0 and p[lo] > 0.5 ** 0.5:
        lo -= 1
    hi = i
    while hi < p.size - 1 and p[hi] > 0.5 ** 0.5:
        hi += 1
    # linear interpolation of the -3 dB crossings
    t = 0.5 ** 0.5
    xl = lo + (t - p[lo]) / (p[lo + 1] - p[lo])
    xh = hi - (t - p[hi]) / (p[hi - 1] - p[hi])
    return (xh - xl) * step


def test_point_spread_widths_follow_resolution_formulas():
    # Single target at the scene centre, C1 array, fine pixel grid.  The -3 dB
    # width of a uniform-aperture response is 0.886 of the Rayleigh-type
    # resolution of (24)-(26); accept +-30 % as the array is a polyline.
    wl = W.C1
    arr = geometry.build(wl.array)
    s = simulate.echo(arr, np.zeros((1, 3)), np.ones(1))
    grid = W.ImageGrid(nx=41, ny=41, x0=-0.04, y0=-0.04, dx=0.002, dy=0.002)
    G = hybrid.spectrum(arr, grid, s)                 # (n_kz, ny, nx)
    pad = 16
    n = G.shape[0]
    Gp = np.zeros((n * pad,) + G.shape[1:], dtype=complex)
    h = (n + 1) // 2
    Gp[:h] = G[:h]
    Gp[-(n - h):] = G[h:]
    g = np.abs(np.fft.ifft(Gp, axis=0))
    iz, iy, ix = np.unravel_index(np.argmax(g), g.shape)
    lam_c = C / (0.5 * (wl.array.f_start + wl.array.f_stop))
    ends = arr.chord_ends
    theta_h = np.arctan2(ends[-1, 1, 1], ends[-1, 1, 0]) - np.arctan2(ends[0, 0, 1], ends[0, 0, 0])
    dx_pred = lam_c / (4 * np.sin(theta_h / 2))                           # (24)
    dy_pred = C / (2 * (wl.array.f_stop - wl.array.f_start))               # (26)
    half_scan = 0.5 * wl.array.n_scan * wl.array.scan_step
    theta_z = 2 * np.arctan(half_scan / wl.array.radius)
    dz_pred = lam_c / (4 * np.sin(theta_z / 2))                           # (25)
    wx = _width_3db(g[iz, iy, :], grid.dx)
    wy = _width_3db(g[iz, :, ix], grid.dy)
    wz = _width_3db(np.roll(g[:, iy, ix], n * pad // 2 - iz), wl.array.scan_step / pad)
    for w, pred in ((wx, dx_pred), (wy, dy_pred), (wz, dz_pred)):
        assert 0.7 < w / (0.886 * pred) < 1.3, (w, pred)


def test_multistatic_point_targets_focus_at_true_positions():
    # Tx at the chord ends and Rx spread along each chord: the range of
    # (19b) is rho_T + rho_R, with the dispersion relation (18).
    arr_desc = W.ArrayDesc(mode="multi", n_chords=3, radius=0.5, n_elem=16, spacing=W._D_MULTI,
                           n_tx=4, n_scan=24, scan_step=0.005, n_freq=16, f_start=26e9, f_stop=34e9)
    grid = W.ImageGrid.centred(32, 0.30)
    scene = W.Scene(n=4, kind="box", half=(0.12, 0.12, 0.04), seed=21, min_sep=0.06)
    arr = geometry.build(arr_desc)
    pos, refl = W.scatterers(scene)
    refl = refl / np.abs(refl)                    # equal strengths
    a = np.abs(hybrid.image(arr, grid, simulate.echo(arr, pos, refl)))
    x, y = geometry.pixel_centres(grid)
    for p in pos:
        idx = (np.argmin(abs(arr.z_scan - p[2])), np.argmin(abs(y - p[1])), np.argmin(abs(x - p[0])))
        assert _local_max_near(a, idx), f"no focus near target {p}"
        z, yy, xx = idx
        near = a[max(z - 1, 0):z + 2, max(yy - 1, 0):yy + 2, max(xx - 1, 0):xx + 2]
        assert near.max() > 0.1 * a.max()


def test_multistatic_image_matches_bp_shape():
    # BP sums exp(+j k (R_T + R_R)) with 3-D distances; the hybrid image built
    # on rho_T + rho_R must match it in shape on the plane of a target.
    from oracle import bp
    arr_desc = W.ArrayDesc(mode="multi", n_chords=3, radius=0.5, n_elem=16, spacing=W._D_MULTI,
                           n_tx=4, n_scan=24, scan_step=0.005, n_freq=16, f_start=26e9, f_stop=34e9)
    grid = W.ImageGrid.centred(32, 0.30)
    arr = geometry.build(arr_desc)
    pos = np.array([[0.03, 0.02, 0.0], [-0.07, -0.05, 0.0]])
    s = simulate.echo(arr, pos, np.ones(2))
    iz = int(np.argmin(abs(arr.z_scan)))
    gh = np.abs(hybrid.image(arr, grid, s))[iz]
    gb = np.abs(bp.bp_image(arr, grid, s, z_index=[iz]))[0]
    a, b = gh / gh.max(), gb / gb.max()
    focal = (a > 0.1) | (b > 0.1)
    assert np.corrcoef(a[focal], b[focal])[0, 1] > 0.95


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_single_scan_position_is_bp_on_the_scan_plane(mode):
    # One scan position: the only spatial frequency is k_z = 0, where (5)
    # and (18) give k_rho = 2k (mono) and k (multi, range rho_T + rho_R);
    # on the plane of the scan the 3-D distances equal the horizontal ones,
    # so the hybrid image is exactly the brute-force BP sum there.
    from oracle import bp
    wl = W.tiny(mode)
    arr = geometry.build(replace(wl.array, n_scan=1))
    rng = np.random.default_rng(9)
    s = W.complex_normal(rng, arr_echo_shape(arr))
    gh = hybrid.image(arr, wl.grid, s)
    gb = bp.bp_image(arr, wl.grid, s, z_index=[0])
    assert gh.shape == gb.shape == (1, wl.grid.ny, wl.grid.nx)
    assert np.linalg.norm(gh - gb) <= 1e-12 * np.linalg.norm(gb)


def test_image_adjoint_dot_product():
    # <H s, g> = <s, H^H g> for random echo and image (inner products in the
    # complex128 sense, conjugate on the first argument)
    wl = W.tiny("multi")
    arr = geometry.build(wl.array)
    rng = np.random.default_rng(5)
    s = W.complex_normal(rng, arr_echo_shape(arr))
    g = W.complex_normal(rng, (arr.z_scan.size, wl.grid.ny, wl.grid.nx))
    lhs = np.vdot(hybrid.image(arr, wl.grid, s), g)
    rhs = np.vdot(s, hybrid.image_adjoint(arr, wl.grid, g))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_image_adjoint_is_the_conjugate_transpose():
    # brute force on a tiny problem: the matrix of the adjoint, built column
    # by column from unit images, equals the conjugate transpose of the
    # matrix of the forward operator built from unit echoes
    desc = W.ArrayDesc(mode="mono", n_chords=2, radius=0.5, n_elem=2, spacing=W._D_MONO, n_scan=4,
                       scan_step=0.005, n_freq=3, f_start=26e9, f_stop=34e9)
    grid = W.ImageGrid(nx=2, ny=2, x0=-0.01, y0=0.02, dx=0.015, dy=0.01)
    arr = geometry.build(desc)
    es = arr_echo_shape(arr)
    ne, ni = int(np.prod(es)), 4 * 2 * 2
    M = np.zeros((ni, ne), dtype=np.complex128)
    for j in range(ne):
        e = np.zeros(ne, dtype=np.complex128)
        e[j] = 1.0
        M[:, j] = hybrid.image(arr, grid, e.reshape(es)).ravel()
    A = np.zeros((ne, ni), dtype=np.complex128)
    for j in range(ni):
        e = np.zeros(ni, dtype=np.complex128)
        e[j] = 1.0
        A[:, j] = hybrid.image_adjoint(arr, grid, e.reshape(4, 2, 2)).ravel()
    assert np.allclose(A, M.conj().T, rtol=0, atol=1e-12 * np.abs(M).max())


def arr_echo_shape(arr):
    return (arr.tx.shape[0], arr.z_scan.size, arr.k.size)
