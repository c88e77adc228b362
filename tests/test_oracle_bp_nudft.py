"""Pins of the oracle's back-projection (comparison method) and of the direct
NUDFT of the range-compression step (8a)."""
import numpy as np
import pytest

import workloads as W
from oracle import bp, geometry, hybrid, nudft, simulate


def _voxels(arr, grid, z_index):
    x = grid.x0 + grid.dx * np.arange(grid.nx)
    y = grid.y0 + grid.dy * np.arange(grid.ny)
    zz, yy, xx = np.meshgrid(arr.z_scan[z_index], y, x, indexing="ij")
    return xx.ravel(), yy.ravel(), zz.ravel()


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_bp_is_adjoint_of_simulator_with_k_weight(mode):
    # <sigma, BP(s)> = <A sigma, W s> with A the echo model at voxel centres and
    # W = diag(k_f): BP is the matched filter of eqs. (1)/(10).
    wl = W.tiny(mode)
    arr = geometry.build(wl.array)
    zi = np.array([1, 4, 8])
    vx, vy, vz = _voxels(arr, wl.grid, zi)
    rng = np.random.default_rng(11)
    sigma = W.complex_normal(rng, vx.size)
    s = W.random_echo(wl.array, 12, np.complex128)
    a_sigma = simulate.echo(arr, np.stack([vx, vy, vz], 1), sigma)
    lhs = np.vdot(sigma, bp.bp_voxels(arr, s, vx, vy, vz))
    rhs = np.vdot(a_sigma, s * arr.k[None, None, :])
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)
    img = bp.bp_image(arr, wl.grid, s, z_index=zi)
    assert np.allclose(img.ravel(), bp.bp_voxels(arr, s, vx, vy, vz), atol=1e-12 * np.abs(img).max())


def test_bp_linearity():
    wl = W.tiny("mono")
    arr = geometry.build(wl.array)
    vx, vy, vz = _voxels(arr, wl.grid, np.array([2]))
    s1 = W.random_echo(wl.array, 1, np.complex128)
    s2 = W.random_echo(wl.array, 2, np.complex128)
    lhs = bp.bp_voxels(arr, 2j * s1 - s2, vx, vy, vz)
    rhs = 2j * bp.bp_voxels(arr, s1, vx, vy, vz) - bp.bp_voxels(arr, s2, vx, vy, vz)
    assert np.allclose(lhs, rhs, atol=1e-10 * np.abs(rhs).max())


def test_bp_focuses_c1_targets_like_the_hybrid_method():
    # Independent route to the same scene: BP and the hybrid image must peak
    # at the same voxels, and their magnitudes must agree in shape (Sec. III
    # compares the two methods' focusing on simulated point targets and finds
    # them close).
    wl = W.C1
    arr = geometry.build(wl.array)
    pos, refl = W.scatterers(wl.scene)
    s = simulate.echo(arr, pos, refl)
    g = np.abs(hybrid.image(arr, wl.grid, s))
    strongest = np.argmax(np.abs(refl))
    iz = int(np.argmin(abs(arr.z_scan - pos[strongest, 2])))
    gb = np.abs(bp.bp_image(arr, wl.grid, s, z_index=[iz]))[0]
    gh = g[iz]
    assert np.unravel_index(np.argmax(gb), gb.shape) == np.unravel_index(np.argmax(gh), gh.shape)
    a = gb / gb.max()
    b = gh / gh.max()
    focal = (a > 0.1) | (b > 0.1)
    corr = np.corrcoef(a[focal], b[focal])[0, 1]
    assert corr > 0.9


def test_nudft_on_grid_is_inverse_fft():
    n, du = 64, 0.0013
    rng = np.random.default_rng(4)
    nf = rng.choice(np.arange(-n // 2, n // 2), size=17, replace=False)
    a = W.complex_normal(rng, nf.size)
    kp = 2 * np.pi * nf / (n * du)
    u = du * np.arange(n)
    spec = np.zeros(n, complex)
    spec[nf % n] = a
    assert np.allclose(nudft.nudft(a, kp, u), n * np.fft.ifft(spec), atol=1e-12)


def test_nudft_monostatic_kz0_is_uniform():
    # At k_z = 0 the monostatic k_rho = 2k is uniform in f; with the matching
    # grid step the range compression is a plain inverse FFT of the weights.
    wl = W.tiny("mono")
    arr = geometry.build(wl.array)
    krho, valid = hybrid.dispersion("mono", arr.k, 0.0)
    dk = krho[1] - krho[0]
    assert np.allclose(np.diff(krho), dk, rtol=1e-12)
    n = 32
    du = 2 * np.pi / (n * dk)
    u = du * np.arange(n)
    a = W.complex_normal(np.random.default_rng(9), arr.k.size)
    spec = np.zeros(n, complex)
    spec[: arr.k.size] = a
    q = nudft.nudft(a, krho - krho[0], u)
    assert np.allclose(q, n * np.fft.ifft(spec), atol=1e-11)
