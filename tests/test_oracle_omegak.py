"""Pins of the oracle's omega-K variant (range transform by resampling onto a
uniform wavenumber grid and an inverse FFT) against facts that do not come
from it: the textbook properties of Lagrange interpolation (exactness on
polynomials, the remainder bound of a centred cubic stencil), the closed-form
spectrum of a reflector at the reference path, the reduction to the exact
frequency sum when the grid coincides with the samples, and convergence to
the exact sum as the sweep is refined."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry, hybrid, omegak, simulate


# ------------------------------------------------------ Lagrange interpolation
@pytest.mark.parametrize("n_nodes", [1, 2, 3, 4])
def test_lagrange_weights_reproduce_polynomials(n_nodes):
    rng = np.random.default_rng(n_nodes)
    nodes = np.cumsum(rng.uniform(0.5, 1.5, n_nodes))
    for _ in range(20):
        coef = rng.standard_normal(n_nodes)          # degree n_nodes - 1
        t = rng.uniform(nodes[0] - 1.0, nodes[-1] + 1.0)
        w = omegak.lagrange_weights(t, nodes)
        assert np.isclose(w.sum(), 1.0, atol=1e-12)
        assert np.isclose(w @ np.polyval(coef, nodes), np.polyval(coef, t), atol=1e-10)
    # one degree more is not reproduced
    if n_nodes < 4:
        t = nodes[0] + 0.37
        w = omegak.lagrange_weights(t, nodes)
        p = lambda x: np.prod([x - xi for xi in nodes])
        assert abs(w @ np.array([p(x) for x in nodes]) - p(t)) > 1e-6


def _sweep(n_freq, f_start=26e9, f_stop=34e9):
    return 2.0 * math.pi * np.linspace(f_start, f_stop, n_freq) / W.SPEED_OF_LIGHT


def test_stencil_is_the_centred_cubic():
    # With k_z = 0 and L_ref = 0 the row values are interpolated as they are.
    # For exp(j alpha f) the centred 4-point stencil's remainder is
    # alpha^4 / 4! |(t+1) t (t-1) (t-2)| <= alpha^4 / 4! * 9/16 (t in [0, 1]
    # between the middle nodes); a one-sided stencil reaches alpha^4 / 4! * 1.
    k = _sweep(64)
    dk = k[1] - k[0]
    alpha = 0.3
    f = np.arange(k.size)
    row = np.exp(1j * alpha * f)
    klm, Q = omegak.uniform_samples(k, 0.0, row, 0.37 * dk, 0.0)
    t = (klm - k[0]) / dk
    vals = Q / (klm * 0.37)
    inner = (t > 1.0) & (t < k.size - 2.0)
    err = np.abs(vals[inner] - np.exp(1j * alpha * t[inner]))
    frac = t[inner] - np.floor(t[inner])
    bound = alpha ** 4 / 24.0 * np.abs((frac + 1) * frac * (frac - 1) * (frac - 2))
    assert np.all(err <= 1.05 * bound + 1e-12)
    assert err.max() > 0.5 * alpha ** 4 / 24.0 * 9.0 / 16.0   # the bound is attained, not vacuous


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("kz,n_prop", [(0.0, 48), (400.0, 48), (1180.0, 35), (1343.0, 12), (1414.0, 2)])
def test_reflector_at_reference_path(kz, n_prop):
    # S_f = P(k_f) exp(-j k_L,f L0) with P a polynomial of degree < the
    # stencil size: demodulating at L_ref = L0 leaves P, which the stencil
    # reproduces, so Q_m = P(k_m) exp(-j k_L,m L0) k_L,m dkl/dk exactly, with
    # k_m = sqrt(k_L,m^2 + k_z^2/4).  The larger k_z leave n_prop propagating
    # samples at the top of the 48-sample sweep (2: a linear stencil).
    k = _sweep(48)
    dk = k[1] - k[0]
    kl = np.sqrt(np.maximum(k * k - kz * kz / 4.0, 0.0))
    valid = k * k - kz * kz / 4.0 > 0.0
    n_valid = int(valid.sum())
    assert n_valid == n_prop
    deg = min(3, n_valid - 1)
    coef = np.array([0.3 - 0.2j, -1.1, 0.7j, 2.0])[-(deg + 1):] / np.array([700.0 ** p for p in range(deg, -1, -1)])
    L0 = 1.37
    row = np.where(valid, np.polyval(coef, k) * np.exp(-1j * kl * L0), 0.0)
    dkl = 0.83 * dk
    klm, Q = omegak.uniform_samples(k, kz, row, dkl, L0)
    assert klm.size > 0
    assert klm[0] >= kl[valid][0] - 1e-6 and klm[-1] <= kl[-1] + 1e-6
    km = np.sqrt(klm ** 2 + kz * kz / 4.0)
    expect = np.polyval(coef, km) * np.exp(-1j * klm * L0) * klm * dkl / dk
    assert np.allclose(Q, expect, rtol=1e-9, atol=1e-12 * np.abs(expect).max())
    # every grid point of the propagating band is present
    assert klm.size == math.floor(kl[-1] / dkl) - math.ceil(kl[valid][0] / dkl) + 1


def test_evanescent_row_is_empty():
    k = _sweep(16)
    klm, Q = omegak.uniform_samples(k, 2.0 * k[-1] + 1.0, np.ones(16), 1.0, 0.3)
    assert klm.size == 0 and Q.size == 0


def _point_case(mode, n_freq, scan_step=0.004, n_scan=32):
    if mode == "mono":
        a = W.ArrayDesc(mode="mono", n_chords=3, radius=0.5, n_elem=8, spacing=W._D_MONO, n_scan=n_scan,
                        scan_step=scan_step, n_freq=n_freq, f_start=26e9, f_stop=34e9)
    else:
        a = W.ArrayDesc(mode="multi", n_chords=3, radius=0.5, n_elem=6, spacing=W._D_MULTI, n_tx=2,
                        n_scan=n_scan, scan_step=scan_step, n_freq=n_freq, f_start=26e9, f_stop=34e9)
    arr = geometry.build(a)
    grid = W.ImageGrid.centred(16, 0.2)
    echo = simulate.echo(arr, np.array([[0.03, -0.02, 0.01]]), np.array([1.0 + 0j]))
    return arr, grid, echo


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_aligned_grid_reduces_to_exact_sum(mode):
    # At k_z = 0, k_L = k; with dkl = dk and f_start a multiple of the
    # frequency step, the grid points are the samples themselves and the
    # variant is the exact frequency sum of eq. (7) / (19).
    arr, grid, echo = _point_case(mode, 33)          # 0.25 GHz steps, 26 GHz = 104 steps
    dk = arr.k[1] - arr.k[0]
    G_ex = hybrid.spectrum(arr, grid, echo, [0])
    G_om = omegak.spectrum(arr, grid, echo, dk, [0])
    assert np.linalg.norm(G_om - G_ex) <= 1e-10 * np.linalg.norm(G_ex)


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_converges_to_exact_sum(mode):
    # The resampled sum is a quadrature of the same integral (k dk = k_L dk_L)
    # as the exact frequency sum; refining the sweep 4x (65 -> 257 samples
    # over 26-34 GHz) shrinks the difference, which stays at the percent
    # level.  k_z up to 736 rad/m puts k_L / k down to 0.74: a Jacobian of
    # k_m instead of k_L,m, a demodulation of the wrong sign or the
    # monostatic k_m = sqrt(k_L^2 + k_z^2) each fail this.
    kap = [0, 5, 10, 14]
    errs = {}
    for nf in (65, 257):
        arr, grid, echo = _point_case(mode, nf)
        dk = arr.k[1] - arr.k[0]
        G_ex = hybrid.spectrum(arr, grid, echo, kap)
        G_om = omegak.spectrum(arr, grid, echo, 0.7 * dk, kap)
        errs[nf] = np.array([np.linalg.norm(G_om[i] - G_ex[i]) / np.linalg.norm(G_ex[i]) for i in range(len(kap))])
    assert np.all(errs[257] < 2e-2), errs
    assert np.all(errs[257] < 0.6 * errs[65]), errs


def test_periodic_in_path_length():
    # The uniform grid makes q periodic in L with period 2 pi / dkl -- the
    # range period of the inverse FFT the fast path uses.
    arr, grid, echo = _point_case("multi", 33)
    S = hybrid.scan_spectrum(echo)
    dkl = 0.9 * (arr.k[1] - arr.k[0])
    l_ref = omegak.reference_lengths(arr, grid)
    klm, Q = omegak.uniform_samples(arr.k, hybrid.kz_grid(32, 0.004)[3], S[2, 3], dkl, l_ref[2])
    L = np.array([0.4, 0.9, 1.3])
    q0 = np.exp(1j * np.outer(L, klm)) @ Q
    q1 = np.exp(1j * np.outer(L + 2 * np.pi / dkl, klm)) @ Q
    assert np.allclose(q0, q1, rtol=1e-9, atol=1e-9 * np.abs(q0).max())
