"""The 'omega-K BP' variant: the range transform (8a)/(19a) evaluated by
resampling the spectrum onto a uniform wavenumber grid and an inverse FFT, the
conventional route that the paper's NUFFT replaces (Sec. I; Sec. II-A after
eq. 8, where the nonuniform k_rho' samples are the reason a plain IFFT does
not apply; the variant without NUFFT is the middle column of Table 2 and the
'omega-K BP' curves of the 1-D cuts in Sec. III).

Test infrastructure: see the package header.

The paper does not spell this variant out.  Readings used here:
  * Everything is written in the path length L = rho_T + rho_R (monostatic:
    L = 2 rho) and its wavenumber k_L = sqrt(k^2 - k_z^2 / 4) (eq. 18); for
    the monostatic case k_L L equals k_rho rho of eq. (5).
  * The uniform grid is k_L,m = m * dkl for integer m; the step dkl is a
    parameter of the method (an inverse FFT of the grid values is periodic in
    L with period 2 pi / dkl).  Grid points between the k_L of the first and
    of the last propagating frequency are kept (a point within 1e-9 of a step
    outside counts as inside); nothing is extrapolated.
  * The measure "k dk" changes variable as k dk = k_L dk_L, so the frequency
    sum sum_f k_f S_f exp(j k_L,f L) (the exact form, constant dk dropped)
    becomes (dkl / dk) sum_m k_L,m S(k_m) exp(j k_L,m L) with
    k_m = sqrt(k_L,m^2 + k_z^2 / 4) and dk the wavenumber step of the
    (uniform) frequency sweep.
  * S(k_m) is a 4-point Lagrange interpolation, over the frequency index, of
    the spectrum demodulated by exp(+j k_L,f L_ref), then remodulated by
    exp(-j k_L,m L_ref); L_ref is the path length from the channel to the
    centre of the image grid.  The stencil is the two samples on each side of
    k_m, shifted to stay on propagating samples; a row with fewer than four
    propagating samples uses all of them.
  * Where the fast path evaluates the inverse FFT on a range grid and
    interpolates it at each pixel, this module evaluates the trigonometric sum
    at each pixel's path length directly (the FFT's values are this sum on its
    grid).
"""
from __future__ import annotations

import math

import numpy as np

from .hybrid import kz_grid, pixel_grid, range_of, scan_spectrum

EDGE_SLACK = 1e-9   # grid steps: tolerance at the band edges


def path_wavenumber(k, kz):
    """k_L = sqrt(k^2 - k_z^2/4) and the mask of propagating terms (eq. 18)."""
    k = np.asarray(k, dtype=np.float64)
    arg = k * k - 0.25 * kz * kz
    valid = arg > 0.0
    return np.sqrt(np.where(valid, arg, 0.0)), valid


def lagrange_weights(t, nodes):
    """Lagrange basis at t for the given nodes: w_j = prod_{i != j} (t - x_i) / (x_j - x_i)."""
    x = np.asarray(nodes, dtype=np.float64)
    w = np.ones(x.size)
    for j in range(x.size):
        for i in range(x.size):
            if i != j:
                w[j] *= (t - x[i]) / (x[j] - x[i])
    return w


def uniform_samples(k, kz, s_row, dkl, l_ref):
    """Grid wavenumbers k_L,m and values Q_m of one (channel, k_z) row, so that
    q(L) = sum_m Q_m exp(j k_L,m L) approximates sum_f k_f S_f exp(j k_L,f L)."""
    k = np.asarray(k, dtype=np.float64)
    s_row = np.asarray(s_row, dtype=np.complex128)
    kl, valid = path_wavenumber(k, kz)
    idx = np.nonzero(valid)[0]
    if idx.size == 0 or k.size < 2:
        return np.zeros(0), np.zeros(0, dtype=np.complex128)
    f0, f1 = int(idx[0]), int(idx[-1])       # k_L grows with k: the propagating samples are contiguous
    m_lo = math.ceil(kl[f0] / dkl - EDGE_SLACK)
    m_hi = math.floor(kl[f1] / dkl + EDGE_SLACK)
    if m_hi < m_lo:
        return np.zeros(0), np.zeros(0, dtype=np.complex128)
    dk = (k[-1] - k[0]) / (k.size - 1)
    a = s_row * np.exp(1j * kl * l_ref)      # demodulated spectrum
    n_pts = min(4, f1 - f0 + 1)
    klm = dkl * np.arange(m_lo, m_hi + 1, dtype=np.float64)
    Q = np.zeros(klm.size, dtype=np.complex128)
    for i, kL in enumerate(klm):
        km = math.sqrt(kL * kL + 0.25 * kz * kz)
        t = (km - k[0]) / dk
        start = min(max(int(math.floor(t)) - 1, f0), f1 - n_pts + 1)
        nodes = np.arange(start, start + n_pts)
        v = lagrange_weights(t, nodes) @ a[nodes]
        Q[i] = v * np.exp(-1j * kL * l_ref) * kL * (dkl / dk)
    return klm, Q


def path_lengths(arr, px, py):
    """L[c, p] = rho_T + rho_R (monostatic: 2 rho)."""
    L = range_of(arr, px, py)
    return 2.0 * L if arr.mode == "mono" else L


def reference_lengths(arr, grid):
    """Path length from each channel to the centre of the image grid."""
    cx = grid.x0 + 0.5 * (grid.nx - 1) * grid.dx
    cy = grid.y0 + 0.5 * (grid.ny - 1) * grid.dy
    return path_lengths(arr, np.array([cx]), np.array([cy]))[:, 0]


def spectrum_at(arr, S, kappas, px, py, dkl, l_ref):
    """G[kappa, p] = sum_c sum_m Q_m(c, kappa) exp(j k_L,m L_c(p))."""
    kz = kz_grid(arr.z_scan.size, arr.scan_step)
    L = path_lengths(arr, px, py)
    out = np.zeros((len(kappas), L.shape[1]), dtype=np.complex128)
    for i, kap in enumerate(kappas):
        for c in range(L.shape[0]):
            klm, Q = uniform_samples(arr.k, kz[kap], S[c, kap, :], dkl, l_ref[c])
            if klm.size:
                out[i] += np.exp(1j * np.outer(L[c], klm)) @ Q
    return out


def spectrum(arr, grid, echo, dkl, kappas=None):
    """G[kappa][y][x] of the omega-K variant for the listed (default: all) k_z indices."""
    S = scan_spectrum(echo)
    kappas = list(range(arr.z_scan.size) if kappas is None else kappas)
    px, py = pixel_grid(grid)
    G = spectrum_at(arr, S, kappas, px, py, dkl, reference_lengths(arr, grid))
    return G.reshape(len(kappas), grid.ny, grid.nx)


def image(arr, grid, echo, dkl):
    """g[z][y][x]: inverse FFT over k_z (eq. 9) of the omega-K spectrum."""
    return np.fft.ifft(spectrum(arr, grid, echo, dkl), axis=0)
