"""Hybrid time-domain / spatial-frequency inversion, exact discrete form.

Test infrastructure: see the package header.

Monostatic chain (Sec. II-A):
  (2)  Fourier transform of the echo over the scan coordinate z'.
  (3)-(5)  the transform of the round-trip Green's function is
       exp(-j k_rho rho) exp(-j k_z z) with rho the horizontal antenna-pixel
       distance and k_rho = sqrt(4k^2 - k_z^2).
  (7)  g(x, y, k_z) = integral of s(x', y', k_z, k) exp(+j k_rho rho) k dk dx'dy'.
  (8a)/(8b) split (7) into a 1-D transform over k to a range axis l followed
       by an element sum of q evaluated at l = rho times exp(+j k_rho0 rho).
       Because q(rho) exp(j k_rho0 rho) equals the k-sum of (7) exactly, the
       reference wavenumber k_rho0 cancels; the NUFFT and the interpolation of
       (8a)/(8b) are numerical devices that approximate (7).
  (9)  image = inverse FFT over k_z.
Multistatic chain (Sec. II-B): the same with (18) k_rho = sqrt(k^2 - k_z^2/4)
and the range l = rho_T + rho_R of (17)/(19b).

This module evaluates (7)/(19) by direct summation over channels and
frequencies -- the plain definition the fast method approximates.

Readings of the paper used here:
  * The transform over z' uses exp(-j k_z z') (consistent with (3) after
    stationary phase) with numpy's unnormalised FFT; k_z = 2 pi fftfreq.  The
    final transform over k_z is numpy's ifft (with 1/N).  The image z axis is
    then the scan grid: the offset of the scan origin cancels between the two
    transforms.
  * The measure "k dk" becomes the weight k_f; the constant dk is dropped.
    Parity unpinned for this factor: no value the paper prints or closed
    form it gives fixes the weight (leaving it out tapers the image's
    amplitude smoothly in range and moves no peak), so only the GPU parity
    tests tie the GPU's weight to this one.
  * Amplitude and constant-phase factors of the stationary-phase results are
    omitted (the paper omits them), so the image scale is fixed by the weight.
  * Evanescent terms (k_rho^2 < 0) are dropped.
"""
from __future__ import annotations

import numpy as np


def scan_spectrum(echo):
    """S[c, kappa, f] = sum_m s[c, m, f] exp(-j 2 pi kappa m / N_z)  (eqs. 2, 12)."""
    return np.fft.fft(np.asarray(echo, dtype=np.complex128), axis=1)


def kz_grid(n_scan, scan_step):
    """Spatial frequencies of the scan axis in rad/m, numpy FFT order.  A
    single scan position has the one frequency k_z = 0 (a DFT of length 1),
    whatever the step."""
    if n_scan == 1:
        return np.zeros(1)
    return 2.0 * np.pi * np.fft.fftfreq(n_scan, d=scan_step)


def dispersion(mode, k, kz):
    """k_rho(k, k_z) and a mask of propagating terms.

    mono:  k_rho = sqrt(4 k^2 - k_z^2)      (eq. 5)
    multi: k_rho = sqrt(k^2 - k_z^2 / 4)    (eq. 18)
    """
    k = np.asarray(k, dtype=np.float64)
    if mode == "mono":
        arg = 4.0 * k * k - kz * kz
    elif mode == "multi":
        arg = k * k - kz * kz / 4.0
    else:
        raise ValueError(mode)
    valid = arg > 0.0
    return np.sqrt(np.where(valid, arg, 0.0)), valid


def range_of(arr, px, py):
    """l[c, p]: rho (mono, eq. 4) or rho_T + rho_R (multi, eqs. 11a/11b)."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    if arr.mode == "mono":
        return np.hypot(px[None, :] - arr.tx[:, 0:1], py[None, :] - arr.tx[:, 1:2])
    rho_t = np.hypot(px[None, :] - arr.tx[:, 0:1], py[None, :] - arr.tx[:, 1:2])
    rho_r = np.hypot(px[None, :] - arr.rx[:, 0:1], py[None, :] - arr.rx[:, 1:2])
    return rho_t + rho_r


def spectrum_at(arr, S, kappas, px, py):
    """G[kappa, p] = sum_c sum_f k_f S[c,kappa,f] exp(+j k_rho(f,kappa) l_c(p)).

    Eq. (7) (monostatic) / (19a)+(19b) (multistatic) with exact sums, for the
    listed k_z indices and pixel coordinates (arrays of equal length).
    """
    kz = kz_grid(arr.z_scan.size, arr.scan_step)
    l = range_of(arr, px, py)                      # (n_ch, P)
    out = np.zeros((len(kappas), l.shape[1]), dtype=np.complex128)
    for i, kap in enumerate(kappas):
        krho, valid = dispersion(arr.mode, arr.k, kz[kap])
        a = S[:, kap, :] * (arr.k * valid)[None, :]  # weight k dk -> k_f
        for c in range(l.shape[0]):
            out[i] += np.exp(1j * np.outer(l[c], krho)) @ a[c]
    return out


def pixel_grid(grid):
    x = grid.x0 + grid.dx * np.arange(grid.nx)
    y = grid.y0 + grid.dy * np.arange(grid.ny)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    return xx.ravel(), yy.ravel()


def spectrum(arr, grid, echo, kappas=None):
    """G[kappa][y][x] for all pixels and the listed (default: all) k_z indices."""
    S = scan_spectrum(echo)
    kappas = range(arr.z_scan.size) if kappas is None else kappas
    px, py = pixel_grid(grid)
    G = spectrum_at(arr, S, list(kappas), px, py)
    return G.reshape(len(G), grid.ny, grid.nx)


def image(arr, grid, echo):
    """g[z][y][x]: inverse FFT over k_z of the full spectrum (eq. 9)."""
    return np.fft.ifft(spectrum(arr, grid, echo), axis=0)


def image_adjoint(arr, grid, g):
    """Adjoint of `image`: the echo-shaped s~[c][m][f] with
    <image(s), g> = <s, image_adjoint(g)> for every echo s and image g.

    `image` is s -> S = fft over m (unnormalised) -> G[kappa, p] =
    sum_c sum_f k_f S[c,kappa,f] exp(+j k_rho l_c(p)) -> g = ifft over kappa.
    Its adjoint takes the steps in reverse with conjugate phases: the adjoint
    of numpy's ifft (1/N sum exp(+j..)) is fft / N, the adjoint of the
    element-and-frequency sum is S~[c,kappa,f] = k_f sum_p exp(-j k_rho l_c(p))
    G~[kappa,p] (evanescent terms dropped as in the forward), and the adjoint
    of the unnormalised fft is N ifft.  Used as the echo model of the
    least-squares refinement (the forward model taken as the adjoint of the
    imaging operator).
    """
    n_z = arr.z_scan.size
    px, py = pixel_grid(grid)
    g = np.asarray(g, dtype=np.complex128).reshape(n_z, px.size)
    Gt = np.fft.fft(g, axis=0) / n_z
    kz = kz_grid(n_z, arr.scan_step)
    l = range_of(arr, px, py)                      # (n_ch, P)
    St = np.zeros((l.shape[0], n_z, arr.k.size), dtype=np.complex128)
    for kap in range(n_z):
        krho, valid = dispersion(arr.mode, arr.k, kz[kap])
        w = arr.k * valid
        for c in range(l.shape[0]):
            St[c, kap, :] = w * (np.exp(-1j * np.outer(krho, l[c])) @ Gt[kap])
    return np.fft.ifft(St, axis=1) * n_z
