"""Direct nonuniform DFT: the range-compression sum of eqs. (8a)/(19a).

Test infrastructure: see the package header.

For one channel and one k_z, eq. (8a) is q(l) = sum_f a_f exp(+j k'_f l) with
k'_f = k_rho(f) - k_rho0 nonuniform in f.  The paper evaluates it with an
inverse NUFFT on a uniform l grid; this is the exact sum it approximates.
"""
from __future__ import annotations

import numpy as np


def nudft(strengths, kprime, l):
    """q[i] = sum_f strengths[f] exp(+j kprime[f] l[i])."""
    a = np.asarray(strengths, dtype=np.complex128)
    kp = np.asarray(kprime, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    return np.exp(1j * np.outer(l, kp)) @ a


def range_profiles(arr, S, kappa, k_ref, l_grid):
    """q[c, i] of eq. (8a)/(19a) on per-channel l grids for one k_z index.

    ``l_grid`` is (n_ch, n_l); ``k_ref`` is the reference wavenumber k_rho0.
    Strengths are k_f S[c, kappa, f] (weight k dk -> k_f), evanescent terms
    dropped.
    """
    from .hybrid import dispersion, kz_grid

    kz = kz_grid(arr.z_scan.size, arr.scan_step)[kappa]
    krho, valid = dispersion(arr.mode, arr.k, kz)
    a = S[:, kappa, :] * (arr.k * valid)[None, :]
    return np.stack([nudft(a[c], krho - k_ref, l_grid[c]) for c in range(a.shape[0])])
