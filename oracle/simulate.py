"""Point-scatterer echo model, eq. (1) (monostatic) and eqs. (10)-(11) (multistatic).

Test infrastructure: see the package header.

For point scatterers g(r) = sum_p sigma_p delta(r - r_p) the integrals of
eqs. (1) and (10) become sums.  Monostatic echoes carry the round-trip phase
exp(-j 2 k R); multistatic ones exp(-j k (R_T + R_R)).  A monostatic channel
is a multistatic one with coinciding Tx and Rx, so both are written as
exp(-j k (R_T + R_R)) with R_T = R_R in the monostatic case.  As in the paper
there is no amplitude decay and no antenna pattern.
"""
from __future__ import annotations

import numpy as np


def distances(tx_xy, rx_xy, z_scan, pos):
    """R_T and R_R for one channel: arrays (n_scan, n_scat)."""
    dzt = pos[None, :, 2] - z_scan[:, None]
    rt = np.sqrt((pos[None, :, 0] - tx_xy[0]) ** 2 + (pos[None, :, 1] - tx_xy[1]) ** 2 + dzt ** 2)
    rr = np.sqrt((pos[None, :, 0] - rx_xy[0]) ** 2 + (pos[None, :, 1] - rx_xy[1]) ** 2 + dzt ** 2)
    return rt, rr


def echo(arr, pos, refl, channels=None, chunk=256):
    """s[c][m][f] = sum_p sigma_p exp(-j k_f (R_T + R_R)), complex128.

    ``channels`` optionally restricts the output to a subset of channel
    indices (the result then has len(channels) rows).
    """
    pos = np.asarray(pos, dtype=np.float64)
    refl = np.asarray(refl, dtype=np.complex128)
    chans = np.arange(arr.n_channels) if channels is None else np.asarray(channels)
    out = np.zeros((chans.size, arr.z_scan.size, arr.k.size), dtype=np.complex128)
    for oi, c in enumerate(chans):
        for s0 in range(0, pos.shape[0], chunk):
            p = pos[s0:s0 + chunk]
            rt, rr = distances(arr.tx[c], arr.rx[c], arr.z_scan, p)
            path = rt + rr                                   # (n_scan, n_s)
            ph = np.exp(-1j * arr.k[None, :, None] * path[:, None, :])  # (n_scan, n_f, n_s)
            out[oi] += ph @ refl[s0:s0 + chunk]
    return out


def echo_samples(arr, pos, refl, c_idx, m_idx, f_idx):
    """Individual samples s[c_i, m_i, f_i] for parallel index arrays."""
    pos = np.asarray(pos, dtype=np.float64)
    refl = np.asarray(refl, dtype=np.complex128)
    c_idx, m_idx, f_idx = (np.asarray(a) for a in (c_idx, m_idx, f_idx))
    out = np.zeros(c_idx.size, dtype=np.complex128)
    for i in range(c_idx.size):
        c, m, f = c_idx[i], m_idx[i], f_idx[i]
        dz = pos[:, 2] - arr.z_scan[m]
        rt = np.sqrt((pos[:, 0] - arr.tx[c, 0]) ** 2 + (pos[:, 1] - arr.tx[c, 1]) ** 2 + dz ** 2)
        rr = np.sqrt((pos[:, 0] - arr.rx[c, 0]) ** 2 + (pos[:, 1] - arr.rx[c, 1]) ** 2 + dz ** 2)
        out[i] = np.sum(refl * np.exp(-1j * arr.k[f] * (rt + rr)))
    return out


def add_noise(s, snr_db, unit_noise):
    """Add white noise with power 10^(snr_db/10) * mean|s|^2 (snr_db < 0)."""
    p = np.mean(np.abs(s) ** 2)
    return s + np.sqrt(p * 10.0 ** (snr_db / 10.0)) * unit_noise
