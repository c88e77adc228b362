"""Brute-force back-projection, the paper's comparison method (Sec. III, Table 2).

Test infrastructure: see the package header.

The paper never writes the BP formula.  Reading used here: the matched
filter of the echo models (1)/(10) with the same weight k as the hybrid
method's measure k dk, summed over the full aperture with no beam limiting:

  g_BP(x, y, z) = sum_c sum_m' sum_f k_f s[c, m', f] exp(+j k_f (R_T + R_R))

with R_T, R_R the 3-D distances from the channel's Tx and Rx at scan height
z'_m' to the voxel (R_T = R_R for monostatic channels, i.e. exp(+j 2 k R)).
Voxel z coordinates are the scan grid.
"""
from __future__ import annotations

import numpy as np


def bp_voxels(arr, echo, vx, vy, vz, chunk=512):
    """Back-projected values at voxel coordinates (parallel 1-D arrays)."""
    echo = np.asarray(echo, dtype=np.complex128)
    vx, vy, vz = (np.asarray(a, dtype=np.float64) for a in (vx, vy, vz))
    w = echo * arr.k[None, None, :]                 # k_f s[c, m', f]
    out = np.zeros(vx.size, dtype=np.complex128)
    for v0 in range(0, vx.size, chunk):
        sl = slice(v0, v0 + chunk)
        dz = vz[sl][None, :] - arr.z_scan[:, None]                  # (n_scan, V)
        for c in range(arr.n_channels):
            rt = np.sqrt((vx[sl] - arr.tx[c, 0]) ** 2 + (vy[sl] - arr.tx[c, 1]) ** 2 + dz ** 2)
            rr = np.sqrt((vx[sl] - arr.rx[c, 0]) ** 2 + (vy[sl] - arr.rx[c, 1]) ** 2 + dz ** 2)
            path = rt + rr                                            # (n_scan, V)
            ph = np.exp(1j * arr.k[None, :, None] * path[:, None, :])  # (n_scan, n_f, V)
            out[sl] += np.einsum("mf,mfv->v", w[c], ph)
    return out


def bp_image(arr, grid, echo, z_index=None):
    """g_BP[z][y][x] over the pixel grid and the listed scan planes (default all)."""
    zi = np.arange(arr.z_scan.size) if z_index is None else np.asarray(z_index)
    x = grid.x0 + grid.dx * np.arange(grid.nx)
    y = grid.y0 + grid.dy * np.arange(grid.ny)
    zz, yy, xx = np.meshgrid(arr.z_scan[zi], y, x, indexing="ij")
    vals = bp_voxels(arr, echo, xx.ravel(), yy.ravel(), zz.ravel())
    return vals.reshape(zi.size, grid.ny, grid.nx)
