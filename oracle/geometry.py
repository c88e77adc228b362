"""Polyline array geometry (Sec. II-A and II-B, Fig. 1, Table 1).

Test infrastructure: see the package header.

Reading of the paper's geometry (it is given only in words and a figure):
  * The array is ``n_chords`` chords of equal length L inscribed in a circle of
    radius R_0; adjacent chords share their end points (the "joints").
  * Elements are evenly spaced along each chord: L = N * d and element j sits
    at offset (j + 1/2) d - L/2 from the chord midpoint along the chord.
  * Multistatic arrays place the (undersampled) transmitters at the chord ends
    (Sec. II-B; Sec. II-C "at the joints and ends"); by default two per end at
    offsets -L/2, -L/2 + d/2, L/2 - d/2, L/2.  Channels are all Tx-Rx pairs
    within one chord (the restriction used in Sec. III's experiment).
  * All antennas share the scan height z' (Fig. 1: mechanical scan along the
    axis perpendicular to the array plane).
  * Frequencies are an inclusive uniform sweep (Table 1: 51 steps over
    30-35 GHz); k = 2 pi f / c.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SPEED_OF_LIGHT = 299_792_458.0


@dataclass
class Array:
    mode: str
    chord_ends: np.ndarray   # (n_chords, 2, 2): start and end point (x, y) of each chord
    elements: np.ndarray     # (n_chords, n_elem, 2): element (mono) / receiver (multi) xy
    tx_elements: np.ndarray  # (n_chords, n_tx, 2): multistatic transmitters (empty for mono)
    tx: np.ndarray           # (n_ch, 2): transmit phase centre of each channel
    rx: np.ndarray           # (n_ch, 2): receive phase centre of each channel
    chord_of_channel: np.ndarray  # (n_ch,)
    z_scan: np.ndarray       # (n_scan,) scan heights z'_m
    freq: np.ndarray         # (n_freq,) Hz
    k: np.ndarray            # (n_freq,) wavenumbers 2 pi f / c

    @property
    def n_channels(self) -> int:
        return self.tx.shape[0]

    @property
    def scan_step(self) -> float:
        return float(self.z_scan[1] - self.z_scan[0]) if self.z_scan.size > 1 else 0.0


def chord_angle(radius: float, length: float) -> float:
    """Central angle subtended by a chord of the given length."""
    if not (0.0 < length < 2.0 * radius):
        raise ValueError("chord length must lie in (0, 2R)")
    return 2.0 * math.asin(length / (2.0 * radius))


def build(desc) -> Array:
    """Build the array from a ``workloads.ArrayDesc``."""
    R = float(desc.radius)
    n_c = int(desc.n_chords)
    n_e = int(desc.n_elem)
    d = float(desc.spacing)
    L = n_e * d
    alpha = chord_angle(R, L)

    ends = np.zeros((n_c, 2, 2))
    elems = np.zeros((n_c, n_e, 2))
    if desc.mode == "multi":
        if desc.tx_offsets is not None:
            tx_off = np.asarray(desc.tx_offsets, dtype=np.float64)
        elif desc.n_tx == 4:
            tx_off = np.array([-L / 2, -L / 2 + d / 2, L / 2 - d / 2, L / 2])
        elif desc.n_tx == 2:
            tx_off = np.array([-L / 2, L / 2])
        else:
            raise ValueError("default Tx placement exists for 2 or 4 Tx per chord")
        if tx_off.size != desc.n_tx:
            raise ValueError("tx_offsets length must equal n_tx")
    else:
        tx_off = np.zeros(0)
    txe = np.zeros((n_c, tx_off.size, 2))

    for i in range(n_c):
        phi = desc.arc_center + (i - (n_c - 1) / 2.0) * alpha
        a = R * np.array([math.cos(phi - alpha / 2), math.sin(phi - alpha / 2)])
        b = R * np.array([math.cos(phi + alpha / 2), math.sin(phi + alpha / 2)])
        ends[i, 0], ends[i, 1] = a, b
        mid = 0.5 * (a + b)
        t = (b - a) / np.linalg.norm(b - a)
        for j in range(n_e):
            elems[i, j] = mid + ((j + 0.5) * d - L / 2) * t
        for j, u in enumerate(tx_off):
            txe[i, j] = mid + u * t

    if desc.mode == "mono":
        tx = elems.reshape(-1, 2).copy()
        rx = tx.copy()
        chord = np.repeat(np.arange(n_c), n_e)
    elif desc.mode == "multi":
        tx_l, rx_l, ch_l = [], [], []
        for i in range(n_c):
            for t_i in range(tx_off.size):
                for r_i in range(n_e):
                    tx_l.append(txe[i, t_i])
                    rx_l.append(elems[i, r_i])
                    ch_l.append(i)
        tx, rx, chord = np.array(tx_l), np.array(rx_l), np.array(ch_l)
    else:
        raise ValueError(desc.mode)

    z = desc.z0 + desc.scan_step * np.arange(desc.n_scan, dtype=np.float64)
    f = np.linspace(desc.f_start, desc.f_stop, desc.n_freq)
    k = 2.0 * math.pi * f / SPEED_OF_LIGHT
    return Array(mode=desc.mode, chord_ends=ends, elements=elems, tx_elements=txe, tx=tx, rx=rx,
                 chord_of_channel=chord, z_scan=z, freq=f, k=k)


def pixel_centres(grid):
    """Pixel centre coordinates: x (nx,), y (ny,)."""
    x = grid.x0 + grid.dx * np.arange(grid.nx, dtype=np.float64)
    y = grid.y0 + grid.dy * np.arange(grid.ny, dtype=np.float64)
    return x, y
