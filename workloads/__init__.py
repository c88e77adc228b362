"""Seeded synthetic workloads for polyline-array imaging.

This module describes the problem instances (array, scan, frequency sweep,
image grid, scatterer scene) and draws the random numbers they need.  It holds
none of the reconstruction arithmetic: both the FP64 oracle and the GPU
library read the descriptions and arrays produced here, and nothing else is
shared between them.

The paper's own scenes (point targets of its Figs. 3-7, the FEKO model, the
measured knife data) are not available, so these seeded scenes stand in for
them, with the shapes and sizes of the workloads the build is measured on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

SPEED_OF_LIGHT = 299_792_458.0  # m/s (exact, SI definition)


@dataclass(frozen=True)
class ArrayDesc:
    """A polyline array: ``n_chords`` equal chords inscribed in a circle.

    mode        "mono" (transceivers) or "multi" (Tx at chord ends, Rx spread).
    radius      circumscribed-circle radius R_0 in metres.
    n_elem      transceivers per chord (mono) or receivers per chord (multi).
    spacing     element (mono) or receiver (multi) spacing along a chord, m.
    n_tx        transmitters per chord (multi only).
    tx_offsets  chord-local Tx offsets from the chord midpoint, metres, or None
                for the default placement (two at each chord end).
    arc_center  angle of the middle of the arc, radians (-pi/2: the array sits
                below the origin and looks toward +y).
    n_scan, scan_step, scan_z0   scan positions z'_m = scan_z0 + m*scan_step.
    n_freq, f_start, f_stop      inclusive uniform frequency sweep, Hz.
    """

    mode: str
    n_chords: int
    radius: float
    n_elem: int
    spacing: float
    n_scan: int
    scan_step: float
    n_freq: int
    f_start: float
    f_stop: float
    n_tx: int = 0
    tx_offsets: Optional[Tuple[float, ...]] = None
    arc_center: float = -math.pi / 2
    scan_z0: Optional[float] = None  # None: centred scan

    @property
    def z0(self) -> float:
        if self.scan_z0 is not None:
            return float(self.scan_z0)
        return -(self.n_scan - 1) * self.scan_step / 2.0

    @property
    def n_channels(self) -> int:
        if self.mode == "mono":
            return self.n_chords * self.n_elem
        return self.n_chords * self.n_tx * self.n_elem


@dataclass(frozen=True)
class ImageGrid:
    """Horizontal pixel grid; pixel (ix, iy) is centred at (x0+ix*dx, y0+iy*dy).

    The image's z axis is the scan grid of the array (one plane per scan
    position).
    """

    nx: int
    ny: int
    x0: float
    y0: float
    dx: float
    dy: float

    @staticmethod
    def centred(n: int, extent: float) -> "ImageGrid":
        d = extent / n
        c = -extent / 2 + d / 2
        return ImageGrid(n, n, c, c, d, d)


@dataclass(frozen=True)
class Scene:
    """Point-scatterer scene recipe.

    kind "box": uniform in a box of the given half-sizes with a minimum
    separation; kind "shell": on an ellipsoid surface with the given
    semi-axes (Gaussian direction, normalised, then scaled).
    """

    n: int
    kind: str
    half: Tuple[float, float, float]
    seed: int
    min_sep: float = 0.0
    z_limit: Optional[float] = None  # box only: |z| <= z_limit


@dataclass(frozen=True)
class Workload:
    name: str
    array: ArrayDesc
    grid: ImageGrid
    scene: Scene
    noise_db: Optional[float] = None  # echo SNR, None = noise free
    echo_dtype: str = "complex64"


def lambda_min(f_stop: float) -> float:
    return SPEED_OF_LIGHT / f_stop


# ---------------------------------------------------------------------------
# The workloads.  Element spacings follow the half-wavelength rule at the top
# of the band for transceivers and one wavelength for multistatic receivers
# (the monostatic spacing is half of the multistatic one).
# ---------------------------------------------------------------------------
_D_MONO = SPEED_OF_LIGHT / (2 * 34e9)   # 4.408 mm
_D_MULTI = SPEED_OF_LIGHT / 34e9        # 8.817 mm

C1 = Workload(
    name="mono-3x16-24z-16f-32x32",
    array=ArrayDesc(mode="mono", n_chords=3, radius=0.5, n_elem=16, spacing=_D_MONO,
                    n_scan=24, scan_step=0.005, n_freq=16, f_start=26e9, f_stop=34e9),
    grid=ImageGrid.centred(32, 0.30),
    scene=Scene(n=5, kind="box", half=(0.15, 0.15, 0.06), seed=1, min_sep=0.05, z_limit=0.048),
    noise_db=-30.0,
    echo_dtype="complex128",
)

C2 = Workload(
    name="mono-5x64-256z-64f-200x200",
    array=ArrayDesc(mode="mono", n_chords=5, radius=0.6, n_elem=64, spacing=_D_MONO,
                    n_scan=256, scan_step=0.004, n_freq=64, f_start=26e9, f_stop=34e9),
    grid=ImageGrid.centred(200, 0.60),
    scene=Scene(n=2000, kind="shell", half=(0.25, 0.20, 0.50), seed=2),
)

C3 = Workload(
    name="multi-7x(4tx,32rx)-512z-128f-256x256",
    array=ArrayDesc(mode="multi", n_chords=7, radius=0.8, n_elem=32, spacing=_D_MULTI, n_tx=4,
                    n_scan=512, scan_step=0.003, n_freq=128, f_start=26e9, f_stop=34e9),
    grid=ImageGrid.centred(256, 0.60),
    scene=Scene(n=5000, kind="shell", half=(0.25, 0.20, 0.50), seed=3),
)

WORKLOADS = {"C1": C1, "C2": C2, "C3": C3}

def batch_c5(n_scans: int = 16, first_seed: int = 50):
    """The uneven batch: monostatic scans on R = 0.6 m with 4.408 mm elements
    and 4 mm scan steps, each with its own chord count (3-7), elements per
    chord (32-64), scan length (any integer in 128-512) and frequency count
    (32-128, 26-34 GHz), drawn from numpy's default_rng(seed) for seeds
    first_seed, first_seed + 1, ...; 1000 shell scatterers with the z
    semi-axis 0.45 x the scan length; images 128 x 128 over 0.60 m."""
    out = []
    for seed in range(first_seed, first_seed + n_scans):
        rng = np.random.default_rng(seed)
        n_chords = int(rng.integers(3, 8))
        n_elem = int(rng.integers(32, 65))
        n_scan = int(rng.integers(128, 513))
        n_freq = int(rng.integers(32, 129))
        arr = ArrayDesc(mode="mono", n_chords=n_chords, radius=0.6, n_elem=n_elem, spacing=_D_MONO,
                        n_scan=n_scan, scan_step=0.004, n_freq=n_freq, f_start=26e9, f_stop=34e9)
        scene = Scene(n=1000, kind="shell", half=(0.25, 0.20, 0.45 * n_scan * 0.004), seed=seed)
        out.append(Workload(name=f"c5-{seed}-{n_chords}x{n_elem}-{n_scan}z-{n_freq}f-128x128", array=arr,
                            grid=ImageGrid.centred(128, 0.60), scene=scene))
    return out


# ---------------------------------------------------------------------------
# Seeded random draws
# ---------------------------------------------------------------------------
def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """Unit-variance circular complex Gaussian samples, CN(0, 1)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def scatterers(scene: Scene) -> Tuple[np.ndarray, np.ndarray]:
    """Positions (n, 3) float64 in metres and reflectivities (n,) complex128."""
    rng = np.random.default_rng(scene.seed)
    hx, hy, hz = scene.half
    if scene.kind == "box":
        zl = hz if scene.z_limit is None else min(hz, scene.z_limit)
        pts = []
        tries = 0
        while len(pts) < scene.n:
            tries += 1
            if tries > 100000:
                raise RuntimeError("could not place scatterers with the requested separation")
            p = np.array([rng.uniform(-hx, hx), rng.uniform(-hy, hy), rng.uniform(-zl, zl)])
            if all(np.linalg.norm(p - q) >= scene.min_sep for q in pts):
                pts.append(p)
        pos = np.array(pts)
    elif scene.kind == "shell":
        v = rng.standard_normal((scene.n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        pos = v * np.array([hx, hy, hz])[None, :]
    else:
        raise ValueError(scene.kind)
    refl = complex_normal(rng, scene.n)
    return pos.astype(np.float64), refl.astype(np.complex128)


def noise(shape, seed: int) -> np.ndarray:
    """Unit-variance complex white Gaussian noise (to be scaled by the caller)."""
    return complex_normal(np.random.default_rng(seed + 1_000_003), shape)


def random_echo(array: ArrayDesc, seed: int, dtype=np.complex64) -> np.ndarray:
    """A CN(0,1) echo cube s[c][m][f] for operator-level parity checks."""
    rng = np.random.default_rng(seed)
    return complex_normal(rng, (array.n_channels, array.n_scan, array.n_freq)).astype(dtype)


def random_subset(n_total: int, n_pick: int, seed: int) -> np.ndarray:
    """Sorted distinct indices in [0, n_total)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=min(n_pick, n_total), replace=False))


def tiny(mode: str = "mono", **kw) -> Workload:
    """A very small workload for fast CPU pins and ragged-size GPU checks."""
    if mode == "mono":
        arr = ArrayDesc(mode="mono", n_chords=2, radius=0.4, n_elem=6, spacing=_D_MONO,
                        n_scan=10, scan_step=0.006, n_freq=8, f_start=26e9, f_stop=34e9)
    else:
        arr = ArrayDesc(mode="multi", n_chords=2, radius=0.4, n_elem=5, spacing=_D_MULTI, n_tx=4,
                        n_scan=10, scan_step=0.006, n_freq=8, f_start=26e9, f_stop=34e9)
    arr = replace(arr, **{k: v for k, v in kw.items() if k in ArrayDesc.__dataclass_fields__})
    grid = kw.get("grid", ImageGrid.centred(9, 0.2))
    return Workload(name=f"tiny-{mode}", array=arr, grid=grid,
                    scene=Scene(n=3, kind="box", half=(0.08, 0.08, 0.02), seed=7, min_sep=0.03))
