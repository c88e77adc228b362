"""Pins of the oracle's echo simulator, eqs. (1) and (10)-(11)."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import geometry, simulate

C = W.SPEED_OF_LIGHT


def _arr(mode="mono", **kw):
    return geometry.build(W.tiny(mode, **kw).array)


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_single_scatterer_unit_magnitude_and_range_profile(mode):
    # dense sweep: unambiguous range c / df well beyond the round trip
    arr = _arr(mode, n_freq=401)
    pos = np.array([[0.031, 0.012, 0.004]])
    s = simulate.echo(arr, pos, np.array([1.0 + 0.0j]))
    assert np.allclose(np.abs(s), 1.0, atol=1e-12)
    # range compression by an inverse DFT over frequency: exp(-j k D) must
    # focus at the positive delay D / c (a sign error would mirror it)
    df = arr.freq[1] - arr.freq[0]
    pad = 64
    nfft = arr.freq.size * pad
    for c in (0, arr.n_channels - 1):
        for m in (0, arr.z_scan.size - 1):
            h = np.fft.ifft(s[c, m], n=nfft)
            tau = np.argmax(np.abs(h)) / (nfft * df)
            dz = pos[0, 2] - arr.z_scan[m]
            d_t = np.sqrt(np.sum((pos[0, :2] - arr.tx[c]) ** 2) + dz * dz)
            d_r = np.sqrt(np.sum((pos[0, :2] - arr.rx[c]) ** 2) + dz * dz)
            assert abs(tau * C - (d_t + d_r)) < 1.5 * C / (nfft * df)


def test_linearity_in_reflectivity():
    arr = _arr()
    pos, refl = W.scatterers(W.tiny().scene)
    rng = np.random.default_rng(0)
    r2 = W.complex_normal(rng, refl.size)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    lhs = simulate.echo(arr, pos, a * refl + b * r2)
    rhs = a * simulate.echo(arr, pos, refl) + b * simulate.echo(arr, pos, r2)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    # superposition over scatterers
    parts = sum(simulate.echo(arr, pos[i:i + 1], refl[i:i + 1]) for i in range(len(refl)))
    assert np.allclose(parts, simulate.echo(arr, pos, refl), atol=1e-12)


@pytest.mark.parametrize("mode", ["mono", "multi"])
def test_mirror_channels_see_identical_echo(mode):
    arr = _arr(mode)
    pos = np.array([[0.0, 0.05, 0.01], [0.0, -0.03, -0.02]])
    s = simulate.echo(arr, pos, np.array([1.0, 0.5 - 0.5j]))
    # mirror channel: chord i -> N-1-i; element j -> n-1-j; Tx order reversed
    a = W.tiny(mode).array
    n_c, n_e = a.n_chords, a.n_elem
    if mode == "mono":
        perm = [(n_c - 1 - c // n_e) * n_e + (n_e - 1 - c % n_e) for c in range(arr.n_channels)]
    else:
        n_t = a.n_tx
        perm = []
        for c in range(arr.n_channels):
            i, t, r = c // (n_t * n_e), (c // n_e) % n_t, c % n_e
            perm.append(((n_c - 1 - i) * n_t + (n_t - 1 - t)) * n_e + (n_e - 1 - r))
    assert np.allclose(arr.tx[perm] * [-1, 1], arr.tx, atol=1e-12)
    assert np.allclose(s[perm], s, atol=1e-10)


def test_scan_shift_moves_echo_by_one_sample():
    arr = _arr()
    pos = np.array([[0.02, 0.03, 0.0]])
    s0 = simulate.echo(arr, pos, np.ones(1))
    s1 = simulate.echo(arr, pos + [0, 0, arr.scan_step], np.ones(1))
    assert np.allclose(s1[:, 1:], s0[:, :-1], atol=1e-10)
    assert not np.allclose(s1, s0)


def test_multistatic_reciprocity_and_monostatic_limit():
    arr = _arr("multi")
    pos, refl = W.scatterers(W.tiny().scene)
    s = simulate.echo(arr, pos, refl)
    swapped = replace(arr, tx=arr.rx.copy(), rx=arr.tx.copy())
    assert np.allclose(simulate.echo(swapped, pos, refl), s, atol=1e-10)
    # a multistatic channel whose Tx and Rx coincide is a monostatic channel
    mono = _arr("mono")
    as_multi = replace(mono, mode="multi")
    assert np.allclose(simulate.echo(as_multi, pos, refl), simulate.echo(mono, pos, refl), atol=1e-12)


def test_sample_evaluator_matches_cube():
    arr = _arr("multi")
    pos, refl = W.scatterers(W.tiny().scene)
    s = simulate.echo(arr, pos, refl)
    rng = np.random.default_rng(3)
    ci = rng.integers(0, arr.n_channels, 20)
    mi = rng.integers(0, arr.z_scan.size, 20)
    fi = rng.integers(0, arr.k.size, 20)
    assert np.allclose(simulate.echo_samples(arr, pos, refl, ci, mi, fi), s[ci, mi, fi], atol=1e-12)


def test_noise_level():
    s = W.random_echo(W.C1.array, seed=5, dtype=np.complex128)
    n = W.noise(s.shape, seed=5)
    noisy = simulate.add_noise(s, -30.0, n)
    ratio = np.mean(np.abs(noisy - s) ** 2) / np.mean(np.abs(s) ** 2)
    assert abs(10 * np.log10(ratio) + 30.0) < 0.3
