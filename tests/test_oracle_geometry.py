"""Pins of the oracle's array geometry against invariants of the polyline
construction (Sec. II-A/B) and the printed parameters of Table 1."""
import json
import math
import os
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import geometry

pytestmark = pytest.mark.parametrize("wl", [W.C1, W.C2, W.C3], ids=["C1", "C2", "C3"])


def test_chord_ends_on_circle_equal_and_joined(wl):
    arr = geometry.build(wl.array)
    R = wl.array.radius
    ends = arr.chord_ends
    assert np.allclose(np.linalg.norm(ends, axis=-1), R, rtol=0, atol=1e-12)
    lengths = np.linalg.norm(ends[:, 1] - ends[:, 0], axis=-1)
    assert np.allclose(lengths, wl.array.n_elem * wl.array.spacing, rtol=0, atol=1e-12)
    # adjacent sections share their joint
    assert np.allclose(ends[1:, 0], ends[:-1, 1], atol=1e-12)


def test_elements_evenly_spaced_on_chords(wl):
    arr = geometry.build(wl.array)
    d = wl.array.spacing
    for i in range(wl.array.n_chords):
        a, b = arr.chord_ends[i]
        e = arr.elements[i]
        steps = np.linalg.norm(np.diff(e, axis=0), axis=-1)
        assert np.allclose(steps, d, atol=1e-12)
        # collinear with the chord, inside it, half a spacing from each end
        t = (b - a) / np.linalg.norm(b - a)
        n = np.array([-t[1], t[0]])
        assert np.allclose((e - a) @ n, 0.0, atol=1e-12)
        assert math.isclose(np.linalg.norm(e[0] - a), d / 2, abs_tol=1e-12)
        assert math.isclose(np.linalg.norm(e[-1] - b), d / 2, abs_tol=1e-12)


def test_mirror_symmetry_and_orientation(wl):
    arr = geometry.build(wl.array)
    e = arr.elements
    mirrored = e[::-1, ::-1] * np.array([-1.0, 1.0])
    assert np.allclose(e, mirrored, atol=1e-12)
    assert np.all(e[..., 1] < 0.0)  # array below the scene, looking toward +y


def test_channels_and_grids(wl):
    arr = geometry.build(wl.array)
    a = wl.array
    assert arr.n_channels == a.n_channels
    assert np.allclose(np.diff(arr.z_scan), a.scan_step, atol=1e-15)
    assert math.isclose(arr.z_scan.mean(), 0.0, abs_tol=1e-12)  # centred scan
    assert arr.freq[0] == a.f_start and arr.freq[-1] == a.f_stop
    if a.mode == "multi":
        # Tx of each chord: two at each chord end
        for i in range(a.n_chords):
            s, t = arr.chord_ends[i]
            txe = arr.tx_elements[i]
            assert np.allclose(txe[0], s, atol=1e-12) and np.allclose(txe[-1], t, atol=1e-12)
        # all pairs are within one chord
        for c in range(arr.n_channels):
            i = arr.chord_of_channel[c]
            assert any(np.allclose(arr.rx[c], r) for r in arr.elements[i])
            assert any(np.allclose(arr.tx[c], t) for t in arr.tx_elements[i])
    else:
        assert np.array_equal(arr.tx, arr.rx)


def _table1():
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_parameters.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("dummy", [0])
def test_table1_parameters(wl, dummy):
    if wl is not W.C1:
        pytest.skip("one geometry suffices")
    t1 = _table1()
    desc = W.ArrayDesc(mode="mono", n_chords=t1["n_sections"], radius=t1["radius_m"],
                       n_elem=t1["mono_elements_per_section"], spacing=t1["mono_spacing_m"],
                       n_scan=8, scan_step=t1["scan_step_m"], n_freq=t1["n_freq"],
                       f_start=t1["f_start_hz"], f_stop=t1["f_stop_hz"])
    arr = geometry.build(desc)
    # 51 inclusive steps over 30-35 GHz is a 100 MHz step
    assert np.allclose(np.diff(arr.freq), 100e6, rtol=1e-12)
    # the joints of a 3-section polyline are four points spaced by the chord
    # length; Table 1 quotes 19.4 cm between the four transmitters placed there,
    # and 40 x 0.48 cm = 19.2 cm lies within 1.1 % of it
    joints = np.vstack([arr.chord_ends[:, 0], arr.chord_ends[-1:, 1]])
    assert joints.shape == (t1["multi_tx_total"], 2)
    sp = np.linalg.norm(np.diff(joints, axis=0), axis=-1)
    assert np.allclose(sp, 0.192, atol=1e-12)
    assert abs(sp[0] - t1["multi_tx_spacing_m"]) / t1["multi_tx_spacing_m"] < 0.011
    # the multistatic receive spacing is about twice the monostatic one (Sec. III)
    assert 1.9 < t1["multi_rx_spacing_m"] / t1["mono_spacing_m"] < 2.2
    # chord length must be below the diameter, otherwise no polyline exists
    with pytest.raises(ValueError):
        geometry.build(replace(desc, n_elem=500))
