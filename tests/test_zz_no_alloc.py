"""reconstruct_hybrid_static (no workspace, no allocation: the library's
static per-device scratch) against reconstruct_hybrid, through the C ABI.

Two calls in a row, the second on a smaller problem, each bitwise equal to
reconstruct_hybrid with a workspace (same plan, same kernels); a problem
whose workspace exceeds the static scratch and a geometry whose tables were
never uploaded are refused with an error instead of allocating.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pr = pytest.importorskip("paper_2109_02842_amd")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.synchronize()


def _static(g, grid, echo, out, **opts):
    return pr.lib().reconstruct_hybrid_static(g.handle, C.byref(pr._grid(grid)), C.byref(pr._opts(**opts)),
                                              C.c_void_p(echo.data_ptr()), C.c_void_p(out.data_ptr()), pr._stream())


def test_static_scratch_matches_workspace_call_twice_then_refuses():
    for wl, opts, seed in ((W.C1, {}, 3), (W.tiny("multi"), dict(interp="lagrange4"), 4)):
        g = pr.make_geometry(wl.array)
        need = pr.hybrid_workspace_bytes(g, wl.grid, **opts)
        say("static scratch", wl.name, opts, need, "of", pr.STATIC_SCRATCH_BYTES)
        assert need <= pr.STATIC_SCRATCH_BYTES
        echo = torch.from_numpy(W.random_echo(wl.array, seed)).cuda()
        out = torch.full((wl.array.n_scan, wl.grid.ny, wl.grid.nx), complex(7, 7), dtype=torch.complex64,
                         device="cuda")
        assert _static(g, wl.grid, echo, out, **opts) == pr.PL_OK, pr.last_error()
        want = pr.reconstruct_hybrid(g, wl.grid, echo, **opts).cpu().numpy()
        got = out.cpu().numpy()
        assert np.isfinite(got).all()
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        say("   rel L2 vs reconstruct_hybrid", err)
        assert err < 1e-6
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # a problem larger than the static scratch: an error, nothing launched
    g2 = pr.make_geometry(W.C2.array)
    assert pr.hybrid_workspace_bytes(g2, W.C2.grid) > pr.STATIC_SCRATCH_BYTES
    e2 = torch.zeros(g2.echo_shape, dtype=torch.complex64, device="cuda")
    o2 = torch.zeros((W.C2.array.n_scan, W.C2.grid.ny, W.C2.grid.nx), dtype=torch.complex64, device="cuda")
    assert _static(g2, W.C2.grid, e2, o2) == pr.PL_EWORKSPACE
    assert "static scratch" in pr.last_error()
    # a geometry whose tables are not on the device: an error, no upload
    d = pr.GeometryDesc()
    a = W.tiny("mono").array
    d.mode, d.n_chords, d.radius_m, d.arc_center_rad = pr.PL_MONO, a.n_chords, a.radius, a.arc_center
    d.n_elem, d.n_tx, d.spacing_m, d.n_scan, d.n_freq = a.n_elem, 0, a.spacing, a.n_scan, a.n_freq
    d.scan_step_m, d.scan_z0_m, d.f_start_hz, d.f_stop_hz = a.scan_step, a.z0, a.f_start, a.f_stop
    h = C.c_void_p()
    assert pr.lib().make_geometry(C.byref(d), C.byref(h)) == pr.PL_OK
    try:
        grid = C.byref(pr._grid(W.tiny("mono").grid))
        e3 = torch.zeros((a.n_chords * a.n_elem, a.n_scan, a.n_freq), dtype=torch.complex64, device="cuda")
        o3 = torch.zeros((a.n_scan, 9, 9), dtype=torch.complex64, device="cuda")
        rc = pr.lib().reconstruct_hybrid_static(h, grid, C.byref(pr._opts()), C.c_void_p(e3.data_ptr()),
                                                C.c_void_p(o3.data_ptr()), pr._stream())
        assert rc == pr.PL_EINVAL and "geometry_upload" in pr.last_error()
    finally:
        pr.lib().destroy_geometry(h)
    torch.cuda.synchronize()
