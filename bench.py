"""Benchmark: reconstructed voxels/s of the hybrid (NUFFT) reconstruction on one
MI355X, with brute-force BP beside it and the FP64 oracle timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C2]
                       [--precision fp32|bf16|fp16] [--no-cpu] [--no-bp]

One step = one reconstruct_hybrid call (plan tables, scan FFT, range
compression, back-projection, k_z inverse FFT) over the full echo cube of the
workload, inputs resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import replace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reconstructed voxels/sec, hybrid-NUFFT vs BP, FP32 vs BF16-MFMA at stated err"
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0               # MI355X published HBM3E bandwidth
BF16_MFMA_PEAK_TFLOPS = 2500.0      # MI355X published dense BF16 matrix peak
FLOP_PER_TERM = 24                  # (8 + 4P) with P = 4 interpolation taps
CPU_SHARE_THREADS = 16              # host threads that come with one GPU


def stage_rooflines(plan, a, wl, geom, stage, args):
    """Algorithmic HBM bytes (and, for the FP32 NUFFT, FLOP) of the other
    stages over their event-timed durations: the FFTs move the cube in and
    out once; range compression reads the spectrum and writes the profiles
    (FLOP per (c, k_z) pair: 5 n log2 n + n_f W 14 + 2 n_l with n = n_fine)."""
    n_pairs = geom.n_channels * a.n_scan
    npix = wl.grid.nx * wl.grid.ny
    out = {}

    def hbm(name, nbytes):
        t = stage[name] * 1e-3
        gbs = nbytes / t / 1e9
        out[name] = {"bound": "hbm", "bytes": nbytes, "achieved_gbs": gbs, "peak_gbs": HBM_PEAK_GBS,
                     "frac": gbs / HBM_PEAK_GBS}

    hbm("scan_fft", 2 * n_pairs * a.n_freq * 8)
    hbm("range_compress", n_pairs * (a.n_freq + plan.n_l) * 8)
    hbm("kz_ifft", 2 * npix * a.n_scan * 8)
    if args.precision == "fp32" and args.range_method == "nufft":
        n = plan.n_fine
        flop = n_pairs * (5 * n * math.log2(n) + a.n_freq * plan.kernel_width * 14 + 2 * plan.n_l)
        tf = flop / (stage["range_compress"] * 1e-3) / 1e12
        out["range_compress"].update({"flop": flop, "achieved_tflops": tf, "peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
                                      "frac_alu": tf / FP32_VECTOR_PEAK_TFLOPS})
    return out


def bp_roofline(plan, terms: int, bp_ms: float) -> dict:
    """The back-projection's algorithmic FLOP rate over its event-timed
    launch against the roof of the unit it runs on: the FP32 vector peak for
    the VALU kernels, the dense BF16 / FP16 matrix-core peak for the MFMA
    kernels (which issue 6 (split) or 2 (single pass) MFMA 16x16x32 per
    (4x4 pixels, 16 k_z, channel); that rate is reported as issued_tflops)."""
    achieved = FLOP_PER_TERM * terms / (bp_ms * 1e-3) / 1e12
    if plan.mfma_backprojection:
        n_mfma = 2 if plan.bp_kernel == "mfma-1pass" else 6
        return {"bound": "mfma", "achieved": achieved, "peak": BF16_MFMA_PEAK_TFLOPS,
                "frac": achieved / BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "issued_tflops": n_mfma * 2 * 16 * 16 * 32 / 256 * terms / (bp_ms * 1e-3) / 1e12}
    return {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s"}


def measured_traffic(kernel: str, workload: str, precision: str, n_l: int):
    """HBM bytes per back-projection launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None if there is none for this
    kernel, workload and range grid, or the kernel source changed since it
    was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "backproject_c2_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("traffic:"):
            continue
        f = dict(kv.split("=", 1) for kv in line.split()[1:])
        if (f.get("kernel"), f.get("workload"), f.get("precision"), f.get("n_l")) != (kernel, workload, precision,
                                                                                      str(n_l)):
            continue
        src = os.path.join(ROOT, f["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != f["sha256"]:
            return None
        return int(f["fetch_bytes"]) + int(f["write_bytes"])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def describe(wl) -> str:
    a = wl.array
    if a.mode == "mono":
        arr = f"monostatic polyline {a.n_chords} chords x {a.n_elem} elements on R={a.radius} m"
    else:
        arr = f"multistatic polyline {a.n_chords} chords x ({a.n_tx} Tx, {a.n_elem} Rx) on R={a.radius} m"
    return (f"{arr}, {a.n_scan} scans x {a.scan_step * 1e3:g} mm, {a.n_freq} freqs "
            f"{a.f_start / 1e9:g}-{a.f_stop / 1e9:g} GHz, image {wl.grid.nx}x{wl.grid.ny}x{a.n_scan}, "
            f"{wl.scene.n} {wl.scene.kind} scatterers (seed {wl.scene.seed})")


def cpu_baseline(wl, echo_np, budget_s=20.0):
    """The FP64 oracle timed on a bounded sample of the same workload: the
    exact spectrum at a sample of (k_z, pixel) pairs, split over host threads
    (numpy releases the interpreter lock in its array kernels; one BLAS thread
    per call), extrapolated to the image."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from oracle import geometry as ogeom
    from oracle import hybrid as ohyb
    import workloads as W

    arr = ogeom.build(wl.array)
    npix = wl.grid.nx * wl.grid.ny
    px, py = ohyb.pixel_grid(wl.grid)
    S = ohyb.scan_spectrum(echo_np)   # the FFTs: negligible next to the sums
    visible = len(os.sched_getaffinity(0))
    # the CPU share that comes with one GPU is 16 threads (the host may show
    # more cores, shared with the other GPUs' jobs); never more than visible
    threads = max(1, min(CPU_SHARE_THREADS, visible))

    def run(pix, kap):
        chunks = [c for c in np.array_split(pix, threads) if c.size]
        with ThreadPoolExecutor(len(chunks)) as ex:
            t0 = time.perf_counter()
            list(ex.map(lambda c: ohyb.spectrum_at(arr, S, kap, px[c], py[c]), chunks))
            return time.perf_counter() - t0

    with threadpool_limits(limits=1):
        n_pix = min(npix, 256 * threads)
        dt = run(W.random_subset(npix, n_pix, 99), [0])
        # grow the sample to about budget_s of wall time: more pixels, then
        # more k_z planes of the whole image
        target = budget_s / max(dt / n_pix, 1e-9)
        if target <= npix:
            pix, kap = W.random_subset(npix, max(n_pix, int(target)), 98), [0]
        else:
            n_kap = max(1, min(wl.array.n_scan, int(target // npix)))
            pix = np.arange(npix)
            kap = sorted(set(W.random_subset(wl.array.n_scan, n_kap, 97).tolist()))
        dt = run(pix, kap)
    pairs = len(kap) * pix.size
    total_pairs = wl.array.n_scan * npix
    t_full = dt * total_pairs / pairs
    vox = npix * wl.array.n_scan
    return {"value": vox / t_full, "unit": "voxels/s", "cores": threads, "host_cpus_visible": visible,
            "kind": "oracle",
            "sample": (f"exact spectrum (eq. 7 direct sums) at {pairs} (k_z, pixel) pairs of "
                       f"{total_pairs}, {dt:.1f} s on {threads} host threads, extrapolated linearly; "
                       f"scan FFTs excluded")}


def peak_error(pr, torch, W, wl, geom, opts):
    """Peak-position error on isolated point targets: three scatterers at
    seeded voxel centres of this workload's grid and scan, simulated on the
    GPU; for each, the distance in voxels from its true voxel to the largest
    |g| within 4 voxels of it.  Returns the largest of the three."""
    a, grid = wl.array, wl.grid
    rng = np.random.default_rng(7)
    ix = rng.integers(grid.nx // 4, 3 * grid.nx // 4, 3)
    iy = rng.integers(grid.ny // 4, 3 * grid.ny // 4, 3)
    iz = rng.integers(a.n_scan // 4, 3 * a.n_scan // 4, 3)
    pos = np.stack([grid.x0 + ix * grid.dx, grid.y0 + iy * grid.dy, a.z0 + iz * a.scan_step], axis=1)
    refl = np.ones(3, dtype=np.complex128)
    echo = pr.simulate_echo(geom, torch.from_numpy(pos).cuda(), torch.from_numpy(refl).cuda())
    img = pr.reconstruct_hybrid(geom, grid, echo, **opts).abs().cpu().numpy()
    worst = 0.0
    for x, y, z in zip(ix, iy, iz):
        z0, y0, x0 = max(z - 4, 0), max(y - 4, 0), max(x - 4, 0)
        box = img[z0:z + 5, y0:y + 5, x0:x + 5]
        k = np.unravel_index(np.argmax(box), box.shape)
        worst = max(worst, float(np.sqrt((k[0] + z0 - z) ** 2 + (k[1] + y0 - y) ** 2 + (k[2] + x0 - x) ** 2)))
    return worst


def make_timers(pr, torch, W, wl, geom, echo, img):
    """time_path(opts, steps, warmup) and parity(opts) for one workload
    whose echo and image buffers are resident on the device."""
    a = wl.array

    def time_path(opts, steps, warmup, min_warm_s=0.0):
        """min_warm_s: keep warming up until that much wall time has passed
        as well (after seconds of host-side work the GPU starts the next
        calls below its working clock)."""
        plan = pr.hybrid_plan_info(geom, wl.grid, **opts)
        ws = pr.workspace(plan.workspace_bytes)
        # plan build (host plan + device tables), reported apart; the timed
        # calls reuse the prepared tables
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr.hybrid_prepare(geom, wl.grid, ws=ws, **opts)
        torch.cuda.synchronize()
        first_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(warmup):
            pr.reconstruct_hybrid(geom, wl.grid, echo, out=img, ws=ws, prepared=True, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < min_warm_s:
            pr.reconstruct_hybrid(geom, wl.grid, echo, out=img, ws=ws, prepared=True, **opts)
            torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        # the timed steps: plain calls, one event between consecutive calls
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        for e in marks:
            e.record(stream)   # creates the underlying hipEvent
        torch.cuda.synchronize()
        marks[0].record(stream)
        for k in range(steps):
            pr.reconstruct_hybrid(geom, wl.grid, echo, out=img, ws=ws, prepared=True, **opts)
            marks[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = marks[0].elapsed_time(marks[steps]) / steps
        steps_ms = [marks[k].elapsed_time(marks[k + 1]) for k in range(steps)]
        # a second pass with events between the stages, for the breakdown and
        # the back-projection's launch duration
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        for row in evs:
            for e in row:
                e.record(stream)
        torch.cuda.synchronize()
        for k in range(steps):
            pr.reconstruct_hybrid_events(geom, wl.grid, echo, evs[k], out=img, ws=ws, **opts)
        torch.cuda.synchronize()
        stage = {name: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
                 for i, name in enumerate(pr.STAGES)}
        del ws
        return ms, stage, first_ms, float(np.median(steps_ms)), plan

    def parity(opts):
        """Relative L2 error against the FP64 oracle of the same method on
        sampled (k_z, pixel) pairs of the spectrum, for a seeded CN(0,1) echo
        of this workload."""
        from oracle import geometry as ogeom
        from oracle import hybrid as ohyb
        from oracle import omegak as oomk
        s = W.random_echo(a, 4242)
        out = pr.reconstruct_hybrid(geom, wl.grid, torch.from_numpy(s).cuda(), **opts)
        npix = wl.grid.nx * wl.grid.ny
        pix = W.random_subset(npix, 128, 4243)
        cols = out.reshape(a.n_scan, npix)[:, torch.from_numpy(pix).cuda()].cpu().numpy()
        kap = sorted(set(W.random_subset(a.n_scan, 2, 4244).tolist() + [0]))
        got = np.fft.fft(cols.astype(np.complex128), axis=0)[kap]
        arr = ogeom.build(a)
        px, py = ohyb.pixel_grid(wl.grid)
        if opts.get("range_method", "nufft") == "resample":
            dkl = pr.hybrid_plan_info(geom, wl.grid, **opts).dk_uniform
            ref = oomk.spectrum_at(arr, ohyb.scan_spectrum(s), kap, px[pix], py[pix], dkl,
                                   oomk.reference_lengths(arr, wl.grid))
        else:
            ref = ohyb.spectrum_at(arr, ohyb.scan_spectrum(s), kap, px[pix], py[pix])
        return float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), f"{len(kap)} k_z x {pix.size} pixels"


    return time_path, parity


def time_adjoint(pr, torch, geom, grid, img, steps, warmup, base=None):
    """ms per adjoint_hybrid call (image -> echo) of the FP32 plan with the
    pixel-per-lane back-projection (other options from ``base``), or None if
    that plan takes another kernel; same workspace size as the
    reconstruction, one call per step."""
    aopts = dict(base or {}, precision="fp32", mfma_backprojection=0, range_method="nufft")
    aplan = pr.hybrid_plan_info(geom, grid, **aopts)
    if aplan.bp_kernel != "pixel-lanes":
        return None
    aws = pr.workspace(aplan.workspace_bytes)
    aout = torch.empty(geom.echo_shape, dtype=torch.complex64, device="cuda")
    for _ in range(warmup + 1):
        pr.adjoint_hybrid(geom, grid, img, out=aout, ws=aws, **aopts)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        pr.adjoint_hybrid(geom, grid, img, out=aout, ws=aws, **aopts)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del aws, aout
    return ms


def bench_c3(args, torch, pr, W):
    """The multistatic workload (C3) in the same run: the FP32 path and the
    single-pass FP16 matrix-core path, each timed like the headline (plan
    prepared once, inputs resident), with its error against the oracle on
    sampled outputs and its peak-position error."""
    wl = W.C3
    a = wl.array
    log(f"[bench] C3: {describe(wl)}")
    geom = pr.make_geometry(a)
    pos, refl = W.scatterers(wl.scene)
    echo = pr.simulate_echo(geom, torch.from_numpy(pos).cuda(), torch.from_numpy(refl).cuda())
    img = torch.empty((a.n_scan, wl.grid.ny, wl.grid.nx), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    time_path, parity = make_timers(pr, torch, W, wl, geom, echo, img)
    voxels = wl.grid.nx * wl.grid.ny * a.n_scan
    res = {"workload": f"C3: {describe(wl)}"}
    steps = max(1, min(args.steps, 5))
    paths = (("fp32", {}), ("fp16-mfma-bp-1pass", dict(precision="fp16", mfma_backprojection=2)))
    # the GPU timings first, the host-side checks after (see main)
    for name, opts in paths:
        ms, stage, _, med, plan = time_path(opts, steps, 2, min_warm_s=0.3)
        res[name] = {"value": voxels / (ms * 1e-3), "unit": "voxels/s", "ms_per_step": ms, "median_ms": med,
                     "steps": steps, "stages_ms": stage, "bp_kernel": plan.bp_kernel,
                     "roofline": bp_roofline(plan, a.n_scan * wl.grid.nx * wl.grid.ny * geom.n_channels,
                                             stage["backproject"])}
        log(f"[bench] C3 {name}: {ms:.3f} ms/step ({voxels / (ms * 1e-3):.3e} voxels/s)")
    if not args.no_variants:
        ams = time_adjoint(pr, torch, geom, wl.grid, img, steps, 2)
        if ams is not None:
            res["adjoint"] = {"ms_per_call": ams, "voxels_per_s": voxels / (ams * 1e-3),
                              "note": "image -> echo, FP32, NUFFT plan with the pixel-per-lane kernel"}
            log(f"[bench] C3 adjoint: {ams:.3f} ms per call")
        # One GPU's share of the chord-sharded reconstruction: the middle
        # chord's channels (one of seven) at the full pixel and k_z shape.
        # A run over seven GPUs would add one reduce-scatter of the spectrum
        # by pixel rows before the k_z transform, which is not built here.
        a1 = replace(a, n_chords=1)
        wl1 = replace(wl, array=a1)
        geom1 = pr.make_geometry(a1)
        echo1 = pr.simulate_echo(geom1, torch.from_numpy(pos).cuda(), torch.from_numpy(refl).cuda())
        torch.cuda.synchronize()
        time1, _ = make_timers(pr, torch, W, wl1, geom1, echo1, img)
        share = {"channels": geom1.n_channels,
                 "note": "middle chord of C3 at the full 256x256x512 shape; per-GPU compute of a 7-GPU "
                         "chord-sharded run (its reduce-scatter of the spectrum is not built)"}
        for name, opts in paths:
            ms1, st1, _, med1, _ = time1(opts, steps, 2, min_warm_s=0.3)
            share[name] = {"ms_per_step": ms1, "median_ms": med1, "stages_ms": st1,
                           "fraction_of_full": ms1 / res[name]["ms_per_step"]}
            log(f"[bench] C3 one chord ({geom1.n_channels} channels) {name}: {ms1:.3f} ms/step, "
                f"{ms1 / res[name]['ms_per_step']:.3f} of the full array")
        res["one_chord_share"] = share
        del echo1
    if not args.no_parity:
        for name, opts in paths:
            r = res[name]
            r["rel_l2_vs_oracle"], r["parity_sample"] = parity(opts)
            r["peak_position_error_voxels"] = peak_error(pr, torch, W, wl, geom, opts)
            log(f"[bench] C3 {name}: rel L2 {r['rel_l2_vs_oracle']:.2e}")
    del echo, img
    torch.cuda.empty_cache()
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=50,
                    help="untimed steps first: the GPU reaches its steady clock after about 50 (85 ms)")
    ap.add_argument("--config", default="C2", choices=["C1", "C2", "C3", "C5"],
                    help="C5: the uneven 16-scan batch (one call, graph-replayed)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bp", action="store_true")
    ap.add_argument("--bp-planes", type=int, default=4)
    ap.add_argument("--tile", type=int, default=0, help="back-projection tile (0 = automatic)")
    ap.add_argument("--interp", default="bspline4", choices=["bspline4", "lagrange4", "linear"])
    ap.add_argument("--l-oversample", type=float, default=6.0)
    ap.add_argument("--kz-per-lane", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--mfma-bp", type=int, default=0, choices=[-1, 0, 1, 2],
                    help="1: back-projection on the matrix cores (BF16/FP16 modes); 2: its single-pass FP16 form")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--kz-block", type=int, default=0)
    ap.add_argument("--range-method", default="nufft", choices=["nufft", "resample"],
                    help="range compression: NUFFT (the paper's method) or uniform-grid resampling + IFFT")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the multistatic C3 block of the C2 run")
    ap.add_argument("--no-c5", action="store_true", help="skip the C5 batch block of the C2 run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the reconstruction is not sharded across GPUs)", flush=True)
        return 2

    import torch
    import paper_2109_02842_amd as pr
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", flush=True)
        return 1
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}), flush=True)
        return 0
    if args.config == "C5":
        print(json.dumps(bench_batch(args, torch, pr, W)), flush=True)
        return 0
    wl = W.WORKLOADS[args.config]
    a = wl.array
    log(f"[bench] {args.config}: {describe(wl)}")
    geom = pr.make_geometry(a)
    pos, refl = W.scatterers(wl.scene)
    echo = pr.simulate_echo(geom, torch.from_numpy(pos).cuda(), torch.from_numpy(refl).cuda())
    torch.cuda.synchronize()
    opts = dict(precision=args.precision, tile=args.tile, interp=args.interp,
                l_oversample=args.l_oversample, kz_per_lane=args.kz_per_lane, waves=args.waves,
                mfma_backprojection=args.mfma_bp, tile_y=args.tile_y, kz_block=args.kz_block,
                range_method=args.range_method)
    plan = pr.hybrid_plan_info(geom, wl.grid, **opts)
    img = torch.empty((a.n_scan, wl.grid.ny, wl.grid.nx), dtype=torch.complex64, device="cuda")
    log(f"[bench] plan: n_l={plan.n_l} n_fine={plan.n_fine} W={plan.kernel_width} window={plan.window} "
        f"tile={plan.tile} du={plan.du * 1e3:.3f} mm workspace={plan.workspace_bytes / 2**20:.1f} MiB")

    time_path, parity = make_timers(pr, torch, W, wl, geom, echo, img)

    ms, stage, first_ms, med_ms, plan = time_path(opts, args.steps, args.warmup)
    log(f"[bench] {args.precision}: {args.steps} steps {ms:.3f} ms/step (median {med_ms:.3f}); "
        + ", ".join(f"{k} {v:.3f}" for k, v in stage.items()))

    voxels = wl.grid.nx * wl.grid.ny * a.n_scan
    value = voxels / (ms * 1e-3)
    terms = a.n_scan * wl.grid.nx * wl.grid.ny * geom.n_channels
    bp_ms = stage["backproject"]
    roof = bp_roofline(plan, terms, bp_ms)
    out = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {describe(wl)}",
                   "path": f"hybrid-{'NUFFT' if args.range_method == 'nufft' else 'resample'} {args.precision}",
                   "interp": args.interp, "l_oversample": args.l_oversample, "nufft_tol": 1e-6,
                   "tile": list(plan.tile), "kz_block": plan.block},
        "roofline": dict(roof,
                         traffic=measured_traffic(plan.bp_kernel, args.config, args.precision, plan.n_l),
                         kernel="backproject", flop_per_launch=FLOP_PER_TERM * terms, avg_launch_ms=bp_ms),
        "stages_ms": stage,
        "stages_roofline": stage_rooflines(plan, a, wl, geom, stage, args),
        "plan_build_ms": first_ms,
    }
    # Every GPU timing of this workload first, then the checks against the
    # oracle: those run for seconds on the host, and a GPU left idle that
    # long starts the next timed steps below its working clock.
    vopts_of = {}
    if not args.no_variants:
        out["variants"] = {}
        for name, prec, mbp, rm in (("bf16", "bf16", 0, "nufft"), ("fp16", "fp16", 0, "nufft"),
                                    ("fp32", "fp32", 0, "nufft"), ("bf16-mfma-bp", "bf16", 1, "nufft"),
                                    ("fp16-mfma-bp", "fp16", 1, "nufft"), ("fp16-mfma-bp-1pass", "fp16", 2, "nufft"),
                                    ("fp32-resample", "fp32", 0, "resample")):
            if prec == args.precision and mbp == args.mfma_bp and rm == args.range_method:
                continue
            vopts = dict(opts, precision=prec, mfma_backprojection=mbp, range_method=rm)
            if mbp:
                vopts.update(tile=0, tile_y=0, kz_block=0, kz_per_lane=0, waves=0)
            vms, vstage, _, vmed, vplan = time_path(vopts, args.steps, args.warmup)
            out["variants"][name] = {"value": voxels / (vms * 1e-3), "ms_per_step": vms, "stages_ms": vstage,
                                     "speedup_vs_main": ms / vms, "bp_kernel": vplan.bp_kernel,
                                     "roofline": bp_roofline(vplan, terms, vstage["backproject"])}
            vopts_of[name] = vopts
            log(f"[bench] {name}: {vms:.3f} ms/step; range_compress {vstage['range_compress']:.3f} ms; "
                f"backproject {vstage['backproject']:.3f} ms")

    if not args.no_variants:
        # the adjoint (image -> echo) of the FP32 pixel-per-lane plan
        ams = time_adjoint(pr, torch, geom, wl.grid, img, args.steps, args.warmup, opts)
        if ams is not None:
            out["adjoint"] = {"ms_per_call": ams, "voxels_per_s": voxels / (ams * 1e-3),
                              "note": "image -> echo, FP32, NUFFT plan with the pixel-per-lane kernel"}
            log(f"[bench] adjoint: {ams:.3f} ms per call")

    if not args.no_bp:
        nz = max(1, min(args.bp_planes, a.n_scan))
        iz0 = a.n_scan // 2 - nz // 2
        bws = pr.workspace(pr.bp_workspace_bytes(geom, wl.grid, nz))
        bimg = torch.empty((nz, wl.grid.ny, wl.grid.nx), dtype=torch.complex64, device="cuda")
        pr.reconstruct_bp(geom, wl.grid, echo, iz0=iz0, nz=nz, out=bimg, ws=bws)   # warm-up
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pr.reconstruct_bp(geom, wl.grid, echo, iz0=iz0, nz=nz, out=bimg, ws=bws)
        e1.record(stream)
        torch.cuda.synchronize()
        bms = e0.elapsed_time(e1)
        bp_vps = nz * wl.grid.nx * wl.grid.ny / (bms * 1e-3)
        out["bp"] = {"value": bp_vps, "unit": "voxels/s", "planes_timed": nz, "ms": bms,
                     "note": "GPU BP timed on a slab of scan planes; its cost is linear in voxels",
                     "hybrid_speedup": value / bp_vps}
        log(f"[bench] BP: {nz} planes in {bms:.1f} ms -> {bp_vps:.3e} voxels/s; hybrid speedup "
            f"{value / bp_vps:.0f}x")
        # the three methods of the paper's Table 2 on this workload (FP32)
        times = {}
        if args.precision == "fp32" and args.mfma_bp <= 0:
            times[args.range_method] = ms
        for name, rm in (("fp32", "nufft"), ("fp32-resample", "resample")):
            if name in out.get("variants", {}):
                times[rm] = out["variants"][name]["ms_per_step"]
        if "nufft" in times and "resample" in times:
            out["table2_analogue"] = {
                "omegaK_NUFFT_BP_ms": times["nufft"], "omegaK_BP_ms": times["resample"],
                "BP_ms": voxels / bp_vps * 1e3,
                "note": "whole volume, FP32; BP extrapolated from the timed slab"}

    if not args.no_parity:
        err, sample = parity(opts)
        out["rel_l2_vs_oracle"] = {"value": err, "sample": sample, "echo": "seeded CN(0,1)"}
        log(f"[bench] {args.precision}: rel L2 vs oracle {err:.2e} ({sample})")
        pk = peak_error(pr, torch, W, wl, geom, opts)
        out["peak_position_error_voxels"] = pk
        log(f"[bench] {args.precision}: peak-position error {pk:.2f} voxels (3 point targets)")
        for name, vopts in vopts_of.items():
            v = out["variants"][name]
            v["rel_l2_vs_oracle"], _ = parity(vopts)
            v["peak_position_error_voxels"] = peak_error(pr, torch, W, wl, geom, vopts)
            log(f"[bench] {name}: rel L2 {v['rel_l2_vs_oracle']:.2e}; "
                f"peak error {v['peak_position_error_voxels']:.2f} voxels")

    if args.config == "C2" and not args.no_c3:
        out["multistatic_c3"] = bench_c3(args, torch, pr, W)
    if args.config == "C2" and not args.no_variants and not args.no_c5:
        # the uneven batch (C5), as in a --config C5 run
        c5 = bench_batch(args, torch, pr, W, min_warm_s=0.3)
        out["batch_c5"] = {k: c5[k] for k in ("value", "unit", "ms_per_step", "config", "roofline", "batch",
                                               "rel_l2_vs_oracle") if k in c5}

    if not args.no_cpu:
        log("[bench] oracle CPU baseline ...")
        echo_np = echo.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(wl, echo_np)
        log(f"[bench] oracle: {out['cpu_baseline']['value']:.3e} voxels/s")
    print(json.dumps(out), flush=True)
    return 0


def bench_batch(args, torch, pr, W, min_warm_s=0.0) -> dict:
    """The uneven batch (16 monostatic scans of different chords, elements,
    scan lengths and frequency counts, 128 x 128 images): one
    reconstruct_hybrid_batch call (plan tables prepared once) captured in a
    graph and replayed; the same scans as 16 separate reconstruct_hybrid
    calls, plain and prepared, for comparison.  min_warm_s: each timing
    also warms up for that much wall time (after host-side work)."""
    wls = W.batch_c5()
    geoms = [pr.make_geometry(w.array) for w in wls]
    echoes = []
    for w, g in zip(wls, geoms):
        pos, refl = W.scatterers(w.scene)
        echoes.append(pr.simulate_echo(g, torch.from_numpy(pos).cuda(), torch.from_numpy(refl).cuda()))
    torch.cuda.synchronize()
    opts = dict(precision=args.precision)
    # per-scan launch shapes from the autotuner (timed on the device here)
    t0 = time.perf_counter()
    batch = pr.HybridBatch.autotuned(geoms, [w.grid for w in wls], args.precision, echoes=echoes, repeats=3)
    tune_s = time.perf_counter() - t0
    voxels = sum(w.array.n_scan * w.grid.nx * w.grid.ny for w in wls)
    terms = sum(w.array.n_scan * w.grid.nx * w.grid.ny * g.n_channels for w, g in zip(wls, geoms))
    log(f"[bench] C5: {len(wls)} scans, {voxels:.3e} voxels; persistent back-projection: "
        f"{batch.queued_scans} scans, {batch.work_items} work items, {batch.workgroups} workgroups")
    stream = torch.cuda.current_stream()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < min_warm_s:
            fn()
            torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    cap = pr.CapturedBatch(batch, echoes)
    ms = timed(cap.replay, args.steps, args.warmup)
    bws = pr.workspace(batch.workspace_bytes)
    outs = [torch.empty_like(o) for o in cap.outs]
    ms_call = timed(lambda: pr.reconstruct_hybrid_batch(batch, echoes, outs, bws), args.steps, 1)
    wss = [pr.workspace(pr.hybrid_workspace_bytes(g, w.grid, **so)) for g, w, so in zip(geoms, wls, batch.opts)]

    def singles():
        for g, w, e, o, ws, so in zip(geoms, wls, echoes, outs, wss, batch.opts):
            pr.reconstruct_hybrid(g, w.grid, e, out=o, ws=ws, **so)

    ms_single = timed(singles, args.steps, 1)
    # the same with each scan's tables prepared once (the graph replays the
    # prepared batch call)
    for g, w, ws, so in zip(geoms, wls, wss, batch.opts):
        pr.hybrid_prepare(g, w.grid, ws=ws, **so)

    def singles_prepared():
        for g, w, e, o, ws, so in zip(geoms, wls, echoes, outs, wss, batch.opts):
            pr.reconstruct_hybrid(g, w.grid, e, out=o, ws=ws, prepared=True, **so)

    ms_single_p = timed(singles_prepared, args.steps, 1)
    log(f"[bench] C5: graph replay {ms:.3f} ms (prepared batch), batch call {ms_call:.3f} ms, 16 separate calls "
        f"{ms_single:.3f} ms ({ms_single_p:.3f} ms prepared)")
    achieved = FLOP_PER_TERM * terms / (ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": voxels / (ms * 1e-3), "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else args.precision, "data": "synthetic",
        "config": {"workload": "C5: 16 uneven monostatic scans (3-7 chords, 32-64 elements, 128-512 scans, "
                               "32-128 freqs, seeds 50-65), 128x128 images, one graph-replayed batch call",
                   "path": f"hybrid-NUFFT {args.precision} batch"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": None,
                     "kernel": "whole batch call (back-projection FLOP over the call's time: a lower bound)",
                     "flop_per_launch": FLOP_PER_TERM * terms, "avg_launch_ms": ms},
        "batch": {"scans": len(wls), "queued_scans": batch.queued_scans, "work_items": batch.work_items,
                  "workgroups": batch.workgroups, "ms_graph_replay": ms, "ms_batch_call": ms_call,
                  "ms_separate_calls": ms_single, "ms_separate_calls_prepared": ms_single_p,
                  "autotune_s": tune_s,
                  "scan_lengths": [w.array.n_scan for w in wls],
                  "tuned_options": [{k: v for k, v in o.items() if k != "precision"} for o in batch.opts]},
    }
    if not args.no_parity:
        from oracle import geometry as ogeom
        from oracle import hybrid as ohyb
        errs = []
        for i in (0, 15):
            w, g = wls[i], geoms[i]
            s = W.random_echo(w.array, 4242 + i)
            img = pr.reconstruct_hybrid_batch(batch, [torch.from_numpy(s).cuda() if j == i else echoes[j]
                                                      for j in range(len(wls))])[i]
            npix = w.grid.nx * w.grid.ny
            pix = W.random_subset(npix, 96, 4300 + i)
            cols = img.reshape(w.array.n_scan, npix)[:, torch.from_numpy(pix).cuda()].cpu().numpy()
            kap = [0, w.array.n_scan // 3]
            got = np.fft.fft(cols.astype(np.complex128), axis=0)[kap]
            px, py = ohyb.pixel_grid(w.grid)
            ref = ohyb.spectrum_at(ogeom.build(w.array), ohyb.scan_spectrum(s), kap, px[pix], py[pix])
            errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        out["rel_l2_vs_oracle"] = {"value": max(errs), "sample": "2 k_z x 96 pixels of scans 0 and 15",
                                   "echo": "seeded CN(0,1)"}
        log(f"[bench] C5: rel L2 vs oracle {max(errs):.2e}")
    return out


if __name__ == "__main__":
    sys.exit(main())
