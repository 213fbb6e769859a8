#!/usr/bin/env python3
"""Benchmark of the grid-hopping hot path on one MI355X.

One step is one synthetic frame of the paper-scale workload (4 receivers,
Ms = 256 samples x Mc = 128 chirps, complex64, 3 targets, SNR 10 dB, f0 = 24 GHz,
B = 250 MHz, Tc = 256 us) through every row of the hot path, with no host
synchronisation inside the step:
  1. range-Doppler maps (zero padding x4): 4 maps of 1024 x 512 bins;
  2. grid-hopping decision, bilinear, on the 128 x 128 x 32 x 32 grid
     (16,777,216 points), FP32 volume written, block maxima, global argmax;
  3. direct decision on the stride-2 64 x 64 x 16 x 16 subgrid (1,048,576
     points), volume written, block maxima, global argmax;
  4. Block-OMP, 3 iterations: the first selection is the argmax of step 2
     (gh_bomp_seed: the maps of step 1 are the run's maps of the frame, and
     its decision is the first selection's sweep), then per iteration the
     least-squares fit and residual, and for the next selection the maps of
     the residual (from the maps of the frame and the fitted atoms in closed
     form) and a grid-hopping argmax-only sweep with the support excluded;
  5. Newton refinement of the 3 selected cells.
Grid points evaluated per step: 3 x 16,777,216 (grid hopping: the sweep of
step 2 and the two later selections) + 1,048,576 (direct).  `value` is that
count divided by the measured step time.  The step is captured once in a
HIP graph (kernel launches only; no memset) and the timed steps are graph
replays.  Row 3 is independent of the rest: by default (`--streams 2`) it
runs on a second stream beside rows 1, 2 and 4, and the last Block-OMP fit
(which the refinement does not need) runs there beside the refinement; the
second stream is forked from and joined back into the capture stream.
`--streams 1` captures everything on one stream in the order above.  The
per-row times come from eager
one-stream steps with HIP events, and after the replays the step's outputs
(argmax cells, Block-OMP support and coefficients, refined estimates) are
compared with those of an eager step (`graph_matches_eager`).

The roofline object covers the dominant kernel, the grid-hopping sweep of
step 2, timed with HIP events on the stream it runs on (20 volume-writing
launches back to back, so that no host launch gap falls between the events);
its algorithmic bytes per launch are the FP32 volume write, one read of the
four maps and the block maxima.  The CPU baseline runs the FP64 numpy oracle in a child process on a
bounded sample of the same frame, one thread, and scales its per-point rates
to the step.

Beside the step (not part of `value`), the batching workload is measured: 64
seeded frames of mixed shapes (K 3..8, Ms 128/256, Mc 64/128, grids 64^2..192^2
x 16^2..32^2) through the batch entry points (maps, bilinear decision with
block maxima, per-frame argmax; three persistent launches plus the argmax),
launch shapes autotuned, one run captured in a HIP graph and replayed.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CFG = 2
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0   # dense matrix-core BF16
FLOP_PER_POINT_RX = {"bilinear": 12, "bicubic": 44}   # algorithmic, per grid point and receiver
PRECISION_CFG = 3
CUS = 256                 # MI355X compute units
CLOCK_HZ = 2.4e9          # peak engine clock
BOMP_ITERS = 3
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "gh_sweep_columns_paper_scale_hbm_traffic.md")
SWEEP_SOURCES = [os.path.join(ROOT, "paper_2307_16550_amd", "csrc", f) for f in ("sweep_fast.hip", "sweep_table.h")]
INTERNAL_HEADER = os.path.join(ROOT, "paper_2307_16550_amd", "csrc", "gh_internal.h")
DEVICE_PART_END = "// ---- batches of frames"   # gh_internal.h from here on declares host launchers only
BATCH_REPLAYS = 10
EAGER_ROW_STEPS = 20


def direct_flop(radar, n):
    """Algorithmic FLOPs of the direct decision: both complex contractions per
    receiver, range zoom K Nloc Ms Mc and Doppler zoom K Nloc Nv Mc multiply-adds."""
    nloc, nv = n[0] * n[1], n[2] * n[3]
    return 8.0 * radar.k * radar.mc * nloc * (radar.ms + nv)


def recorded_traffic(key="traffic_bytes_per_launch"):
    """A per-launch figure of the bilinear sweep from the committed counter record
    (HBM bytes by default; "valu_insts_per_launch" for the VALU wave
    instructions), or None when the sweep sources have changed since the
    counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_RECORD).read()
        h = hashlib.sha256()
        for f in SWEEP_SOURCES:
            with open(f, "rb") as fh:
                h.update(fh.read())
        header = open(INTERNAL_HEADER).read()
        h.update(header[:header.index(DEVICE_PART_END)].encode())
    except (OSError, ValueError):
        return None
    m_bytes = re.search(r"^" + key + r":\s*(\d+)", text, re.M)
    m_sha = re.search(r"^sweep_source_sha256:\s*([0-9a-f]{64})", text, re.M)
    if not m_bytes or not m_sha or m_sha.group(1) != h.hexdigest():
        return None
    return int(m_bytes.group(1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--streams", type=int, choices=(1, 2), default=2,
                    help="streams of the captured step: 2 runs the independent rows beside Block-OMP")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batching-workload measurement")
    ap.add_argument("--step-only", action="store_true",
                    help="time the step alone: no side measurements, batch or CPU baseline (profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only measure the batching workload and print its JSON object (profiling)")
    ap.add_argument("--interp", choices=["bilinear", "bicubic"], default="bilinear")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this size (HBM counter calibration) and exit")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-parallel", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


# ----------------------------------------------------------------------------- CPU baseline (oracle)

_POOL_ARGS = {}


def _pool_gh(lo, hi):
    a = _POOL_ARGS
    from oracle import gh as ogh
    return ogh.gh_points(a["z"], a["r"], *(p[lo:hi] for p in a["pts"]), a["interp"])


def _pool_dir(lo, hi):
    a = _POOL_ARGS
    from oracle import direct as odirect
    return odirect.direct_points(a["y"], a["r"], *(p[lo:hi] for p in a["dpts"]))


def cpu_worker(path, parallel=False):
    """Child process: time the FP64 oracle on a bounded sample; compare with the GPU samples.
    With `parallel`, the sampled grid-hopping and direct points are split over a process
    pool of every core the process may use (the oracle itself unchanged)."""
    import numpy as np

    from oracle import bomp as obomp, direct as odirect, gh as ogh, maps as omaps
    from oracle import radar as ordr, refine as orefine
    from paper_2307_16550_amd import scene as sc

    job = np.load(path, allow_pickle=False)
    s = sc.make_scene(CFG, 0)
    r = ordr.radar_from_scene(s)
    grid = s.grid
    dgrid = sc.direct_grid(s, CFG)
    interp = int(job["interp"])
    t0 = time.perf_counter()
    z = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    t_maps = time.perf_counter() - t0

    def points(g, idx):
        ax = ordr.grid_axes(g)
        n = g.n
        return (ax[0][idx // (n[1] * n[2] * n[3])], ax[1][(idx // (n[2] * n[3])) % n[1]],
                ax[2][(idx // n[3]) % n[2]], ax[3][idx % n[3]])

    gh_idx = job["gh_idx"]
    pts = points(grid, gh_idx)
    d_idx = job["dir_idx"]
    dpts = points(dgrid, d_idx)
    cores = len(os.sched_getaffinity(0)) if parallel else 1
    if parallel:
        import multiprocessing as mp
        _POOL_ARGS.update(z=z, r=r, pts=pts, dpts=dpts, y=s.y, interp=interp)
        ctx = mp.get_context("fork")     # workers inherit the oracle's inputs; nothing large is pickled
        with ctx.Pool(cores) as pool:
            def split(n):
                b = np.linspace(0, n, 4 * cores + 1).astype(int)
                return list(zip(b[:-1], b[1:]))
            t0 = time.perf_counter()
            gh_ref = np.concatenate(pool.starmap(_pool_gh, split(len(gh_idx))))
            t_gh_pt = (time.perf_counter() - t0) / len(gh_idx)
            t0 = time.perf_counter()
            dir_ref = np.concatenate(pool.starmap(_pool_dir, split(len(d_idx))))
            t_dir_pt = (time.perf_counter() - t0) / len(d_idx)
    else:
        t0 = time.perf_counter()
        gh_ref = ogh.gh_points(z, r, *pts, interp)
        t_gh_pt = (time.perf_counter() - t0) / len(gh_idx)
        t0 = time.perf_counter()
        dir_ref = odirect.direct_points(s.y, r, *dpts)
        t_dir_pt = (time.perf_counter() - t0) / len(d_idx)

    support = [int(c) for c in job["support"]]
    t0 = time.perf_counter()
    for t in range(1, len(support) + 1):
        obomp.fit(s.y, r, grid, support[:t])
    t_fit = time.perf_counter() - t0
    t0 = time.perf_counter()
    orefine.refine(s.y, r, grid, support[:1])
    t_ref1 = time.perf_counter() - t0

    n_gh, n_dir = grid.size, dgrid.size
    # the step's work: maps of the frame and of the residual before each later
    # selection, BOMP_ITERS sweeps of the grid, the direct subgrid, the fits and
    # the refinement of every selected cell
    t_step = BOMP_ITERS * (t_maps + n_gh * t_gh_pt) + n_dir * t_dir_pt + t_fit + len(support) * t_ref1
    sampled = t_maps + len(gh_idx) * t_gh_pt + len(d_idx) * t_dir_pt + t_fit + t_ref1
    gh_scale = max(float(np.max(gh_ref)), float(job["gh_max"]))
    dir_scale = max(float(np.max(dir_ref)), float(job["dir_max"]))
    out = {
        "value": (BOMP_ITERS * n_gh + n_dir) / t_step,
        "unit": "grid points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"FP64 numpy oracle, {'a pool of ' + str(cores) + ' processes of 1 thread for the sampled points' if parallel else '1 thread'}: "
                   f"maps of the frame, grid hopping at {len(gh_idx)} points, "
                   f"direct at {len(d_idx)} points, BOMP fits for supports of 1..{len(support)}, one refinement; "
                   f"per-point and per-call times scaled to the step ({sampled:.1f} s measured)"),
        "step_seconds_estimate": t_step,
        "gh_points_per_s": 1.0 / t_gh_pt,
        "direct_points_per_s": 1.0 / t_dir_pt,
        "max_rel_error_gh": float(np.max(np.abs(job["gh_gpu"] - gh_ref)) / gh_scale),
        "max_rel_error_direct": float(np.max(np.abs(job["dir_gpu"] - dir_ref)) / dir_scale),
    }
    print(json.dumps(out))


def cpu_baseline(job, parallel=False):
    import numpy as np
    fd, path = tempfile.mkstemp(suffix=".npz")
    os.close(fd)
    try:
        np.savez(path, **job)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
                   HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", path] + (["--cpu-parallel"] if parallel else [])
        res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
        if res.returncode != 0:
            return {"error": res.stderr[-2000:]}
        return json.loads(res.stdout.strip().splitlines()[-1])
    finally:
        os.unlink(path)


# ----------------------------------------------------------------------------- GPU benchmark

def factored_timings(gh, torch, radar, grid, y, stream, reps=50):
    """The paper's factorised estimator (eqs. (5)-(6)) on the step's frame: grid hopping with
    polar range interpolation and nearest-bin Doppler (range spectra included), and the direct
    method with FP32 matrix-core range zoom; ms per frame by HIP events."""
    spec = gh.range_spectra(radar, y)
    ws_g = torch.empty(gh.factored_workspace_bytes(radar, grid, gh.FACTOR_GH), dtype=torch.uint8, device=y.device)
    ws_d = torch.empty(gh.factored_workspace_bytes(radar, grid, gh.FACTOR_DIRECT), dtype=torch.uint8,
                       device=y.device)
    out = {}
    for name, fn in (("gh_polar_nearest_ms", lambda: (gh.range_spectra(radar, y, spec),
                                                      gh.factored_decision(radar, grid, gh.FACTOR_GH, spec, gh.POLAR,
                                                                           ws=ws_g))),
                     ("direct_f32_ms", lambda: gh.factored_decision(radar, grid, gh.FACTOR_DIRECT, y, ws=ws_d))):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    out["locations"] = grid.n[0] * grid.n[1]
    out["velocities"] = grid.n[2] * grid.n[3]
    return out


def batch_workload(gh, sc, torch, stream):
    """Frames/s and grid points/s of the batching workload (graph replays, HIP events)."""
    scenes = sc.make_batch()
    b = gh.Batch.from_scenes(scenes, gh.BILINEAR)
    tuned = gh.autotune(b, reps=3)
    g = b.capture()
    g.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(BATCH_REPLAYS):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / BATCH_REPLAYS
    info = b.info()
    b.close()
    return {"workload": "64 seeded frames of mixed shapes, bilinear, maps + decision (block maxima) + argmax",
            "frames": info["n_frames"], "points": info["points"], "ms_per_batch": ms,
            "frames_per_s": info["n_frames"] / ms * 1e3, "points_per_s": info["points"] / ms * 1e3,
            "replays": BATCH_REPLAYS, "hip_graph": True,
            "launch_shape": {"workgroups": info["workgroups"], "sweep_waves": info["sweep_waves"],
                             "column_height": info["column_height"], "sweep_locations": info["sweep_locations"],
                             "range_chirps": info["range_chirps"], "doppler_rows": info["doppler_rows"]},
            "autotune_trials": len(tuned["trials"])}


def main():
    args = parse()
    if args.cpu_worker:
        cpu_worker(args.cpu_worker, args.cpu_parallel)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the frame path shards by frames across GPUs, which this benchmark does not run)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2307_16550_amd import gridhop as gh
    from paper_2307_16550_amd import scene as sc

    dev = torch.device("cuda:0")
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration_mib, "launches": 3}))
        return 0

    if args.batch_only:
        print(json.dumps(batch_workload(gh, sc, torch, torch.cuda.current_stream())), flush=True)
        return 0

    interp = gh.BICUBIC if args.interp == "bicubic" else gh.BILINEAR
    s = sc.make_scene(CFG, 0)
    radar = gh.Radar.from_scene(s)
    grid = gh.grid_of(s.grid)
    dgrid_s = sc.direct_grid(s, CFG)
    dgrid = gh.grid_of(dgrid_s)
    y = torch.from_numpy(s.y).to(dev)
    maps = torch.empty((radar.k, radar.nr, radar.nd), dtype=torch.complex64, device=dev)
    n_gh, n_dir = s.grid.size, dgrid_s.size
    nloc, nloc_d = s.grid.n[0] * s.grid.n[1], dgrid_s.n[0] * dgrid_s.n[1]
    dec = torch.empty(tuple(s.grid.n), dtype=torch.float32, device=dev)
    block = gh.peaks_tensor(nloc, dev)
    arg = gh.peaks_tensor(1, dev)
    ws = torch.empty(gh.direct_workspace_bytes(radar, dgrid), dtype=torch.uint8, device=dev)
    ddec = torch.empty(tuple(dgrid_s.n), dtype=torch.float32, device=dev)
    dblock = gh.peaks_tensor(nloc_d, dev)
    darg = gh.peaks_tensor(1, dev)
    bomp = gh.BompState(radar, grid, y, max_support=BOMP_ITERS, use_direct=False, interp=interp)
    fmaps = bomp.maps       # the frame's maps: the grid-hopping row's and Block-OMP's
    theta = torch.empty((BOMP_ITERS, 4), dtype=torch.float64, device=dev)
    rws = torch.empty(gh.refine_workspace_bytes(radar, grid, BOMP_ITERS), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    marks = []

    def step(record):
        e = [ev() for _ in range(6)] if record else None
        if record:
            e[0].record(stream)
        gh.rd_maps(radar, y, fmaps)
        if record:
            e[1].record(stream)
        gh.decision(radar, grid, fmaps, interp, dec=dec, block=block, want_argmax=False)
        if record:
            e[2].record(stream)
        # the grid-hopping argmax is Block-OMP's first selection: one launch for both
        bomp.reset()
        bomp.seed(block, selected=arg)
        if record:
            e[3].record(stream)
        gh.direct_decision(radar, dgrid, y, ws=ws, dec=ddec, block=dblock, want_argmax=False)
        if record:
            e[4].record(stream)
        gh.argmax(dblock, darg)
        bomp.fit()
        for _ in range(BOMP_ITERS - 1):
            bomp.step()
        gh.refine(radar, grid, y, bomp.support, theta=theta, ws=rws)
        if record:
            e[5].record(stream)
            marks.append(e)

    # eager steps: warm-up, then per-row HIP events on the launch stream
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    for _ in range(min(args.steps, EAGER_ROW_STEPS)):
        step(True)
    torch.cuda.synchronize()
    snap = lambda: [t.clone() for t in (arg, darg, bomp.support, bomp.alpha, theta)]
    ref = snap()

    # The direct decision (B) is independent of the chain maps -> sweep ->
    # argmax -> Block-OMP -> refinement (A; the sweep is Block-OMP's first
    # selection).  With two streams, A runs on the capture stream; a second
    # stream (default priority), forked from and joined back into it, waits
    # for the last selection, then runs the last fit (the refinement needs only
    # the selections) and B beside the refinement, whose 96 workgroups leave
    # most of the chip to them.
    side = torch.cuda.Stream(device=dev) if args.streams == 2 else None

    def step_two_streams():
        main_s = torch.cuda.current_stream()
        join = torch.cuda.Event()
        gh.rd_maps(radar, y, fmaps)
        gh.decision(radar, grid, fmaps, interp, dec=dec, block=block, want_argmax=False)
        bomp.reset()
        bomp.seed(block, selected=arg)
        bomp.fit()
        for _ in range(BOMP_ITERS - 2):
            bomp.step()
        bomp.select()
        selected = torch.cuda.Event()
        selected.record(main_s)
        side.wait_event(selected)
        with torch.cuda.stream(side):
            bomp.fit()
            gh.direct_decision(radar, dgrid, y, ws=ws, dec=ddec, block=dblock, want_argmax=False)
            gh.argmax(dblock, darg)
        gh.refine(radar, grid, y, bomp.support, theta=theta, ws=rws)
        join.record(side)
        main_s.wait_event(join)

    # the timed steps: the whole step captured once in a HIP graph and replayed
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        if side is not None:
            step_two_streams()
        else:
            step(False)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph_matches_eager = all(torch.equal(a, b) for a, b in zip(snap(), ref))

    # the volume-writing sweep's average launch duration, for the roofline: 20 launches back to
    # back between two events on its stream (the eager row events also hold the host's launch
    # gap after the short map passes)
    for _ in range(3):
        gh.decision(radar, grid, fmaps, interp, dec=dec, block=block, want_argmax=False)
    v0, v1 = ev(), ev()
    v0.record(stream)
    for _ in range(20):
        gh.decision(radar, grid, fmaps, interp, dec=dec, block=block, want_argmax=False)
    v1.record(stream)
    torch.cuda.synchronize()
    t_sweep_launch = v0.elapsed_time(v1) * 1e-3 / 20

    def avg(i, j):
        return float(np.mean([m[i].elapsed_time(m[j]) for m in marks])) * 1e-3

    t_maps, t_sweep, t_arg, t_dir, t_total = avg(0, 1), avg(1, 2), avg(2, 3), avg(3, 4), avg(0, 5)

    def side_measurements():
        """Beside the step, not part of `value`: step-time distribution, device-copy bandwidth,
        grid hopping on the direct subgrid, the BF16 direct decision, the factorised estimator."""
        # step-time distribution: each replay bracketed by events (a separate pass, after the timed one)
        per = []
        for _ in range(min(args.steps, 50)):
            a, b = ev(), ev()
            a.record(stream)
            graph.replay()
            b.record(stream)
            per.append((a, b))
        torch.cuda.synchronize()
        step_ms = np.array([a.elapsed_time(b) for a, b in per])

        # the same step captured on one stream, timed the same way as `value`
        one_ms = None
        if side is not None:
            g1 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g1):
                step(False)
            for _ in range(args.warmup):
                g1.replay()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                g1.replay()
            torch.cuda.synchronize()
            one_ms = (time.perf_counter() - t1) / args.steps * 1e3
            del g1

        # device-copy bandwidth (read + write bytes of a 256 MiB copy) as the practical HBM ceiling
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        c0, c1 = ev(), ev()
        c0.record(stream)
        for _ in range(10):
            dst.copy_(src)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 2 * src.numel() * 4 * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        del src, dst

        # grid hopping on the direct method's 64x64x16x16 subgrid: the same points as the direct row
        sub_dec = torch.empty(tuple(dgrid_s.n), dtype=torch.float32, device=dev)
        for _ in range(3):
            gh.rd_maps(radar, y, maps)
            gh.decision(radar, dgrid, maps, interp, dec=sub_dec, block=dblock, argmax=darg)
        s0, s1 = ev(), ev()
        s0.record(stream)
        for _ in range(20):
            gh.rd_maps(radar, y, maps)
            gh.decision(radar, dgrid, maps, interp, dec=sub_dec, block=dblock, argmax=darg)
        s1.record(stream)
        torch.cuda.synchronize()
        t_gh_sub = s0.elapsed_time(s1) * 1e-3 / 20

        # the selection sweep alone: argmax only (no volume), the frame's maps, no exclusions
        sel_block = gh.peaks_tensor(nloc, dev)
        for _ in range(3):
            gh.decision(radar, grid, fmaps, interp, block=sel_block, write_volume=False, want_argmax=False)
        a0, a1 = ev(), ev()
        a0.record(stream)
        for _ in range(20):
            gh.decision(radar, grid, fmaps, interp, block=sel_block, write_volume=False, want_argmax=False)
        a1.record(stream)
        torch.cuda.synchronize()
        t_sel = a0.elapsed_time(a1) * 1e-3 / 20

        # the precision workload's sweep (K = 8, 256 x 256 x 32 x 32, complex64 maps): its
        # 268 MB volume is larger than the 256 MB Infinity Cache
        s3 = sc.make_scene(PRECISION_CFG, 0)
        r3 = gh.Radar.from_scene(s3)
        g3 = gh.grid_of(s3.grid)
        y3 = torch.from_numpy(s3.y).to(dev)
        z3 = gh.rd_maps(r3, y3)
        dec3 = torch.empty(tuple(s3.grid.n), dtype=torch.float32, device=dev)
        blk3 = gh.peaks_tensor(s3.grid.n[0] * s3.grid.n[1], dev)
        for _ in range(3):
            gh.decision(r3, g3, z3, interp, dec=dec3, block=blk3, want_argmax=False)
        p0, p1 = ev(), ev()
        p0.record(stream)
        for _ in range(10):
            gh.decision(r3, g3, z3, interp, dec=dec3, block=blk3, want_argmax=False)
        p1.record(stream)
        torch.cuda.synchronize()
        t3 = p0.elapsed_time(p1) * 1e-3 / 10
        bytes3 = 4 * s3.grid.size + z3.numel() * 8 + 16 * blk3.shape[0]
        del z3
        # the BF16 direct decision on the same whole grid (volume written)
        ws3 = torch.empty(gh.direct_workspace_bytes(r3, g3, gh.GEMM_BF16), dtype=torch.uint8, device=dev)
        for _ in range(2):
            gh.direct_decision(r3, g3, y3, gemm=gh.GEMM_BF16, ws=ws3, dec=dec3, block=blk3, want_argmax=False)
        q0, q1 = ev(), ev()
        q0.record(stream)
        for _ in range(5):
            gh.direct_decision(r3, g3, y3, gemm=gh.GEMM_BF16, ws=ws3, dec=dec3, block=blk3, want_argmax=False)
        q1.record(stream)
        torch.cuda.synchronize()
        t_dir3 = q0.elapsed_time(q1) * 1e-3 / 5
        flop_dir3 = direct_flop(r3, s3.grid.n)
        del dec3, ws3, y3

        # the step's FP32 direct decision timed on its own, launches back to back (in the step it
        # runs beside the refinement)
        for _ in range(3):
            gh.direct_decision(radar, dgrid, y, ws=ws, dec=ddec, block=dblock, want_argmax=False)
        ef0, ef1 = ev(), ev()
        ef0.record(stream)
        for _ in range(10):
            gh.direct_decision(radar, dgrid, y, ws=ws, dec=ddec, block=dblock, want_argmax=False)
        ef1.record(stream)
        torch.cuda.synchronize()
        t_dir_f32 = ef0.elapsed_time(ef1) * 1e-3 / 10

        # the direct decision with BF16 matrix-core operands, timed on its own (not part of the step)
        ws_b = torch.empty(gh.direct_workspace_bytes(radar, dgrid, gh.GEMM_BF16), dtype=torch.uint8, device=dev)
        ddec_b = torch.empty_like(ddec)
        for _ in range(3):
            gh.direct_decision(radar, dgrid, y, gemm=gh.GEMM_BF16, ws=ws_b, dec=ddec_b, block=dblock, want_argmax=False)
        eb0, eb1 = ev(), ev()
        eb0.record(stream)
        for _ in range(10):
            gh.direct_decision(radar, dgrid, y, gemm=gh.GEMM_BF16, ws=ws_b, dec=ddec_b, block=dblock, want_argmax=False)
        eb1.record(stream)
        torch.cuda.synchronize()
        t_dir_bf16 = eb0.elapsed_time(eb1) * 1e-3 / 10
        err_bf16 = float((ddec_b.double() - ddec.double()).abs().max() / ddec.double().max())
        return {
            "ms_per_step_p10_p50_p90": [float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
            "ms_per_step_one_stream": one_ms,
            "copy_gbs": copy_gbs,
            "t_gh_sub": t_gh_sub,
            "t_dir_bf16": t_dir_bf16,
            "t_dir_f32": t_dir_f32,
            "t_dir_bf16_precision": t_dir3,
            "flop_dir_bf16_precision": flop_dir3,
            "err_bf16": err_bf16,
            "t_sel": t_sel,
            "precision": {"t": t3, "bytes": bytes3, "points": s3.grid.size, "k": r3.k},
            "factored": factored_timings(gh, torch, radar, grid, y, stream),
        }

    ms_step = wall / args.steps * 1e3
    pts_step = BOMP_ITERS * n_gh + n_dir     # the sweep of step 2 is the first selection's
    sweep_bytes = 4 * n_gh + radar.k * radar.nr * radar.nd * 8 + 16 * nloc
    achieved = sweep_bytes / t_sweep_launch / 1e9

    line = {
        "metric": "4D grid points/s, grid hopping vs direct on 1 MI355X at stated error",
        "value": pts_step / (ms_step * 1e-3),
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"paper-scale frame: K=4 RX, Ms=256 x Mc=128 complex64, 3 targets, SNR 10 dB, pad x4; "
                         f"grid hopping ({args.interp}) on 128x128x32x32, direct (FP32) on the 64x64x16x16 subgrid, "
                         f"Block-OMP x{BOMP_ITERS}, refinement of {BOMP_ITERS} cells"),
            "grid_points_per_step": pts_step,
            "gh_grid": list(s.grid.n),
            "direct_grid": list(dgrid_s.n),
            "interp": args.interp,
        },
        "step_launch": "hip_graph",
        "step_streams": args.streams,
        "graph_matches_eager": graph_matches_eager,
        "rows_ms": {"rd_maps": t_maps * 1e3, "gh_sweep": t_sweep * 1e3, "argmax": t_arg * 1e3,
                    "direct": t_dir * 1e3, "bomp_refine_rest": (t_total - t_maps - t_sweep - t_arg - t_dir) * 1e3},
        "gh_points_per_s": n_gh / (t_maps + t_sweep + t_arg),
        "gh_sweep_points_per_s": n_gh / t_sweep,
        "direct_points_per_s": n_dir / t_dir,
        "speedup_gh_over_direct_per_point": (n_gh / (t_maps + t_sweep + t_arg)) / (n_dir / t_dir),
        "rd_maps_gbs": (y.numel() * 8 + radar.k * radar.nr * radar.nd * 8) / t_maps / 1e9,
        "roofline": {"kernel": "gh_sweep_columns<bilinear>" if interp == gh.BILINEAR else "gh_sweep_columns<bicubic>",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic() if interp == gh.BILINEAR else None,
                     "algorithmic_bytes_per_launch": sweep_bytes,
                     "avg_launch_us": t_sweep_launch * 1e6},
    }
    # The sweep is limited by VALU issue and LDS, not HBM: the share of the
    # launch's CU-cycles (one VALU wave instruction per CU per cycle) that the
    # recorded VALU instruction count needs at the live launch time.
    valu = recorded_traffic("valu_insts_per_launch") if interp == gh.BILINEAR else None
    line["roofline"]["valu_issue_frac"] = (valu / CUS / (t_sweep_launch * CLOCK_HZ)) if valu else None

    if not args.step_only:
        x = side_measurements()
        line.update({
            "direct_bf16_points_per_s": n_dir / x["t_dir_bf16"],
            "direct_bf16_max_rel_diff_vs_f32": x["err_bf16"],
            # algorithmic matrix-core work (8 flops per complex multiply-add of both zooms)
            # against the dense BF16 peak, on the paper-scale subgrid and the precision grid
            "direct_bf16_mfma": {
                "unit": "TFLOP/s", "peak": BF16_PEAK_TFLOPS,
                "subgrid": {"us": x["t_dir_bf16"] * 1e6, "flop": direct_flop(radar, dgrid_s.n),
                            "achieved": direct_flop(radar, dgrid_s.n) / x["t_dir_bf16"] / 1e12,
                            "frac": direct_flop(radar, dgrid_s.n) / x["t_dir_bf16"] / 1e12 / BF16_PEAK_TFLOPS},
                "precision_grid": {"us": x["t_dir_bf16_precision"] * 1e6, "flop": x["flop_dir_bf16_precision"],
                                   "achieved": x["flop_dir_bf16_precision"] / x["t_dir_bf16_precision"] / 1e12,
                                   "frac": x["flop_dir_bf16_precision"] / x["t_dir_bf16_precision"] / 1e12
                                   / BF16_PEAK_TFLOPS}},
            # the step's FP32 direct decision alone, against the FP32 matrix peak
            "direct_f32_mfma": {
                "unit": "TFLOP/s", "peak": FP32_PEAK_TFLOPS, "us": x["t_dir_f32"] * 1e6,
                "flop": direct_flop(radar, dgrid_s.n),
                "achieved": direct_flop(radar, dgrid_s.n) / x["t_dir_f32"] / 1e12,
                "frac": direct_flop(radar, dgrid_s.n) / x["t_dir_f32"] / 1e12 / FP32_PEAK_TFLOPS},
            "speedup_gh_over_direct_same_subgrid": t_dir / x["t_gh_sub"],
            "ms_per_step_p10_p50_p90": x["ms_per_step_p10_p50_p90"],
            "ms_per_step_one_stream": x["ms_per_step_one_stream"],
            "copy_gbs": x["copy_gbs"],
            "factored": x["factored"],
        })
        line["roofline"]["frac_of_copy"] = achieved / x["copy_gbs"]
        # the Block-OMP selection sweeps write no volume: no HBM bytes to speak of;
        # their algorithmic FP32 work against the vector peak
        flops_sel = FLOP_PER_POINT_RX[args.interp] * radar.k * n_gh
        line["selection_sweep"] = {"avg_launch_us": x["t_sel"] * 1e6, "points_per_s": n_gh / x["t_sel"],
                                   "bound": "alu", "achieved": flops_sel / x["t_sel"] / 1e12,
                                   "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": flops_sel / x["t_sel"] / 1e12 / FP32_PEAK_TFLOPS,
                                   "flop_per_point_rx": FLOP_PER_POINT_RX[args.interp]}
        p = x["precision"]
        ach3 = p["bytes"] / p["t"] / 1e9
        line["roofline_precision_frame"] = {
            "kernel": line["roofline"]["kernel"], "workload": "K=8, Ms=64 x Mc=32, grid 256x256x32x32, volume written",
            "bound": "hbm", "achieved": ach3, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach3 / HBM_PEAK_GBS,
            "traffic": None, "algorithmic_bytes_per_launch": p["bytes"], "avg_launch_us": p["t"] * 1e6,
            "points_per_s": p["points"] / p["t"], "frac_of_copy": ach3 / x["copy_gbs"]}
    if not args.no_batch and not args.step_only:
        line["batch"] = batch_workload(gh, sc, torch, stream)

    if not args.no_cpu_baseline and not args.step_only:
        rng = np.random.default_rng(2024)
        gh_idx = rng.integers(0, n_gh, 4_000_000)     # about 10 s of one core's oracle work in all
        dir_idx = rng.integers(0, n_dir, 200_000)
        torch.cuda.synchronize()
        dv = dec.view(-1).cpu().numpy()
        ddv = ddec.view(-1).cpu().numpy()
        job = {"gh_idx": gh_idx, "dir_idx": dir_idx, "gh_gpu": dv[gh_idx].astype(np.float64),
               "dir_gpu": ddv[dir_idx].astype(np.float64), "gh_max": np.float64(dv.max()),
               "dir_max": np.float64(ddv.max()), "support": bomp.support.cpu().numpy(),
               "interp": np.int64(interp)}
        line["cpu_baseline"] = cpu_baseline(job)
        line["cpu_baseline_all_cores"] = cpu_baseline(job, parallel=True)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
