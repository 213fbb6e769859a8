#!/usr/bin/env python3
"""Write argmax_full_size.json: the FP64 oracle's maxima over the full workload grids.

Test infrastructure.  This script calls only the oracle package and the seeded
scene generator (which holds none of the method's arithmetic); nothing in it
comes from the GPU library.  The GPU parity tests read the file and require
the GPU's argmax cell to be the oracle's, or a reported near tie
(D_oracle(gpu cell) >= (1 - tau) D_oracle(oracle cell)), for the decisions
whose full volumes the oracle cannot recompute within a test's time:

  gh_cfg2_bilinear, gh_cfg2_bicubic   eq. (7) on the 128x128x32x32 grid of the
                                      paper-scale frame (4 RX, 256 x 128)
  direct_cfg2_subgrid                 the direct decision (scalar products with
                                      the atoms of eq. (3)) on its stride-2
                                      64x64x16x16 subgrid
  bomp_cfg2_bilinear                  three Block-OMP selections on the oracle's
                                      own residuals (grid hopping, bilinear)
  gh_cfg3_bilinear                    eq. (7) on the 256x256x32x32 grid of the
                                      precision frame (8 RX, 64 x 32)
  direct_cfg3                         the direct decision on that whole grid
  batch_bilinear                      eq. (7) per frame of the 64-frame batching
                                      workload: each frame's maximum

For every decision the file holds the maximum (value, lowest linear index) and
the runner-up (the largest value at any other cell), so a reader sees the
margin that the near-tie rule works against.  Ties go to the lowest linear
index (eqs. (5)-(6) take an argmax; the paper is silent on ties).  Each case
also records the SHA-256 of the complex64 frame it was computed from; the
tests refuse to compare against a golden whose frame the generator no longer
reproduces.

Usage: python tests/golden/make_argmax_golden.py [--jobs N] [--only name,...]
(about 10 minutes on 8 cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")        # one thread per pool worker
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import bomp as obomp, direct as odirect, gh as ogh, maps as omaps, radar as ordr  # noqa: E402
from paper_2307_16550_amd import scene as sc  # noqa: E402

OUT = os.path.join(HERE, "argmax_full_size.json")

_JOB = {}


def frame_sha(y) -> str:
    return hashlib.sha256(np.ascontiguousarray(np.asarray(y, np.complex64)).tobytes()).hexdigest()


def slab_grid(grid, ix):
    """The one-location-row sub-grid at x index ix (the same x value, bit for bit)."""
    x = ordr.grid_axes(grid)[0][ix]
    return sc.Grid((x, grid.lo[1], grid.lo[2], grid.lo[3]), (x, grid.hi[1], grid.hi[2], grid.hi[3]),
                   (1, grid.n[1], grid.n[2], grid.n[3]))


def top2(flat, base):
    """Largest two (value, index) of a flat slab, ties to the lowest index."""
    order = np.lexsort((np.arange(flat.size), -flat))[:2]
    return [(float(flat[i]), int(base + i)) for i in order]


def _slab_top(ix):
    j = _JOB
    g = slab_grid(j["grid"], ix)
    if j["kind"] == "direct":
        d = odirect.direct_decision(j["y"], j["radar"], g)
    else:
        d = ogh.gh_decision(j["z"], j["radar"], g, j["interp"])
    flat = d.ravel()
    for e in j["exclude"]:
        lo = ix * flat.size
        if lo <= e < lo + flat.size:
            flat[e - lo] = -np.inf
    return top2(flat, ix * flat.size)


def volume_top2(pool, kind, radar, grid, y=None, z=None, interp=ogh.BILINEAR, exclude=()):
    """(max, runner-up) of a whole decision volume, computed slab by slab in a process pool."""
    _JOB.clear()
    _JOB.update(kind=kind, radar=radar, grid=grid, y=y, z=z, interp=interp, exclude=list(exclude))
    cands = []
    for part in pool(list(range(grid.n[0]))):
        cands.extend(part)
    cands.sort(key=lambda c: (-c[0], c[1]))
    return cands[0], cands[1]


def entry(best, second, **extra):
    out = {"argmax": best[1], "value": best[0], "runner_up": second[1], "runner_up_value": second[0],
           "margin": 1.0 - second[0] / best[0]}
    out.update(extra)
    return out


def make_pool(jobs):
    def run(items):
        ctx = mp.get_context("fork")      # the workers inherit _JOB; only indices and results are pickled
        with ctx.Pool(jobs) as p:
            return p.map(_slab_top, items, chunksize=1)
    return run


def case_gh(pool, cfg, interp):
    s = sc.make_scene(cfg, 0)
    r = ordr.radar_from_scene(s)
    z = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    best, second = volume_top2(pool, "gh", r, s.grid, z=z, interp=interp)
    return entry(best, second, cfg=cfg, trial=0, interp=["bilinear", "bicubic"][interp], grid=list(s.grid.n),
                 frame_sha256=frame_sha(s.y))


def case_direct(pool, cfg):
    s = sc.make_scene(cfg, 0)
    r = ordr.radar_from_scene(s)
    g = sc.direct_grid(s, cfg)
    best, second = volume_top2(pool, "direct", r, g, y=s.y)
    return entry(best, second, cfg=cfg, trial=0, grid=list(g.n), frame_sha256=frame_sha(s.y))


def case_bomp(pool, cfg, iters, interp):
    """Block-OMP selections on the oracle's own FP64 residuals (grid hopping)."""
    s = sc.make_scene(cfg, 0)
    r = ordr.radar_from_scene(s)
    resid = s.y.astype(np.complex128)
    support, steps = [], []
    for _ in range(iters):
        z = omaps.rd_maps(resid, r.pad_r, r.pad_d, r.centered)
        best, second = volume_top2(pool, "gh", r, s.grid, z=z, interp=interp, exclude=support)
        support.append(best[1])
        _, resid = obomp.fit(s.y, r, s.grid, support)
        steps.append(entry(best, second))
    return {"cfg": cfg, "trial": 0, "interp": ["bilinear", "bicubic"][interp], "grid": list(s.grid.n),
            "frame_sha256": frame_sha(s.y), "selections": steps}


def case_batch(pool, interp):
    frames = []
    for f, s in enumerate(sc.make_batch()):
        r = ordr.radar_from_scene(s)
        z = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
        best, second = volume_top2(pool, "gh", r, s.grid, z=z, interp=interp)
        frames.append(entry(best, second, frame=f, grid=list(s.grid.n), frame_sha256=frame_sha(s.y)))
        print(f"  batch frame {f}: {best[1]} margin {frames[-1]['margin']:.3g}", flush=True)
    return {"trial": 0, "interp": ["bilinear", "bicubic"][interp], "frames": frames}


CASES = {
    "gh_cfg2_bilinear": lambda p: case_gh(p, 2, ogh.BILINEAR),
    "gh_cfg2_bicubic": lambda p: case_gh(p, 2, ogh.BICUBIC),
    "direct_cfg2_subgrid": lambda p: case_direct(p, 2),
    "bomp_cfg2_bilinear": lambda p: case_bomp(p, 2, 3, ogh.BILINEAR),
    "gh_cfg3_bilinear": lambda p: case_gh(p, 3, ogh.BILINEAR),
    "direct_cfg3": lambda p: case_direct(p, 3),
    "batch_bilinear": lambda p: case_batch(p, ogh.BILINEAR),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--only", default="")
    a = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    pool = make_pool(a.jobs)
    names = [n for n in a.only.split(",") if n] or list(CASES)
    for name in names:
        t0 = time.perf_counter()
        data[name] = CASES[name](pool)
        print(f"{name}: {time.perf_counter() - t0:.0f} s", flush=True)
        data["_about"] = ("FP64 oracle maxima over the full workload grids, written by "
                          "tests/golden/make_argmax_golden.py from the oracle and the seeded generator only")
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()
