"""The FP64 oracle's maxima over the full workload grids (tests/golden/argmax_full_size.json).

The file is written by tests/golden/make_argmax_golden.py, which calls only the
oracle and the seeded generator.  `load` checks that the generator still
reproduces the frame a golden entry was computed from (SHA-256 of the
complex64 frame); `check` applies the argmax rule: the GPU cell must be the
oracle's cell, or a reported near tie, D_oracle(gpu cell) >= (1 - tau) times
the oracle's maximum, where D_oracle(gpu cell) is recomputed by the oracle at
that one cell.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "argmax_full_size.json")
_CACHE = {}


def frame_sha(y) -> str:
    return hashlib.sha256(np.ascontiguousarray(np.asarray(y, np.complex64)).tobytes()).hexdigest()


def load(name: str, y=None):
    if not _CACHE:
        with open(PATH) as fh:
            _CACHE.update(json.load(fh))
    g = _CACHE[name]
    if y is not None:
        assert g["frame_sha256"] == frame_sha(y), f"golden {name}: the generator no longer draws the same frame"
    return g


def check(gpu_idx: int, golden: dict, oracle_at, tau: float, label: str) -> int:
    """0 when the cells are identical, 1 for a reported near tie; fails otherwise."""
    if int(gpu_idx) == int(golden["argmax"]):
        return 0
    v = float(oracle_at(int(gpu_idx)))
    print(f"[near-tie] {label}: gpu cell {gpu_idx} oracle cell {golden['argmax']} "
          f"oracle values {v:.9g} vs {golden['value']:.9g} (bar {tau:g})", flush=True)
    assert v >= (1.0 - tau) * float(golden["value"]), f"{label}: argmax differs beyond the near-tie bar"
    return 1
