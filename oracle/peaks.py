"""Block and global argmax of a decision volume (test infrastructure; see the package header).

The estimators of the paper take the argmax of their decision function over
the grid (eqs. (4)-(6)).  A "block" is one location's velocity slab (Nvx*Nvy
consecutive entries of the volume in (ix, iy, ivx, ivy) order, vy fastest).
Ties go to the lowest linear index (the paper is silent on ties).
"""
from __future__ import annotations

import numpy as np


def first_max(values: np.ndarray):
    """(max value, lowest index attaining it) of a 1D array, written out as a scan."""
    best = -np.inf
    where = -1
    for i, v in enumerate(values.tolist()):
        if v > best:
            best, where = v, i
    return best, where


def block_peaks(d: np.ndarray):
    """Per-location (value, linear index into the volume) of the velocity-slab maximum."""
    nloc = d.shape[0] * d.shape[1]
    nv = d.shape[2] * d.shape[3]
    flat = d.reshape(nloc, nv)
    top = flat.max(axis=1)
    vals = np.empty(nloc)
    idx = np.empty(nloc, dtype=np.int64)
    for b in range(nloc):
        hits = np.nonzero(flat[b] == top[b])[0]
        vals[b] = top[b]
        idx[b] = b * nv + int(hits[0])
    return vals, idx


def global_peak(d: np.ndarray, exclude=()):
    """(value, linear index) of the volume maximum, skipping the linear indices in `exclude`."""
    flat = np.array(d, dtype=np.float64).ravel()
    for e in exclude:
        flat[int(e)] = -np.inf
    top = flat.max()
    return float(top), int(np.nonzero(flat == top)[0][0])
