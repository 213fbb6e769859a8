"""Pins of the full-size golden argmax file (tests/golden/argmax_full_size.json)
against the oracle itself: the seeded generator still draws the recorded
frames, and the oracle's decision over the whole location row (x index) that
holds each recorded maximum peaks at the recorded cell with the recorded
value.  The full volumes take minutes; one row per entry takes seconds."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import _golden  # noqa: E402
import make_argmax_golden as mk  # noqa: E402
from oracle import bomp as obomp, direct as odirect, gh as ogh, maps as omaps, radar as ord_  # noqa: E402
from paper_2307_16550_amd import scene as sc  # noqa: E402


def row_peak(kind, r, grid, idx, y=None, z=None, interp=ogh.BILINEAR, exclude=()):
    """(max, runner-up) of the oracle decision over the location row holding linear index idx."""
    ix = idx // (grid.n[1] * grid.n[2] * grid.n[3])
    g = mk.slab_grid(grid, ix)
    d = odirect.direct_decision(y, r, g) if kind == "direct" else ogh.gh_decision(z, r, g, interp)
    flat = d.ravel().copy()
    base = ix * flat.size
    for e in exclude:
        if base <= e < base + flat.size:
            flat[e - base] = -np.inf
    return mk.top2(flat, base)


def check(gold, best):
    assert best[1] == gold["argmax"]
    assert abs(best[0] - gold["value"]) <= 1e-12 * gold["value"]


@pytest.mark.parametrize("name,cfg,interp", [("gh_cfg2_bilinear", 2, ogh.BILINEAR), ("gh_cfg2_bicubic", 2, ogh.BICUBIC),
                                             ("gh_cfg3_bilinear", 3, ogh.BILINEAR)])
def test_gh_golden_rows(name, cfg, interp):
    s = sc.make_scene(cfg, 0)
    gold = _golden.load(name, s.y)
    r = ord_.radar_from_scene(s)
    z = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    check(gold, row_peak("gh", r, s.grid, gold["argmax"], z=z, interp=interp)[0])


@pytest.mark.parametrize("name,cfg", [("direct_cfg2_subgrid", 2), ("direct_cfg3", 3)])
def test_direct_golden_rows(name, cfg):
    s = sc.make_scene(cfg, 0)
    gold = _golden.load(name, s.y)
    r = ord_.radar_from_scene(s)
    check(gold, row_peak("direct", r, sc.direct_grid(s, cfg), gold["argmax"], y=s.y)[0])


def test_bomp_golden_rows():
    """Each recorded selection is the maximum of its row on the oracle's own residual
    (the residual of the least-squares fit over the selections before it)."""
    s = sc.make_scene(2, 0)
    sel = _golden.load("bomp_cfg2_bilinear", s.y)["selections"]
    r = ord_.radar_from_scene(s)
    support = []
    for g in sel:
        resid = obomp.fit(s.y, r, s.grid, support)[1] if support else s.y.astype(np.complex128)
        z = omaps.rd_maps(resid, r.pad_r, r.pad_d, r.centered)
        check(g, row_peak("gh", r, s.grid, g["argmax"], z=z, exclude=support)[0])
        support.append(g["argmax"])
    assert sel[0]["argmax"] == _golden.load("gh_cfg2_bilinear")["argmax"]


@pytest.mark.parametrize("frame", [0, 21, 63])
def test_batch_golden_rows(frame):
    s = sc.make_batch()[frame]
    gold = _golden.load("batch_bilinear")["frames"][frame]
    assert gold["frame_sha256"] == _golden.frame_sha(s.y)
    r = ord_.radar_from_scene(s)
    z = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    check(gold, row_peak("gh", r, s.grid, gold["argmax"], z=z)[0])


def test_golden_runner_up_is_below_the_maximum():
    with open(_golden.PATH) as fh:
        import json
        data = json.load(fh)
    entries = [v for k, v in data.items() if k.startswith(("gh_", "direct_"))]
    entries += data["bomp_cfg2_bilinear"]["selections"] + data["batch_bilinear"]["frames"]
    for e in entries:
        assert e["runner_up"] != e["argmax"] and e["runner_up_value"] <= e["value"]
