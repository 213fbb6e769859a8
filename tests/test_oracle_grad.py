"""Pins of the oracle's decision gradients (oracle/grad.py).

Each analytic gradient is checked against central finite differences of the
oracle's own decision functions in FP64 (which share no derivative code with
it), with h = 1e-4 m and m/s as stated for the differentiation axis, and
against a stationarity property: the direct decision of a noise-free single
target has zero gradient at the true (x, v).
"""
import copy
import math

import numpy as np
import pytest

from oracle import direct, gh, grad, maps, radar as rd
from paper_2307_16550_amd import scene as sc

H = 1e-4


def fd_theta(fun, theta):
    g = np.zeros(4)
    for a in range(4):
        e = np.zeros(4)
        e[a] = H
        g[a] = (fun(theta + e) - fun(theta - e)) / (2 * H)
    return g


def with_rx(r: rd.Radar, q: int, delta) -> rd.Radar:
    r2 = copy.copy(r)
    r2.rx = r.rx.copy()
    r2.rx[q] = r2.rx[q] + delta
    return r2


def points_near_target(s, n, seed):
    rng = np.random.default_rng(seed)
    t = np.concatenate([s.pos[0], s.vel[0]])
    return [t + rng.uniform(-0.4, 0.4, 4) * np.array([0.6, 0.6, 0.6, 0.6]) for _ in range(n)]


def test_direct_gradient_matches_finite_differences():
    s = sc.make_scene(1, 0, ms=32, mc=16)
    r = rd.radar_from_scene(s)
    f = lambda th: float(direct.direct_points(s.y, r, *th))
    for th in points_near_target(s, 4, 1):
        d, g, g_rx = grad.direct_value_grad(s.y, r, th)
        assert abs(d - f(th)) <= 1e-12 * d
        gf = fd_theta(f, th)
        assert np.max(np.abs(g - gf)) <= 1e-5 * np.max(np.abs(g)), (g, gf)
        for q in range(r.k):
            for a in range(2):
                e = np.zeros(2)
                e[a] = H
                fp = float(direct.direct_points(s.y, with_rx(r, q, e), *th))
                fm = float(direct.direct_points(s.y, with_rx(r, q, -e), *th))
                assert abs(g_rx[q, a] - (fp - fm) / (2 * H)) <= 1e-5 * np.max(np.abs(g)), (q, a)


def test_direct_gradient_vanishes_at_noise_free_truth():
    s = sc.make_scene(1, 3, snr_db=math.inf, ms=32, mc=16)
    r = rd.radar_from_scene(s)
    truth = np.concatenate([s.pos[0], s.vel[0]])
    _, g0, g0_rx = grad.direct_value_grad(s.y, r, truth)
    _, g1, _ = grad.direct_value_grad(s.y, r, truth + np.array([0.05, -0.05, 0.05, 0.05]))
    assert np.max(np.abs(g0)) <= 1e-7 * np.max(np.abs(g1))
    # moving a receiver away from its true position can only lower the matched energy
    assert np.max(np.abs(g0_rx)) <= 1e-7 * np.max(np.abs(g1))


@pytest.mark.parametrize("kind", [gh.BILINEAR, gh.BICUBIC])
def test_gh_gradient_matches_finite_differences(kind):
    s = sc.make_scene(1, 2, ms=32, mc=16)
    r = rd.radar_from_scene(s)
    z = maps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    f = lambda th: float(gh.gh_points(z, r, *th, kind))
    checked = 0
    for th in points_near_target(s, 12, 2):
        # bilinear: keep both coordinates of every receiver away from a node (the
        # derivative jumps there), so the difference quotient stays within one cell
        ok = True
        for q in range(r.k):
            tr, td = rd.bin_coords(r, q, *th)
            for t in (tr, td):
                fr = t - math.floor(t)
                ok &= 0.01 < fr < 0.99
        if kind == gh.BILINEAR and not ok:
            continue
        d, g, g_rx = grad.gh_value_grad(z, r, th, kind)
        assert abs(d - f(th)) <= 1e-12 * d
        gf = fd_theta(f, th)
        scale = np.max(np.abs(g))
        assert np.max(np.abs(g - gf)) <= 2e-4 * scale, (g, gf)
        for q in range(r.k):
            for a in range(2):
                e = np.zeros(2)
                e[a] = H
                fp = float(gh.gh_points(z, with_rx(r, q, e), *th, kind))
                fm = float(gh.gh_points(z, with_rx(r, q, -e), *th, kind))
                assert abs(g_rx[q, a] - (fp - fm) / (2 * H)) <= 2e-4 * scale, (q, a)
        checked += 1
    assert checked >= 3


def test_keys_derivative_matches_difference_quotient():
    d = np.linspace(-2.2, 2.2, 441)
    d = d[np.abs(np.abs(d) - 1.0) > 1e-3]
    h = 1e-6
    fd = (gh.keys_weight(d + h) - gh.keys_weight(d - h)) / (2 * h)
    assert np.max(np.abs(grad.keys_derivative(d) - fd)) <= 1e-6
