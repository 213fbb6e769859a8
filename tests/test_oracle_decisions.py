"""Pins of the oracle's grid-hopping and direct decisions and of its argmax."""
import math

import numpy as np
import pytest

from oracle import direct, gh, maps, peaks, radar as rd
from paper_2307_16550_amd import scene as sc
from _fixtures import node_aligned_scene, true_cell


def small_radar(centered=1, ms=16, mc=8, k=2, pad=4):
    return rd.Radar(24e9, 250e6, 256e-6, sc.C_LIGHT, ms, mc, pad, pad, np.zeros(2),
                    np.array([[0.0, 3.0], [0.0, -4.0], [0.0, 7.0]])[:k], centered)


@pytest.mark.parametrize("kind", [gh.BILINEAR, gh.BICUBIC])
@pytest.mark.parametrize("centered", [0, 1])
def test_interpolation_exact_at_nodes(kind, centered):
    rng = np.random.default_rng(5)
    zq = rng.standard_normal((64, 32)) + 1j * rng.standard_normal((64, 32))
    i = rng.integers(-70, 140, size=50)
    l = rng.integers(-40, 70, size=50)
    got = gh.interpolate(zq, i.astype(float), l.astype(float), kind, 16, 8, centered)
    assert np.allclose(got, maps.node_value(zq, i, l, 16, 8, centered), rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", [gh.BILINEAR, gh.BICUBIC])
def test_weights_are_a_partition_of_unity(kind):
    t = np.linspace(-3.2, 7.9, 101)
    _, ws = gh.taps_and_weights(t, kind)
    assert np.allclose(sum(ws), 1.0, atol=1e-14)


def test_keys_kernel_values():
    # Keys (a = -1/2): W(0)=1, W(1)=W(2)=0, W(1/2)=9/16, W(3/2)=-1/16
    assert gh.keys_weight(0.0) == 1.0
    assert abs(gh.keys_weight(1.0)) < 1e-15 and abs(gh.keys_weight(2.0)) < 1e-15
    assert abs(gh.keys_weight(0.5) - 9 / 16) < 1e-15 and abs(gh.keys_weight(1.5) + 1 / 16) < 1e-15


def test_bilinear_reproduces_affine_and_keys_reproduces_quadratic_maps():
    ii, ll = np.meshgrid(np.arange(64.0), np.arange(32.0), indexing="ij")
    affine = (0.3 - 1.1j) + (0.25 + 0.5j) * ii - (0.75 - 0.1j) * ll
    quad = affine + (0.01 + 0.02j) * ii ** 2 - 0.03 * ii * ll + (0.05 - 0.01j) * ll ** 2
    rng = np.random.default_rng(6)
    tr = rng.uniform(2, 60, 200)
    td = rng.uniform(2, 28, 200)
    exp_aff = (0.3 - 1.1j) + (0.25 + 0.5j) * tr - (0.75 - 0.1j) * td
    exp_quad = exp_aff + (0.01 + 0.02j) * tr ** 2 - 0.03 * tr * td + (0.05 - 0.01j) * td ** 2
    assert np.allclose(gh.interpolate(affine, tr, td, gh.BILINEAR, 16, 8, 0), exp_aff, atol=1e-11)
    assert np.allclose(gh.interpolate(quad, tr, td, gh.BICUBIC, 16, 8, 0), exp_quad, atol=1e-10)
    # bilinear is not exact on a quadratic (the test above is not vacuous)
    assert not np.allclose(gh.interpolate(quad, tr, td, gh.BILINEAR, 16, 8, 0), exp_quad, atol=1e-3)


@pytest.mark.parametrize("kind", [gh.BILINEAR, gh.BICUBIC])
@pytest.mark.parametrize("centered", [0, 1])
def test_periodicity_in_doppler(kind, centered):
    rng = np.random.default_rng(7)
    zq = rng.standard_normal((64, 32)) + 1j * rng.standard_normal((64, 32))
    tr = rng.uniform(3, 60, 40)
    td = rng.uniform(-40, 40, 40)
    a = gh.interpolate(zq, tr, td, kind, 16, 8, centered)
    b = gh.interpolate(zq, tr, td + 32, kind, 16, 8, centered)
    sign = -1.0 if centered else 1.0      # (-1)^(Mc-1) with Mc = 8
    assert np.allclose(b, sign * a, atol=1e-12)


def test_centring_removes_interpolation_loss_of_a_tone():
    """A tone midway between Doppler nodes: centred maps keep more energy under bilinear interpolation."""
    ms, mc, pad = 16, 8, 4
    r = small_radar(ms=ms, mc=mc)
    fr, fd = 5.0 / (pad * ms), 2.5 / (pad * mc)
    s = np.arange(ms)[None, :]
    m = np.arange(mc)[:, None]
    y = np.exp(2j * np.pi * (fr * s + fd * m))[None]
    e = {}
    for cen in (0, 1):
        z = maps.rd_maps(y, pad, pad, cen)
        e[cen] = abs(gh.interpolate(z[0], 5.0, 2.5, gh.BILINEAR, ms, mc, cen)) ** 2
    exact = abs(direct.correlation(y[0], fr, fd)) ** 2
    assert e[1] > e[0] and e[1] <= exact * (1 + 1e-12)


def brute_direct(y, r, pts):
    out = []
    for (x, y_, vx, vy) in pts:
        tot = 0.0
        for q in range(r.k):
            fr, fd = rd.sensed_freqs(r, q, x, y_, vx, vy)
            acc = 0j
            for m in range(r.mc):
                for s in range(r.ms):
                    acc += complex(y[q, m, s]) * complex(np.exp(-2j * math.pi * (fr * s + fd * m)))
            tot += abs(acc) ** 2
        out.append(tot)
    return np.array(out)


def test_direct_equals_brute_force_quadruple_sum():
    r = small_radar(ms=8, mc=4, k=2)
    rng = np.random.default_rng(8)
    y = (rng.standard_normal((2, 4, 8)) + 1j * rng.standard_normal((2, 4, 8))).astype(np.complex64)
    grid = sc.Grid((6.0, -3.0, -5.0, -4.0), (14.0, 5.0, 6.0, 7.0), (4, 4, 2, 2))
    vol = direct.direct_decision(y, r, grid)
    ax = rd.grid_axes(grid)
    pts = [(a, b, c, d) for a in ax[0] for b in ax[1] for c in ax[2] for d in ax[3]]
    ref = brute_direct(y, r, pts)
    assert np.allclose(vol.ravel(), ref, rtol=1e-12, atol=0)
    p = np.array(pts)
    assert np.allclose(direct.direct_points(y, r, p[:, 0], p[:, 1], p[:, 2], p[:, 3]), ref, rtol=1e-12)


def test_location_energy_is_eq5_objective():
    r = small_radar(ms=8, mc=4, k=2)
    rng = np.random.default_rng(9)
    y = rng.standard_normal((2, 4, 8)) + 1j * rng.standard_normal((2, 4, 8))
    x, y_ = 9.3, 1.7
    ref = 0.0
    for q in range(2):
        fr, _ = rd.sensed_freqs(r, q, x, y_, 0.0, 0.0)
        for m in range(4):
            acc = sum(y[q, m, s] * np.exp(-2j * math.pi * fr * s) for s in range(8))
            ref += abs(acc) ** 2
    assert abs(direct.location_energy(y, r, x, y_) - ref) < 1e-12 * ref


@pytest.mark.parametrize("trial", range(4))
def test_cauchy_schwarz_bound_and_on_grid_recovery_direct(trial):
    s = sc.make_scene(1, trial, snr_db=math.inf, on_grid=True)
    r = rd.radar_from_scene(s)
    vol = direct.direct_decision(s.y, r, s.grid)
    bound = np.sum(np.abs(s.alpha[0]) ** 2) * (s.ms * s.mc) ** 2
    assert vol.max() <= bound * (1 + 1e-6)
    cell = true_cell(s)
    assert abs(vol.ravel()[cell] - bound) <= 1e-6 * bound
    assert peaks.global_peak(vol)[1] == cell


@pytest.mark.parametrize("trial", range(3))
@pytest.mark.parametrize("centered", [0, 1])
def test_node_aligned_scene_grid_hopping_recovers_truth(trial, centered):
    s = node_aligned_scene(1, trial, centered=centered)
    r = rd.radar_from_scene(s)
    z = maps.rd_maps(s.y, r.pad_r, r.pad_d, centered)
    cell = true_cell(s)
    bound = np.sum(np.abs(s.alpha[0]) ** 2) * (s.ms * s.mc) ** 2
    for kind in (gh.BILINEAR, gh.BICUBIC):
        p = rd.grid_point(s.grid, cell)
        val = gh.gh_points(z, r, *p, kind)
        assert abs(val - bound) <= 1e-6 * bound
        assert abs(val - direct.direct_points(s.y, r, *p)) <= 1e-6 * bound
    vol = gh.gh_decision(z, r, s.grid, gh.BILINEAR)
    assert vol.max() <= bound * (1 + 1e-6)
    assert peaks.global_peak(vol)[1] == cell


def test_gh_equals_direct_wherever_coordinates_are_nodes_for_any_data():
    s = node_aligned_scene(1, 5, snr_db=0.0)      # noisy data: the identity holds for any frame
    r = rd.radar_from_scene(s)
    z = maps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    p = rd.grid_point(s.grid, true_cell(s))
    for kind in (gh.BILINEAR, gh.BICUBIC):
        a = gh.gh_points(z, r, *p, kind)
        b = direct.direct_points(s.y, r, *p)
        assert abs(a - b) <= 1e-9 * b


def test_gh_decision_matches_pointwise_evaluation():
    s = sc.make_scene(1, 0)
    r = rd.radar_from_scene(s)
    z = maps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    small = sc.Grid(s.grid.lo, s.grid.hi, (3, 4, 2, 5))
    vol = gh.gh_decision(z, r, small, gh.BICUBIC)
    rng = np.random.default_rng(10)
    for idx in rng.integers(0, small.size, 10):
        assert abs(vol.ravel()[idx] - gh.gh_points(z, r, *rd.grid_point(small, int(idx)), gh.BICUBIC)) < 1e-9 * vol.max()


def test_block_peaks_and_ties():
    d = np.zeros((2, 3, 2, 2))
    d[0, 0] = [[1.0, 3.0], [3.0, 2.0]]          # tie inside a block: lowest index (1) wins
    d[1, 2] = [[5.0, 5.0], [0.0, 5.0]]
    d[0, 1, 1, 1] = 5.0                          # global tie with block (1,2): lowest linear index wins
    vals, idx = peaks.block_peaks(d)
    assert idx[0] == 1 and vals[0] == 3.0
    assert idx[5] == 5 * 4 + 0 and vals[5] == 5.0
    assert idx[1] == 1 * 4 + 3
    assert peaks.global_peak(d) == (5.0, 7)
    assert peaks.global_peak(d, exclude=[7]) == (5.0, 20)
    assert peaks.first_max(np.array([0.5, 2.0, -1.0, 2.0])) == (2.0, 1)
