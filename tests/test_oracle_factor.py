"""Pins of the oracle's factorised decisions and polar rule (oracle/factor.py).

* range spectra: the brute-force DFT on a tiny frame, and the 2D maps (an
  independent route: the library 2D FFT) as their DFT over chirps;
* polar rule: exact at the three taps and centred on the nearest bin; its
  angle against the circumcircle of the three atoms, computed geometrically
  in R^(2 Ms); on pure tones it is far more accurate than linear
  interpolation, and the computed angle beats perturbed angles;
* location energy: the closed form Mc Ms^2 sum |alpha_q|^2 at a noise-free
  target, and Cauchy-Schwarz against the joint decision,
  D_dir(x, v) <= Mc E(x), with equality at the noise-free truth;
* grid hopping equals direct where the coordinates fall on map nodes (the
  node-aligned scene), for every range rule;
* the nearest-bin velocity decision against a brute-force DFT over chirps;
* the factorised estimate recovers the true cell of noise-free scenes.
"""
import math

import numpy as np
import pytest

from oracle import direct, factor, maps, radar as rd
from paper_2307_16550_amd import scene as sc
from _fixtures import node_aligned_scene, true_cell

KINDS = [factor.BILINEAR, factor.BICUBIC, factor.POLAR]


@pytest.mark.parametrize("centered", [0, 1])
def test_range_spectra_brute_force(centered):
    rng = np.random.default_rng(1)
    y = rng.standard_normal((2, 4, 8)) + 1j * rng.standard_normal((2, 4, 8))
    z = factor.range_spectra(y, 2, centered)
    nr, ms = 16, 8
    c = (ms - 1) / 2.0 if centered else 0.0
    for q in range(2):
        for m in range(4):
            for i in range(nr):
                ref = sum(y[q, m, s] * np.exp(-2j * np.pi * i * (s - c) / nr) for s in range(ms))
                assert abs(z[q, m, i] - ref) <= 1e-12 * 8


@pytest.mark.parametrize("centered", [0, 1])
def test_range_spectra_against_maps(centered):
    rng = np.random.default_rng(2)
    y = rng.standard_normal((2, 8, 16)) + 1j * rng.standard_normal((2, 8, 16))
    zr = factor.range_spectra(y, 4, centered)
    z2 = maps.rd_maps(y, 4, 2, centered)
    nd, mc = 16, 8
    cm = (mc - 1) / 2.0 if centered else 0.0
    m = np.arange(mc)
    for l in range(nd):
        ref = np.einsum("qmi,m->qi", zr, np.exp(-2j * np.pi * l * (m - cm) / nd))
        assert np.max(np.abs(z2[:, :, l] - ref)) <= 1e-10 * np.max(np.abs(z2))


def test_polar_exact_at_taps():
    for theta in (0.3, 0.6, 2.0):
        for tau, want in ((-1.0, (1, 0, 0)), (0.0, (0, 1, 0)), (1.0, (0, 0, 1))):
            w = factor.polar_weights(tau, theta)
            assert np.allclose(w, want, atol=1e-14)
        w = factor.polar_weights(np.linspace(-0.5, 0.5, 11), theta)
        assert np.allclose(w[0] + w[1] + w[2], 1.0, atol=1e-14)


def test_polar_taps_centre_on_the_nearest_bin():
    """The index set is the nearest bin and its two neighbours: the dominant weight
    sits on the bin nearest the coordinate."""
    theta = factor.polar_theta(64, 4, 1)
    for t in np.random.default_rng(9).uniform(3.0, 60.0, 200):
        taps, ws = factor.range_taps(t, factor.POLAR, theta)
        k = int(np.argmax(np.abs(np.array(ws, dtype=np.float64))))
        assert abs(int(taps[k]) - t) <= 0.5


def atom_vec(ms, nr, centered, t):
    s = np.arange(ms)
    c = (ms - 1) / 2.0 if centered else 0.0
    a = np.exp(2j * np.pi * t * (s - c) / nr)
    return np.concatenate([a.real, a.imag])


@pytest.mark.parametrize("ms,pad,centered", [(64, 4, 1), (256, 4, 1), (64, 2, 0), (32, 8, 1), (128, 1, 1)])
def test_polar_angle_is_the_circumcircle_angle(ms, pad, centered):
    nr = ms * pad
    p0, p1, p2 = (atom_vec(ms, nr, centered, 10.0 + t) for t in (-1.0, 0.0, 1.0))
    # circumcentre of three points in R^n: C = p0 + a u + b v in their plane
    u, v = p1 - p0, p2 - p0
    uu, vv, uv = u @ u, v @ v, u @ v
    den = 2.0 * (uu * vv - uv * uv)
    a = vv * (uu - uv) / den
    b = uu * (vv - uv) / den
    c = p0 + a * u + b * v
    r1, r2 = p1 - c, p2 - c
    ang = math.acos(np.clip(r1 @ r2 / math.sqrt((r1 @ r1) * (r2 @ r2)), -1, 1))
    assert abs(ang - factor.polar_theta(ms, pad, centered)) <= 1e-9


def tone_errors(ms, pad, rule_theta, kind, n=200):
    """Max |interpolated - exact| / Ms of one chirp's correlation with a pure tone at random offsets."""
    nr = ms * pad
    rng = np.random.default_rng(3)
    worst = 0.0
    for f_bins in rng.uniform(20.0, 40.0, n):
        y = np.exp(2j * np.pi * f_bins * np.arange(ms) / nr)[None, None, :]
        z = factor.range_spectra(y, pad, 1)[0]
        got = factor.chirp_values(z, f_bins, kind, ms, 1, rule_theta)[0]
        exact = np.sum(y[0, 0] * np.exp(-2j * np.pi * f_bins * (np.arange(ms) - (ms - 1) / 2.0) / nr))
        worst = max(worst, abs(got - exact) / ms)
    return worst


@pytest.mark.parametrize("ms,pad", [(64, 4), (256, 4), (64, 2)])
def test_polar_accuracy_on_tones(ms, pad):
    theta = factor.polar_theta(ms, pad, 1)
    e_polar = tone_errors(ms, pad, theta, factor.POLAR)
    e_lin = tone_errors(ms, pad, None, factor.BILINEAR)
    assert e_polar <= 0.1 * e_lin, (e_polar, e_lin)
    for scale in (0.8, 1.25):
        assert e_polar < tone_errors(ms, pad, theta * scale, factor.POLAR)


def test_location_energy_closed_form_and_cauchy_schwarz():
    s = sc.make_scene(1, 4, snr_db=math.inf, ms=32, mc=16)
    r = rd.radar_from_scene(s)
    p, v = s.pos[0], s.vel[0]
    e = direct.location_energy(s.y, r, p[0], p[1])
    want = r.mc * r.ms ** 2 * float(np.sum(np.abs(s.alpha[0]) ** 2))
    assert abs(e - want) <= 1e-5 * want        # the frame is stored in complex64
    d = direct.direct_points(s.y, r, p[0], p[1], v[0], v[1])
    assert abs(d - r.mc * e) <= 1e-5 * d
    noisy = sc.make_scene(1, 5, ms=32, mc=16)
    rn = rd.radar_from_scene(noisy)
    rng = np.random.default_rng(6)
    for _ in range(20):
        x = rng.uniform([5, -10], [25, 10])
        vv = rng.uniform(-10, 10, 2)
        dd = direct.direct_points(noisy.y, rn, x[0], x[1], vv[0], vv[1])
        assert dd <= rn.mc * direct.location_energy(noisy.y, rn, x[0], x[1]) * (1 + 1e-12)


@pytest.mark.parametrize("kind", KINDS)
def test_gh_equals_direct_on_nodes(kind):
    s = node_aligned_scene(1, 2, snr_db=20.0)
    r = rd.radar_from_scene(s)
    zr = factor.range_spectra(s.y, r.pad_r, r.centered)
    cell = true_cell(s)
    g = s.grid
    nv = g.n[2] * g.n[3]
    loc = cell // nv
    ix, iy = divmod(loc, g.n[1])
    one = sc.Grid((g.axis(0)[ix], g.axis(1)[iy], g.lo[2], g.lo[3]), (g.axis(0)[ix], g.axis(1)[iy], g.hi[2], g.hi[3]),
                  (1, 1, g.n[2], g.n[3]))
    e_gh = factor.gh_location_energy(zr, r, one, kind)[0, 0]
    e_dir = factor.direct_location_energy(s.y, r, one)[0, 0]
    assert abs(e_gh - e_dir) <= 1e-9 * e_dir
    # nearest-bin velocity equals the exact decision at the node-aligned true velocity
    vgh = factor.gh_velocity(zr, r, g, loc, kind).ravel()[cell % nv]
    vdir = factor.direct_velocity(s.y, r, g, loc).ravel()[cell % nv]
    assert abs(vgh - vdir) <= 1e-9 * vdir


def test_gh_velocity_against_brute_force_dft():
    s = sc.make_scene(1, 7, ms=32, mc=16, n=(6, 6, 5, 7))
    r = rd.radar_from_scene(s)
    zr = factor.range_spectra(s.y, r.pad_r, r.centered)
    loc = 17
    got = factor.gh_velocity(zr, r, s.grid, loc, factor.BICUBIC)
    ax = rd.grid_axes(s.grid)
    ix, iy = divmod(loc, s.grid.n[1])
    cm = (r.mc - 1) / 2.0
    want = np.zeros(got.shape)
    for q in range(r.k):
        tr, _ = rd.bin_coords(r, q, ax[0][ix], ax[1][iy], 0.0, 0.0)
        g = factor.chirp_values(zr[q], float(tr), factor.BICUBIC, r.ms, r.centered, None)
        for a, vx in enumerate(ax[2]):
            for b, vy in enumerate(ax[3]):
                _, td = rd.bin_coords(r, q, ax[0][ix], ax[1][iy], vx, vy)
                l = math.floor(td + 0.5)
                c = sum(g[m] * np.exp(-2j * np.pi * l * (m - cm) / r.nd) for m in range(r.mc))
                want[a, b] += abs(c) ** 2
    assert np.max(np.abs(got - want)) <= 1e-10 * want.max()


def test_factored_estimate_recovers_noise_free_targets():
    s = sc.make_scene(1, 8, snr_db=math.inf, on_grid=True, n=(16, 16, 8, 8))
    r = rd.radar_from_scene(s)
    cell = true_cell(s)
    e = factor.direct_location_energy(s.y, r, s.grid)
    il, iv, idx, _, _ = factor.factored_estimate(e, lambda l: factor.direct_velocity(s.y, r, s.grid, l))
    assert idx == cell
    a = node_aligned_scene(1, 3)
    ra = rd.radar_from_scene(a)
    zr = factor.range_spectra(a.y, ra.pad_r, ra.centered)
    for kind in KINDS:
        e = factor.gh_location_energy(zr, ra, a.grid, kind)
        _, _, idx, _, _ = factor.factored_estimate(e, lambda l: factor.gh_velocity(zr, ra, a.grid, l, kind))
        assert idx == true_cell(a), kind
