"""Pins of the oracle's range-Doppler maps and geometry against definitions, closed forms and the paper."""
import json
import math
import os

import numpy as np
import pytest

from oracle import maps, radar as rd
from paper_2307_16550_amd import scene as sc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_dft(y, pad_r, pad_d, centered):
    """The 2D correlation map written as explicit loops (tiny sizes only)."""
    k, mc, ms = y.shape
    nr, nd = pad_r * ms, pad_d * mc
    cs = (ms - 1) / 2.0 if centered else 0.0
    cm = (mc - 1) / 2.0 if centered else 0.0
    z = np.zeros((k, nr, nd), dtype=np.complex128)
    for q in range(k):
        for i in range(nr):
            for l in range(nd):
                acc = 0j
                for m in range(mc):
                    for s in range(ms):
                        acc += complex(y[q, m, s]) * complex(np.exp(-2j * math.pi * (i * (s - cs) / nr + l * (m - cm) / nd)))
                z[q, i, l] = acc
    return z


def rand_frame(rng, k, mc, ms):
    return (rng.standard_normal((k, mc, ms)) + 1j * rng.standard_normal((k, mc, ms))).astype(np.complex64)


@pytest.mark.parametrize("centered", [0, 1])
@pytest.mark.parametrize("pads", [(1, 1), (2, 4), (4, 2)])
def test_maps_equal_brute_force_dft(centered, pads):
    rng = np.random.default_rng(1)
    y = rand_frame(rng, 2, 4, 8)
    z = maps.rd_maps(y, pads[0], pads[1], centered)
    ref = brute_dft(y, pads[0], pads[1], centered)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("centered", [0, 1])
def test_maps_parseval(centered):
    rng = np.random.default_rng(2)
    y = rand_frame(rng, 3, 32, 64)
    z = maps.rd_maps(y, 4, 4, centered)
    lhs = np.sum(np.abs(z) ** 2)
    rhs = 16 * 32 * 64 * np.sum(np.abs(y.astype(np.complex128)) ** 2)
    assert abs(lhs - rhs) <= 1e-12 * rhs


def test_single_on_node_tone():
    ms, mc, pad = 16, 8, 1
    i0, l0 = 5, 3
    alpha = 0.7 - 0.2j
    s = np.arange(ms)[None, :]
    m = np.arange(mc)[:, None]
    y = (alpha * np.exp(2j * np.pi * (i0 * s / (pad * ms) + l0 * m / (pad * mc))))[None]
    z = maps.rd_maps(y, pad, pad, 0)
    assert abs(z[0, i0, l0] - alpha * ms * mc) < 1e-11
    mask = np.ones_like(z[0], dtype=bool)
    mask[i0, l0] = False
    assert np.max(np.abs(z[0][mask])) < 1e-11
    # with zero padding the tone stays on its node, times P on each axis
    z4 = maps.rd_maps(y, 4, 4, 0)
    assert abs(z4[0, 4 * i0, 4 * l0] - alpha * ms * mc) < 1e-11


def dirichlet(delta, n):
    """sum_{k<n} exp(j 2 pi delta k) in closed form."""
    if abs(delta - round(delta)) < 1e-15:
        return complex(n)
    return np.exp(1j * np.pi * delta * (n - 1)) * np.sin(np.pi * delta * n) / np.sin(np.pi * delta)


@pytest.mark.parametrize("centered", [0, 1])
def test_off_node_tone_dirichlet_closed_form(centered):
    ms, mc, pad = 32, 16, 4
    fr, fd = 0.2137, -0.3711
    s = np.arange(ms)[None, :]
    m = np.arange(mc)[:, None]
    y = np.exp(2j * np.pi * (fr * s + fd * m))[None]
    z = maps.rd_maps(y, pad, pad, centered)
    rng = np.random.default_rng(3)
    for _ in range(20):
        i, l = rng.integers(0, pad * ms), rng.integers(0, pad * mc)
        val = dirichlet(fr - i / (pad * ms), ms) * dirichlet(fd - l / (pad * mc), mc)
        if centered:
            val *= np.exp(2j * np.pi * (i * (ms - 1) / 2 / (pad * ms) + l * (mc - 1) / 2 / (pad * mc)))
        assert abs(z[0, i, l] - val) < 1e-10


@pytest.mark.parametrize("centered", [0, 1])
def test_node_value_outside_one_period(centered):
    """Values at indices beyond one period equal the correlation evaluated at that frequency."""
    rng = np.random.default_rng(4)
    y = rand_frame(rng, 1, 8, 16)
    pad = 2
    z = maps.rd_maps(y, pad, pad, centered)
    nr, nd = pad * 16, pad * 8
    cs, cm = (15 / 2, 7 / 2) if centered else (0.0, 0.0)
    for i, l in [(-1, 3), (nr, -2), (nr + 3, nd + 1), (5, -nd - 1), (-nr - 2, 2 * nd + 3)]:
        s = np.arange(16)[None, :]
        m = np.arange(8)[:, None]
        direct = np.sum(y[0].astype(np.complex128) * np.exp(-2j * np.pi * (i * (s - cs) / nr + l * (m - cm) / nd)))
        assert abs(maps.node_value(z[0], i, l, 16, 8, centered) - direct) < 1e-10 * np.abs(z).max()


def test_geometry_collocated_and_symmetric():
    r = rd.Radar(24e9, 250e6, 256e-6, sc.C_LIGHT, 64, 32, 4, 4, np.array([0.0, 0.0]),
                 np.array([[0.0, 0.0], [1.5, -2.0]]))
    x, y = np.array([7.0, -3.0]), np.array([2.0, 4.0])
    rr, wx, wy = rd.sensing(r, 0, x, y)
    nrm = np.hypot(x, y)
    assert np.allclose(rr, 2 * nrm, rtol=1e-15) and np.allclose(wx, 2 * x / nrm) and np.allclose(wy, 2 * y / nrm)
    swapped = rd.Radar(24e9, 250e6, 256e-6, sc.C_LIGHT, 64, 32, 4, 4, np.array([1.5, -2.0]), np.array([[0.0, 0.0]]))
    assert np.allclose(rd.sensing(r, 1, x, y)[0], rd.sensing(swapped, 0, x, y)[0], rtol=1e-15)


def test_geometry_gradient_and_rate_by_finite_differences():
    r = rd.Radar(24e9, 250e6, 256e-6, sc.C_LIGHT, 64, 32, 4, 4, np.array([0.3, -0.2]), np.array([[0.0, 6.0]]))
    p = np.array([11.0, -4.0])
    v = np.array([3.0, -7.5])
    h = 1e-6
    rr, wx, wy = rd.sensing(r, 0, *p)
    gx = (rd.sensing(r, 0, p[0] + h, p[1])[0] - rd.sensing(r, 0, p[0] - h, p[1])[0]) / (2 * h)
    gy = (rd.sensing(r, 0, p[0], p[1] + h)[0] - rd.sensing(r, 0, p[0], p[1] - h)[0]) / (2 * h)
    assert abs(gx - wx) < 1e-8 and abs(gy - wy) < 1e-8
    # U = dR/dt along the motion x(t) = p + v t
    dt = 1e-6
    rate = (rd.sensing(r, 0, *(p + v * dt))[0] - rd.sensing(r, 0, *(p - v * dt))[0]) / (2 * dt)
    assert abs(rate - (wx * v[0] + wy * v[1])) < 1e-6


def test_paper_printed_parameters_fix_the_range_scaling():
    """Resolution c/(2B) = 60 cm (Fig. 3 caption); one resolution of bistatic path (c/B) is P bins."""
    with open(os.path.join(GOLDEN, "paper_parameters.json")) as f:
        g = json.load(f)
    bw = g["bandwidth_hz"]["value"]
    assert round(sc.C_LIGHT / (2 * bw), g["range_resolution_m"]["digits"]) == g["range_resolution_m"]["value"]
    ms = g["samples_per_chirp"]["value"]
    mc = g["chirps_per_frame"]["value"]
    r = rd.Radar(g["carrier_hz"]["value"], bw, g["chirp_s"]["value"], sc.C_LIGHT, ms, mc, 4, 4,
                 np.zeros(2), np.array([[0.0, 0.0]]))
    # monostatic: x at distance d gives R = 2 d; moving by one resolution shifts the range bin by P
    d0, res = 10.0, sc.C_LIGHT / (2 * bw)
    t0, _ = rd.bin_coords(r, 0, d0, 0.0, 0.0, 0.0)
    t1, _ = rd.bin_coords(r, 0, d0 + res, 0.0, 0.0, 0.0)
    assert abs((t1 - t0) - 4.0) < 1e-9
    # Doppler: a radial speed of lambda/(2 Mc Tc) (one Doppler resolution) shifts by P bins
    lam = sc.C_LIGHT / g["carrier_hz"]["value"]
    vres = lam / (2 * mc * g["chirp_s"]["value"])
    _, d_a = rd.bin_coords(r, 0, d0, 0.0, 0.0, 0.0)
    _, d_b = rd.bin_coords(r, 0, d0, 0.0, vres, 0.0)
    assert abs((d_b - d_a) - 4.0) < 1e-9


def test_generator_noise_free_tone_has_unit_modulus_terms():
    s = sc.make_scene(1, 0, snr_db=math.inf)
    y = s.y.astype(np.complex128)
    assert np.allclose(np.abs(y), np.abs(s.alpha[0])[:, None, None], rtol=1e-6)
