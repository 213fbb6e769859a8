"""Pins of the oracle's Block-OMP iteration and off-grid refinement."""
import math

import numpy as np
import pytest

from oracle import bomp, direct, gh, radar as rd, refine
from paper_2307_16550_amd import scene as sc
from _fixtures import true_cell


def dirichlet(delta, n):
    if abs(delta - round(delta)) < 1e-14:
        return complex(n) * np.exp(1j * np.pi * round(delta) * (n - 1) * 0)
    return np.exp(1j * np.pi * delta * (n - 1)) * np.sin(np.pi * delta * n) / np.sin(np.pi * delta)


def test_gram_matches_dirichlet_closed_form():
    s = sc.make_scene(1, 0)
    r = rd.radar_from_scene(s)
    cells = [17, 4000, 60001]
    pts = [rd.grid_point(s.grid, c) for c in cells]
    for q in range(r.k):
        a = np.stack([bomp.atom(r, q, p).ravel() for p in pts], axis=1)
        gram = a.conj().T @ a
        f = [rd.sensed_freqs(r, q, *p) for p in pts]
        for t in range(3):
            for u in range(3):
                closed = dirichlet(f[u][0] - f[t][0], r.ms) * dirichlet(f[u][1] - f[t][1], r.mc)
                assert abs(gram[t, u] - closed) < 1e-9 * r.ms * r.mc


def test_fit_residual_is_orthogonal_to_selected_atoms():
    s = sc.make_scene(1, 1)
    r = rd.radar_from_scene(s)
    support = [123, 40000, 65000]
    alpha, resid = bomp.fit(s.y, r, s.grid, support)
    ynorm = np.linalg.norm(s.y.astype(np.complex128))
    for q in range(r.k):
        for c in support:
            at = bomp.atom(r, q, rd.grid_point(s.grid, c))
            ip = np.vdot(at.ravel(), resid[q].ravel())
            assert abs(ip) <= 1e-10 * ynorm * math.sqrt(at.size)


@pytest.mark.parametrize("use_direct", [True, False])
def test_noise_free_on_grid_target_is_fitted_exactly(use_direct):
    s = sc.make_scene(1, 2, snr_db=math.inf, on_grid=True)
    r = rd.radar_from_scene(s)
    sup, alpha, resid, _ = bomp.bomp_step(s.y, s.y, [], r, s.grid, use_direct=use_direct, kind=gh.BICUBIC)
    if use_direct:
        assert sup == [true_cell(s)]
    if sup == [true_cell(s)]:
        assert np.allclose(alpha[0], s.alpha[0], atol=1e-6)
        assert np.linalg.norm(resid) <= 1e-6 * np.linalg.norm(s.y.astype(np.complex128))


def test_two_on_grid_targets_recovered_in_two_direct_iterations():
    s = sc.make_scene(1, 3, snr_db=math.inf, on_grid=True, targets=2)
    r = rd.radar_from_scene(s)
    truth = {true_cell(s, 0), true_cell(s, 1)}
    sup, resid = [], s.y
    for _ in range(2):
        sup, alpha, resid, _ = bomp.bomp_step(s.y, resid, sup, r, s.grid, use_direct=True)
    assert set(sup) == truth
    order = [sup.index(true_cell(s, t)) for t in range(2)]
    assert np.allclose(alpha[order], s.alpha, atol=1e-6)
    assert np.linalg.norm(resid) <= 1e-6 * np.linalg.norm(s.y.astype(np.complex128))


def test_selection_excludes_support():
    s = sc.make_scene(1, 4)
    r = rd.radar_from_scene(s)
    vol = direct.direct_decision(s.y, r, s.grid)
    first = int(np.argmax(vol))
    sup, *_ = bomp.bomp_step(s.y, s.y, [first], r, s.grid, use_direct=True)
    masked = vol.ravel().copy()
    masked[first] = -np.inf
    assert sup == [first, int(np.argmax(masked))]


def test_derivatives_match_central_differences():
    s = sc.make_scene(1, 5)
    r = rd.radar_from_scene(s)
    theta = np.array([s.pos[0, 0] + 0.13, s.pos[0, 1] - 0.21, s.vel[0, 0] + 0.07, s.vel[0, 1] - 0.05])
    d0, g, h = refine.decision_derivs(s.y, r, theta)
    assert abs(d0 - direct.direct_points(s.y, r, *theta)) < 1e-10 * d0
    eps = 1e-4
    for a in range(4):
        e = np.zeros(4)
        e[a] = eps
        dp, gp, _ = refine.decision_derivs(s.y, r, theta + e)
        dm, gm, _ = refine.decision_derivs(s.y, r, theta - e)
        fd = (dp - dm) / (2 * eps)
        assert abs(fd - g[a]) <= 1e-5 * (abs(g).max() + 1e-3 * d0)
        hfd = (gp - gm) / (2 * eps)
        assert np.allclose(hfd, h[:, a], rtol=0, atol=1e-5 * np.abs(h).max())


@pytest.mark.parametrize("trial", range(3))
def test_refinement_recovers_off_grid_truth_noise_free(trial):
    s = sc.make_scene(1, 10 + trial, snr_db=math.inf)
    r = rd.radar_from_scene(s)
    cell = true_cell(s)
    th = refine.refine(s.y, r, s.grid, [cell], max_iter=40)[0]
    assert np.max(np.abs(th[:2] - s.pos[0])) < 1e-6
    assert np.max(np.abs(th[2:] - s.vel[0])) < 1e-6
