"""Pins of the oracle's Block-OMP iteration and off-grid refinement."""
import math

import numpy as np
import pytest

from oracle import bomp, direct, gh, radar as rd, refine
from paper_2307_16550_amd import scene as sc
from _fixtures import node_aligned_scene, true_cell


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
    """A noise-free target on a grid point is selected and fitted exactly.  The
    direct decision peaks there by Cauchy-Schwarz.  For grid hopping the scene is
    node-aligned (the target's range and Doppler coordinates are map nodes for
    every receiver), where bilinear interpolation is exact and its convex weights
    cannot exceed the node value, so the target's cell is the maximum as well."""
    if use_direct:
        s = sc.make_scene(1, 2, snr_db=math.inf, on_grid=True)
    else:
        s = node_aligned_scene(1, 2)
    r = rd.radar_from_scene(s)
    sup, alpha, resid, _ = bomp.bomp_step(s.y, s.y, [], r, s.grid, use_direct=use_direct, kind=gh.BILINEAR)
    assert sup == [true_cell(s)]
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
    """Noise-free: the true (x, v) is the maximum of D (Cauchy-Schwarz), so the
    converged estimate is the truth."""
    s = sc.make_scene(1, 10 + trial, snr_db=math.inf)
    r = rd.radar_from_scene(s)
    cell = true_cell(s)
    th, conv, _ = refine.refine(s.y, r, s.grid, [cell], report=True)
    assert conv.all()
    assert np.max(np.abs(th[0, :2] - s.pos[0])) < 1e-6
    assert np.max(np.abs(th[0, 2:] - s.vel[0])) < 1e-6


def tiny_scene(trial, snr_db=15.0):
    """A small frame (2 RX, 16 x 16) with a fine local grid around its target:
    cells of 0.25 m and 0.6 m/s, well inside one resolution cell (1.2 m of
    bistatic range, 3 m/s of bistatic rate), so D is unimodal on a cell's box."""
    s = sc.make_scene(1, 20 + trial, snr_db=snr_db, ms=16, mc=16, k=2)
    c = np.round(np.concatenate([s.pos[0], s.vel[0]]), 1)
    half = np.array([1.0, 1.0, 2.4, 2.4])
    s.grid = sc.Grid(tuple(c - half), tuple(c + half), (9, 9, 9, 9))
    return s


def box_maximum(s, r, cell, dense=9):
    """Maximum of D over the one-cell box around `cell` by brute force on a dense
    lattice, polished by scipy's bounded quasi-Newton search (L-BFGS-B, numerical
    gradients of D only) from the lattice maximum: independent of the oracle's
    Newton iteration and of its analytic derivatives."""
    from scipy.optimize import minimize
    h = refine.grid_steps(s.grid)
    th0 = rd.grid_point(s.grid, cell)
    u = np.linspace(-1.0, 1.0, dense)
    zz = np.stack(np.meshgrid(u, u, u, u, indexing="ij"), -1).reshape(-1, 4)
    pts = th0 + zz * h
    vals = direct.direct_points(s.y, r, pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3])
    z_best = zz[int(np.argmax(vals))]
    scale = float(vals.max())
    res = minimize(lambda z: -direct.direct_points(s.y, r, *(th0 + z * h)) / scale, z_best, method="L-BFGS-B",
                   bounds=[(-1.0, 1.0)] * 4, options=dict(ftol=1e-15, gtol=1e-11, maxiter=500))
    return th0 + res.x * h, float(vals.max()), h


@pytest.mark.parametrize("trial", range(4))
def test_refinement_is_the_box_maximum_on_tiny_scenes(trial):
    """From the target's cell of a noisy tiny scene, the converged estimate is the
    maximum of D over the one-cell box: at least every point of a dense 9^4
    lattice of the box, and the point a bounded quasi-Newton search of D finds."""
    s = tiny_scene(trial)
    r = rd.radar_from_scene(s)
    cell = true_cell(s)
    th, conv, _ = refine.refine(s.y, r, s.grid, [cell], report=True)
    assert conv.all()
    d_hat = refine.decision_value(s.y, r, th[0])
    ref, lattice_max, h = box_maximum(s, r, cell)
    assert d_hat >= lattice_max * (1 - 1e-12)
    assert d_hat >= refine.decision_value(s.y, r, ref) * (1 - 1e-12)
    assert np.max(np.abs((th[0] - ref) / np.where(h > 0, h, 1.0))) < 1e-4     # grid-step units


@pytest.mark.parametrize("trial", range(3))
def test_refinement_is_stationary_on_the_box(trial):
    """KKT on the box at the converged point: central differences of D (h = 1e-6
    cells) vanish along free coordinates inside the box and point outwards on an
    active face; moving a free coordinate by 1e-3 cells either way lowers D."""
    s = tiny_scene(trial, snr_db=10.0)
    r = rd.radar_from_scene(s)
    cell = true_cell(s) + 1          # one velocity cell off the target's cell
    th0 = rd.grid_point(s.grid, cell)
    hs = refine.grid_steps(s.grid)
    th, conv, _ = refine.refine(s.y, r, s.grid, [cell], report=True)
    assert conv.all()
    z = (th[0] - th0) / hs
    d0 = refine.decision_value(s.y, r, th[0])
    for a in range(4):
        e = np.zeros(4)
        e[a] = 1e-6 * hs[a]
        g = (refine.decision_value(s.y, r, th[0] + e) - refine.decision_value(s.y, r, th[0] - e)) / 2e-6
        if abs(z[a]) < 1 - 1e-9:
            assert abs(g) <= 1e-6 * d0, (a, g)
            for sgn in (-1, 1):
                assert refine.decision_value(s.y, r, th[0] + sgn * 1e3 * e) <= d0
        else:
            assert np.sign(g) == np.sign(z[a]) or abs(g) <= 1e-6 * d0


def test_refinement_budget_does_not_change_the_answer():
    """The answer is the converged point, not a trajectory: a tighter tolerance and
    a larger budget move it by less than 1e-9 cells."""
    s = tiny_scene(5, snr_db=10.0)
    r = rd.radar_from_scene(s)
    cells = [true_cell(s), true_cell(s) + 7]
    a = refine.refine(s.y, r, s.grid, cells)
    b = refine.refine(s.y, r, s.grid, cells, max_iter=1000, tol=1e-13)
    h = refine.grid_steps(s.grid)
    assert np.max(np.abs((a - b) / np.where(h > 0, h, 1.0))) < 1e-9
