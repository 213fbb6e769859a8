"""GPU parity of the decisions at continuous points and their gradients
(differentiation axis) against the FP64 oracle (oracle/grad.py), the autograd
bindings, top-peak selection and gradient ascent.

Bars: values <= 1e-5 of the largest value checked (FP32 map / per-chirp sums),
gradients <= 1e-4 of the largest gradient component; with BF16 maps, values
<= 1e-2 and gradients <= 2e-2: the interpolant's derivative differences
neighbouring map values, so each value's BF16 rounding (2^-8 relative) enters
with the derivative weights (sum of |W'| up to about 4 for Keys), against a
gradient scale of about |Z| per bin; autograd against central differences
(h = 1e-4) of the GPU forward <= 1e-2.
"""
import math

import numpy as np
import pytest
import torch

from oracle import gh as ogh, grad as ograd, maps as omaps, radar as ord_, refine as orefine
from paper_2307_16550_amd import autograd as ag
from paper_2307_16550_amd import gridhop as gh
from paper_2307_16550_amd import scene as sc

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def say(*a):
    print(*a, flush=True)


def scene_and_radar(cfg, trial=0, **kw):
    s = sc.make_scene(cfg, trial, **kw)
    return s, ord_.radar_from_scene(s), gh.Radar.from_scene(s)


def points_near_targets(s, n, seed, spread=0.5):
    rng = np.random.default_rng(seed)
    h = orefine.grid_steps(s.grid)
    out = []
    for i in range(n):
        t = i % s.pos.shape[0]
        c = np.concatenate([s.pos[t], s.vel[t]])
        out.append(c + rng.uniform(-spread, spread, 4) * h)
    return np.array(out)


def away_from_nodes(r, th, margin=1e-3):
    for q in range(r.k):
        for t in ord_.bin_coords(r, q, *th):
            f = t - math.floor(t)
            if not margin < f < 1.0 - margin:
                return False
    return True


@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_direct_points_parity(cfg):
    say(f"direct points cfg={cfg}")
    s, r, gr = scene_and_radar(cfg)
    pts = points_near_targets(s, 6, 3)
    v, g, grx = gh.direct_points(gr, to_dev(s.y), to_dev(pts), want_grad_rx=True)
    v, g, grx = v.cpu().numpy(), g.cpu().numpy(), grx.cpu().numpy()
    ref = [ograd.direct_value_grad(s.y, r, p) for p in pts]
    rv = np.array([x[0] for x in ref])
    rg = np.stack([x[1] for x in ref])
    rgx = np.stack([x[2] for x in ref])
    ev = np.max(np.abs(v - rv)) / rv.max()
    eg = np.max(np.abs(g - rg)) / np.abs(rg).max()
    ex = np.max(np.abs(grx - rgx)) / np.abs(rg).max()
    say(f"direct points cfg={cfg}: value {ev:.3g} grad {eg:.3g} grad_rx {ex:.3g}")
    assert ev <= 1e-5 and eg <= 1e-4 and ex <= 1e-4


@pytest.mark.parametrize("dtype,tol,gtol", [(gh.MAP_C64, 1e-5, 1e-4), (gh.MAP_BF16, 1e-2, 2e-2)])
@pytest.mark.parametrize("interp", [gh.BILINEAR, gh.BICUBIC])
def test_gh_points_parity(interp, dtype, tol, gtol):
    say(f"gh points interp={interp} dtype={dtype}")
    s, r, gr = scene_and_radar(1, 5)
    pts = points_near_targets(s, 24, 4)
    if interp == gh.BILINEAR:
        pts = np.array([p for p in pts if away_from_nodes(r, p)])
    assert len(pts) >= 6
    z = gh.rd_maps(gr, to_dev(s.y), map_dtype=dtype)
    v, g, grx = gh.gh_points(gr, z, to_dev(pts), interp, want_grad_rx=True)
    v, g, grx = v.cpu().numpy(), g.cpu().numpy(), grx.cpu().numpy()
    zr = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    ref = [ograd.gh_value_grad(zr, r, p, interp) for p in pts]
    rv = np.array([x[0] for x in ref])
    rg = np.stack([x[1] for x in ref])
    rgx = np.stack([x[2] for x in ref])
    ev = np.max(np.abs(v - rv)) / rv.max()
    eg = np.max(np.abs(g - rg)) / np.abs(rg).max()
    ex = np.max(np.abs(grx - rgx)) / np.abs(rg).max()
    say(f"gh points interp={interp} dtype={dtype}: value {ev:.3g} grad {eg:.3g} grad_rx {ex:.3g}")
    assert ev <= tol
    assert eg <= gtol and ex <= gtol


def test_gh_points_agree_with_the_grid_sweep():
    s, r, gr = scene_and_radar(1, 6)
    z = gh.rd_maps(gr, to_dev(s.y))
    g = gh.grid_of(s.grid)
    for interp in (gh.BILINEAR, gh.BICUBIC):
        dec, _, _ = gh.decision(gr, g, z, interp)
        cells = np.random.default_rng(7).integers(0, s.grid.size, 200)
        pts = ag.cell_points(g, cells)
        v, _, _ = gh.gh_points(gr, z, to_dev(pts), interp, want_grad=False)
        dv = dec.view(-1)[torch.from_numpy(cells).to(dev())].double()
        assert float((v - dv).abs().max() / dec.max()) <= 1e-5


def test_autograd_against_kernels_and_finite_differences():
    s, r, gr = scene_and_radar(1, 7)
    y = to_dev(s.y)
    z = gh.rd_maps(gr, y)
    pts = points_near_targets(s, 4, 8)
    h = 1e-4
    for name, fwd in (("direct", lambda th, rx: ag.direct_decision_at(th, gr, y, rx)),
                      ("gh bicubic", lambda th, rx: ag.gh_decision_at(th, gr, z, gh.BICUBIC, rx))):
        theta = to_dev(pts).requires_grad_(True)
        rx = ag.rx_tensor(gr).requires_grad_(True)
        d = fwd(theta, rx)
        d.sum().backward()
        gt = theta.grad.cpu().numpy()
        grx = rx.grad.numpy()
        scale = np.abs(gt).max()
        with torch.no_grad():
            for a in range(4):
                e = torch.zeros(4, dtype=torch.float64, device=dev())
                e[a] = h
                fd = ((fwd(theta + e, rx) - fwd(theta - e, rx)) / (2 * h)).cpu().numpy()
                err = np.max(np.abs(fd - gt[:, a])) / scale
                say(f"{name}: d/dtheta_{a} finite-difference error {err:.3g}")
                assert err <= 1e-2
            for q in range(gr.k):
                for b in range(2):
                    e = torch.zeros_like(rx)
                    e[q, b] = h
                    fd = ((fwd(theta, rx + e) - fwd(theta, rx - e)).sum() / (2 * h)).item()
                    assert abs(fd - grx[q, b]) <= 1e-2 * scale * len(pts)


def test_rx_calibration_gradient():
    """Receivers displaced by a seeded +-5 cm: the GPU receiver gradient at the target matches the
    FP64 analytic one, and a small step along it raises the decision."""
    s, r, gr = scene_and_radar(1, 9, snr_db=math.inf)
    rng = np.random.default_rng(55)
    off = rng.uniform(-0.05, 0.05, gr.rx.shape)
    gr_off = gr.with_rx(gr.rx + off)
    r_off = ord_.radar_from_scene(s)
    r_off.rx = r_off.rx + off
    truth = np.concatenate([s.pos[0], s.vel[0]])[None, :]
    y = to_dev(s.y)
    v, _, grx = gh.direct_points(gr_off, y, to_dev(truth), want_grad_rx=True)
    _, rg, rgx = ograd.direct_value_grad(s.y, r_off, truth[0])
    err = np.max(np.abs(grx.cpu().numpy()[0] - rgx)) / np.abs(rgx).max()
    say(f"rx calibration gradient error {err:.3g}")
    assert err <= 1e-4
    step = 1e-3 * rgx / np.abs(rgx).max()
    v2, _, _ = gh.direct_points(gr_off.with_rx(gr_off.rx + step), y, to_dev(truth), want_grad=False)
    assert float(v2[0]) > float(v[0])


def test_top_peaks_and_gradient_ascent_cfg5():
    """Differentiation workload: 8 RX, Ms=512 x Mc=256, 8 targets (two close pairs), SNR 5 dB,
    grid 128x128x32x32.  Top-16 grid-hopping peaks after 4D suppression, then 20 monotone
    gradient-ascent steps on the direct decision through its adjoint."""
    s, r, gr = scene_and_radar(5)
    y = to_dev(s.y)
    g = gh.grid_of(s.grid)
    z = gh.rd_maps(gr, y)
    _, block, _ = gh.decision(gr, g, z, gh.BILINEAR, write_volume=False)
    cells = ag.top_peaks(block, g, 16)
    assert len(cells) == 16 and len(set(cells.tolist())) == 16
    theta0 = to_dev(ag.cell_points(g, cells))
    vg = lambda th: gh.direct_points(gr, y, th)[:2]
    theta, value, hist = ag.ascend(vg, theta0, ag.grid_steps(g), steps=20)
    hist = hist.cpu().numpy()
    assert np.all(np.diff(hist, axis=0) >= 0.0)
    assert np.all(hist[-1] >= hist[0])
    # suppression: every pair of selected peaks is farther apart than the radius on some axis
    idx = np.stack(np.unravel_index(cells, list(g.n)), axis=1)
    for a in range(16):
        for b in range(a):
            assert np.any(np.abs(idx[a] - idx[b]) > np.array([4, 4, 2, 2]))
    # every peak climbs (the linear receiver array leaves vy weakly determined, so the
    # peaks of a target spread along vy ridges; distances to the targets are reported only)
    h = ag.grid_steps(g)
    truths = np.concatenate([s.pos, s.vel], axis=1)
    th0, th1 = theta0.cpu().numpy(), theta.cpu().numpy()
    for i in range(16):
        d0 = np.abs((th0[i][None, :] - truths) / h).max(axis=1)
        t = int(np.argmin(d0))
        d1 = np.abs((th1[i] - truths[t]) / h).max()
        say(f"peak {i}: nearest target {t} at {d0[t]:.3f} -> {d1:.3f} cells, D {hist[0, i]:.4g} -> {hist[-1, i]:.4g}")
    assert np.sum(hist[-1] > hist[0]) >= 14
    # the gradients the ascent used agree with the FP64 analytic gradient (scale: the gradient
    # at the starting cells, away from the stationary points)
    _, g0, _ = gh.direct_points(gr, y, theta0[:3])
    _, gfin, _ = gh.direct_points(gr, y, theta[:3])
    for i in range(3):
        scale = float(g0[i].abs().max())
        for th, gg in ((th0[i], g0[i]), (th1[i], gfin[i])):
            _, rg, _ = ograd.direct_value_grad(s.y, r, th)
            assert np.max(np.abs(gg.cpu().numpy() - rg)) <= 1e-4 * scale


def _oracle_replay(value_grad64, theta0, h, accepted, step0=0.25, grow=1.5):
    """The ascent of ag.ascend for one point in FP64 with the oracle's gradient,
    taking the GPU's accept/reject decisions (so the two walks see the same
    step lengths and differ only by their gradient arithmetic)."""
    free = h > 0
    theta = np.array(theta0, np.float64)
    _, grad = value_grad64(theta)
    s = step0
    for ok in accepted:
        gz = np.where(free, grad * h, 0.0)
        cand = theta + (s / max(np.abs(gz).max(), 1e-300)) * gz * h
        if ok:
            theta = cand
            _, grad = value_grad64(theta)
            s *= grow
        else:
            s *= 0.5
    return theta


@pytest.mark.parametrize("interp", [gh.BILINEAR, gh.BICUBIC])
def test_gh_gradient_ascent_cfg5(interp):
    """Differentiation workload: the top-16 grid-hopping peaks climbed for 20 steps
    through the adjoint of the grid-hopping decision (GhDecisionAt, torch.autograd);
    three of them replayed in FP64 with the oracle's analytic gradient on the FP64
    maps must land within 1e-3 m and 1e-3 m/s of the GPU walk."""
    say(f"gh ascent cfg5 interp={interp}")
    s, r, gr = scene_and_radar(5)
    y = to_dev(s.y)
    g = gh.grid_of(s.grid)
    z = gh.rd_maps(gr, y)
    _, block, _ = gh.decision(gr, g, z, interp, write_volume=False)
    cells = ag.top_peaks(block, g, 16)
    theta0 = to_dev(ag.cell_points(g, cells))

    def vg(th):
        th = th.detach().clone().requires_grad_(True)
        v = ag.gh_decision_at(th, gr, z, interp)
        v.sum().backward()
        return v.detach(), th.grad.detach()

    h = ag.grid_steps(g)
    theta, value, hist, acc = ag.ascend(vg, theta0, h, steps=20, return_accepted=True)
    hist, acc = hist.cpu().numpy(), acc.cpu().numpy()
    assert np.all(np.diff(hist, axis=0) >= 0.0)
    assert np.sum(hist[-1] > hist[0]) >= 14
    zr = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    vg64 = lambda th: ograd.gh_value_grad(zr, r, th, interp)[:2]
    th0, th1 = theta0.cpu().numpy(), theta.cpu().numpy()
    for i in range(3):
        ref = _oracle_replay(vg64, th0[i], h, acc[:, i])
        dp, dv = np.max(np.abs(th1[i, :2] - ref[:2])), np.max(np.abs(th1[i, 2:] - ref[2:]))
        say(f"peak {i}: {int(acc[:, i].sum())} accepted steps, |dpos| {dp:.3g} m, |dvel| {dv:.3g} m/s")
        assert dp <= 1e-3 and dv <= 1e-3


def test_autograd_finite_differences_cfg5():
    """Differentiation workload: both autograd functions at points near the targets of
    the 8-receiver frame against central differences (h = 1e-4) of the GPU forward
    and against the FP64 analytic gradient (the grid-hopping decision with Keys
    maps, whose weights are differentiable; bilinear has kinks at map nodes)."""
    s, r, gr = scene_and_radar(5)
    y = to_dev(s.y)
    z = gh.rd_maps(gr, y)
    zr = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    pts = points_near_targets(s, 8, 21)
    hfd = 1e-4
    for name, fwd, ref in (
            ("direct", lambda th: ag.direct_decision_at(th, gr, y), lambda p: ograd.direct_value_grad(s.y, r, p)),
            ("gh bicubic", lambda th: ag.gh_decision_at(th, gr, z, gh.BICUBIC),
             lambda p: ograd.gh_value_grad(zr, r, p, gh.BICUBIC))):
        theta = to_dev(pts).requires_grad_(True)
        d = fwd(theta)
        d.sum().backward()
        gt = theta.grad.cpu().numpy()
        scale = np.abs(gt).max()
        rg = np.stack([ref(p)[1] for p in pts])
        ea = np.max(np.abs(gt - rg)) / np.abs(rg).max()
        say(f"{name} cfg5: autograd vs FP64 analytic {ea:.3g}")
        assert ea <= 1e-4
        with torch.no_grad():
            for a in range(4):
                e = torch.zeros(4, dtype=torch.float64, device=dev())
                e[a] = hfd
                fd = ((fwd(theta + e) - fwd(theta - e)) / (2 * hfd)).cpu().numpy()
                err = np.max(np.abs(fd - gt[:, a])) / scale
                say(f"{name} cfg5: d/dtheta_{a} central-difference error {err:.3g}")
                assert err <= 1e-2


def test_rx_calibration_gradient_cfg5():
    """Differentiation workload: the 8 receivers displaced by a seeded +-5 cm; at each
    target the GPU receiver gradient (direct decision, and grid hopping on Keys maps of
    the nominal array) matches the FP64 analytic one, and a small step of the receiver
    positions along it raises the direct decision."""
    s, r, gr = scene_and_radar(5)
    rng = np.random.default_rng(5505)
    off = rng.uniform(-0.05, 0.05, gr.rx.shape)
    gr_off = gr.with_rx(gr.rx + off)
    r_off = ord_.radar_from_scene(s)
    r_off.rx = r_off.rx + off
    y = to_dev(s.y)
    truth = np.concatenate([s.pos, s.vel], axis=1)
    v, _, grx = gh.direct_points(gr_off, y, to_dev(truth), want_grad_rx=True)
    grx = grx.cpu().numpy()
    for t in range(truth.shape[0]):
        _, _, rgx = ograd.direct_value_grad(s.y, r_off, truth[t])
        err = np.max(np.abs(grx[t] - rgx)) / np.abs(rgx).max()
        assert err <= 1e-4, (t, err)
    say(f"rx calibration cfg5 (direct): {truth.shape[0]} targets within 1e-4")
    step = 1e-3 * grx[0] / np.abs(grx[0]).max()
    v2, _, _ = gh.direct_points(gr_off.with_rx(gr_off.rx + step), y, to_dev(truth[:1]), want_grad=False)
    assert float(v2[0]) > float(v[0])
    z = gh.rd_maps(gr, y)
    zr = omaps.rd_maps(s.y, r.pad_r, r.pad_d, r.centered)
    _, _, gxg = gh.gh_points(gr_off, z, to_dev(truth), gh.BICUBIC, want_grad_rx=True)
    gxg = gxg.cpu().numpy()
    for t in range(truth.shape[0]):
        _, _, rgx = ograd.gh_value_grad(zr, r_off, truth[t], gh.BICUBIC)
        err = np.max(np.abs(gxg[t] - rgx)) / np.abs(rgx).max()
        assert err <= 1e-4, (t, err)
    say(f"rx calibration cfg5 (grid hopping, bicubic): {truth.shape[0]} targets within 1e-4")
