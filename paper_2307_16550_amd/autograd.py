"""torch.autograd bindings of the point decisions, peak selection and gradient ascent.

The forward passes call gh_direct_points / gh_gh_points (the library's HIP
kernels compute the values and the hand-written gradients together); the
backward passes scale the saved gradients by the incoming gradient.  Nothing
here evaluates a decision on the CPU.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gridhop as gh


class DirectDecisionAt(torch.autograd.Function):
    """D_dir(theta; rx) at points theta [n, 4] (float64, CUDA), differentiable in
    theta and in the receiver positions rx [K, 2] (float64, any device)."""

    @staticmethod
    def forward(ctx, theta, rx, radar, y):
        r = radar.with_rx(rx.detach().cpu().numpy())
        value, grad, grad_rx = gh.direct_points(r, y, theta.detach(), want_grad=True,
                                                want_grad_rx=ctx.needs_input_grad[1])
        ctx.save_for_backward(grad, grad_rx if grad_rx is not None else torch.empty(0, device=theta.device))
        ctx.rx_meta = (rx.device, rx.dtype)
        return value

    @staticmethod
    def backward(ctx, gout):
        grad, grad_rx = ctx.saved_tensors
        g_theta = gout[:, None] * grad if ctx.needs_input_grad[0] else None
        g_rx = None
        if ctx.needs_input_grad[1]:
            dev, dt = ctx.rx_meta
            g_rx = (gout[:, None, None] * grad_rx).sum(0).to(device=dev, dtype=dt)
        return g_theta, g_rx, None, None


class GhDecisionAt(torch.autograd.Function):
    """D_gh(theta; rx) at points theta [n, 4] from a map tensor (any storage), differentiable in
    theta and rx.  The maps are those of the receivers at their nominal positions: only the
    sensing functions move with rx."""

    @staticmethod
    def forward(ctx, theta, rx, radar, maps, interp):
        r = radar.with_rx(rx.detach().cpu().numpy())
        value, grad, grad_rx = gh.gh_points(r, maps, theta.detach(), interp, want_grad=True,
                                            want_grad_rx=ctx.needs_input_grad[1])
        ctx.save_for_backward(grad, grad_rx if grad_rx is not None else torch.empty(0, device=theta.device))
        ctx.rx_meta = (rx.device, rx.dtype)
        return value

    @staticmethod
    def backward(ctx, gout):
        grad, grad_rx = ctx.saved_tensors
        g_theta = gout[:, None] * grad if ctx.needs_input_grad[0] else None
        g_rx = None
        if ctx.needs_input_grad[1]:
            dev, dt = ctx.rx_meta
            g_rx = (gout[:, None, None] * grad_rx).sum(0).to(device=dev, dtype=dt)
        return g_theta, g_rx, None, None, None


def rx_tensor(radar) -> torch.Tensor:
    return torch.from_numpy(radar.rx.copy())


def direct_decision_at(theta, radar, y, rx=None):
    return DirectDecisionAt.apply(theta, rx_tensor(radar) if rx is None else rx, radar, y)


def gh_decision_at(theta, radar, maps, interp=gh.BILINEAR, rx=None):
    return GhDecisionAt.apply(theta, rx_tensor(radar) if rx is None else rx, radar, maps, interp)


def grid_steps(grid: gh.GhGrid) -> np.ndarray:
    return np.array([0.0 if grid.n[a] == 1 else (grid.hi[a] - grid.lo[a]) / (grid.n[a] - 1) for a in range(4)])


def cell_points(grid: gh.GhGrid, cells) -> np.ndarray:
    """(x, y, vx, vy) of linear grid indices."""
    cells = np.asarray(cells, np.int64)
    n = list(grid.n)
    iv = np.stack(np.unravel_index(cells, n), axis=1).astype(np.float64)
    return np.asarray(grid.lo)[None, :] + iv * grid_steps(grid)[None, :]


def top_peaks(block: torch.Tensor, grid: gh.GhGrid, k=16, radius=(4, 4, 2, 2)):
    """The k largest block maxima after 4D non-maximum suppression: a candidate is
    dropped when it lies within `radius` cells of an already selected peak on every
    axis (choose it about half a resolution cell: c / B in location, which is several
    grid steps on fine location grids).  Returns linear grid indices (int64 numpy
    array), best first."""
    values, index = gh.decode_peaks(block)
    order = np.argsort(-values, kind="stable")
    n = list(grid.n)
    chosen, coords = [], []
    rad = np.asarray(radius)
    for i in order:
        c = np.array(np.unravel_index(int(index[i]), n))
        if any(np.all(np.abs(c - p) <= rad) for p in coords):
            continue
        chosen.append(int(index[i]))
        coords.append(c)
        if len(chosen) == k:
            break
    return np.array(chosen, dtype=np.int64)


def ascend(value_grad, theta0: torch.Tensor, h, steps=20, step0=0.25, grow=1.5, return_accepted=False):
    """Monotone gradient ascent of a decision at n points, `steps` iterations.

    value_grad(theta) -> (value [n], grad [n, 4]).  Coordinates are scaled by the
    grid steps h (an axis with h = 0 is held).  Each iteration proposes
    z + s * g_z / max|g_z| (s in grid steps, per point), accepts it when the
    decision does not decrease (then s *= grow) and otherwise halves s.
    Returns (theta, value, history of values [steps + 1, n]), and with
    return_accepted also the acceptance of each proposal (bool [steps, n]).
    """
    h_t = torch.as_tensor(np.asarray(h, np.float64), device=theta0.device)
    free = h_t > 0
    theta = theta0.clone()
    value, grad = value_grad(theta)
    s = torch.full((theta.shape[0],), float(step0), dtype=torch.float64, device=theta.device)
    hist = [value.clone()]
    accepted = []
    for _ in range(steps):
        gz = torch.where(free, grad * h_t, torch.zeros_like(grad))
        norm = gz.abs().amax(dim=1).clamp_min(1e-300)
        cand = theta + (s / norm)[:, None] * gz * h_t
        v_new, g_new = value_grad(cand)
        ok = v_new >= value
        theta = torch.where(ok[:, None], cand, theta)
        value = torch.where(ok, v_new, value)
        grad = torch.where(ok[:, None], g_new, grad)
        s = torch.where(ok, s * grow, s * 0.5)
        hist.append(value.clone())
        accepted.append(ok)
    if return_accepted:
        return theta, value, torch.stack(hist), torch.stack(accepted)
    return theta, value, torch.stack(hist)
