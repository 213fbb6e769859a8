"""Test fixtures: special scenes built on top of the seeded generator.

node_aligned_scene: the target sits on a grid point and every receiver is
placed so that, at that point, the bistatic range lands exactly on a range bin
and the bistatic rate exactly on a Doppler bin of the zero-padded maps.  The
true cell's atoms then coincide with map nodes, so interpolation there is
exact for any kernel and grid hopping equals the direct decision.
"""
from __future__ import annotations

import math

import numpy as np

from paper_2307_16550_amd import scene as sc


def bins_per_metre(s):
    return s.bw * s.pad / s.c


def bins_per_mps(s):
    return s.f0 * s.tc * s.pad * s.mc / s.c


def node_aligned_scene(cfg=1, trial=0, snr_db=math.inf, k=None, centered=1, seed=None):
    s = sc.make_scene(cfg, trial, seed=seed, snr_db=snr_db, on_grid=True, k=k, targets=1, centered=centered)
    rng = np.random.default_rng(10_000 + 17 * trial + cfg)
    p, v = s.pos[0], s.vel[0]
    d_tx = p - s.tx
    n_tx = float(np.hypot(*d_tx))
    u_tx = d_tx / n_tx
    kr, kd = bins_per_metre(s), bins_per_mps(s)
    speed = float(np.hypot(*v))
    phi_v = math.atan2(v[1], v[0])
    rx = np.empty((s.k, 2))
    for q in range(s.k):
        while True:
            # rate along the receiver leg: v . e = target, |target| <= |v|
            frac = rng.uniform(-0.85, 0.85)
            node_d = round(kd * (float(u_tx @ v) + speed * frac))
            target = node_d / kd - float(u_tx @ v)
            if speed > 0 and abs(target) <= 0.95 * speed:
                break
        phi = phi_v + rng.choice([-1.0, 1.0]) * math.acos(target / speed)
        e = np.array([math.cos(phi), math.sin(phi)])
        node_r = math.ceil(kr * (n_tx + 3.0 + 1.5 * q))
        rho = node_r / kr - n_tx
        rx[q] = p - rho * e
    s.rx = rx
    s.alpha = s.alpha.copy()
    y = sc.synthesize(s.f0, s.bw, s.tc, s.ms, s.mc, s.tx, s.rx, s.pos, s.vel, s.alpha,
                      0.0 if snr_db == math.inf else 10.0 ** (-snr_db / 10.0), rng)
    s.y = y.astype(np.complex64)
    return s


def true_cell(s, t=0):
    ax = [s.grid.axis(a) for a in range(4)]
    idx = [int(np.argmin(abs(ax[0] - s.pos[t, 0]))), int(np.argmin(abs(ax[1] - s.pos[t, 1]))),
           int(np.argmin(abs(ax[2] - s.vel[t, 0]))), int(np.argmin(abs(ax[3] - s.vel[t, 1])))]
    n = s.grid.n
    return ((idx[0] * n[1] + idx[1]) * n[2] + idx[2]) * n[3] + idx[3]
