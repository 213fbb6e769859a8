"""Seeded synthetic multistatic FMCW scenes: the inputs shared by the HIP path and the oracle.

This module only *draws* inputs.  It holds none of the estimator's arithmetic
(no maps, no interpolation, no decision function); it synthesises the
dechirped data of the measurement model so that both the GPU path and the
FP64 oracle can be fed the very same complex64 arrays.

Measurement model (paper, Sec. II, eq. (3)): per receiver q,
    Y_q = alpha_q b(u_q) (x) a(r_q) + W_q,  Y_q in C^{Mc x Ms},
rows are chirps, columns fast-time samples.  The atoms are Fourier vectors
a_m(r) = exp(j 2 pi r m), b_m(u) = exp(j 2 pi u m).  The sensing functions of
eqs. (1)-(2) are used with the physical FMCW scaling (cycles per sample and per
chirp):
    f_r = B * R / (c * Ms),   R = |x - x_TX| + |x - x_RX,q|      (bistatic range sum)
    f_d = f0 * Tc * U / c,    U = <unit(x - x_TX) + unit(x - x_RX,q), v>
which is the scaling the workload definitions state; the paper's own printed
factor 2B/c is the monostatic convention (its 60 cm resolution is c/2B).
Several targets superpose (one scattering coefficient per target and per
receiver, as eq. (3) has one alpha per RX).

Workload recipes (shapes of the paper's experiment, Sec. V: f0 = 24 GHz,
B = 250 MHz, one TX, Q receivers):
  cfg 1  K=3, Ms=64,  Mc=32,  1 target, SNR 20 dB, grid 32x32x8x8
  cfg 2  K=4, Ms=256, Mc=128, 3 targets, SNR 10 dB, grid 128x128x32x32
         (direct method on the stride-2 64x64x16x16 subgrid)
  cfg 3  K=8, Ms=64,  Mc=32,  1 target, SNR 20 dB, grid 256x256x32x32
  cfg 5  K=8, Ms=512, Mc=256, 8 targets, SNR 5 dB, grid 128x128x32x32
  batch  64 frames of mixed shapes (make_batch)
All use Tc = 256 us and zero padding x4 on both axes.  The paper's own
measurement campaign (433 real frames) is private; these synthetic scenes
stand in for it.

Random draws, in this order, from numpy.random.default_rng(seed):
  1. receiver y-coordinates y_q ~ U[-10, 10] (x = 0), redrawn as a whole until
     every pairwise gap is >= 1 m; TX at (0, 0);
  2. per target: position ~ U([5,25] x [-10,10]); then velocity ~ U([-10,10]^2);
  3. scattering coefficients alpha[t, q] ~ CN(0, 1);
  4. noise W ~ CN(0, sigma^2) with sigma^2 = 10^(-SNR/10) per complex sample.
Default seed: 230716550 + 1000 * cfg + trial.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299_792_458.0

# Domains of the parameters of interest (paper Sec. II: subspaces X and V).
X_LO, X_HI = (5.0, -10.0), (25.0, 10.0)
V_LO, V_HI = (-10.0, -10.0), (10.0, 10.0)


@dataclasses.dataclass
class Grid:
    """Inclusive 4D grid over (x, y, vx, vy); point i on axis a is lo + i*(hi-lo)/(n-1)."""

    lo: tuple
    hi: tuple
    n: tuple

    @property
    def size(self) -> int:
        return int(np.prod(self.n))

    def decimate(self, stride: int) -> "Grid":
        """Every `stride`-th point of each axis, starting at index 0."""
        lo, hi, n = [], [], []
        for a in range(4):
            na = (self.n[a] - 1) // stride + 1
            step = 0.0 if self.n[a] == 1 else (self.hi[a] - self.lo[a]) / (self.n[a] - 1)
            lo.append(self.lo[a])
            hi.append(self.lo[a] + (na - 1) * stride * step)
            n.append(na)
        return Grid(tuple(lo), tuple(hi), tuple(n))

    def axis(self, a: int) -> np.ndarray:
        if self.n[a] == 1:
            return np.array([self.lo[a]], dtype=np.float64)
        step = (self.hi[a] - self.lo[a]) / (self.n[a] - 1)
        return self.lo[a] + np.arange(self.n[a], dtype=np.float64) * step


@dataclasses.dataclass
class Scene:
    f0: float
    bw: float
    tc: float
    ms: int
    mc: int
    pad: int
    tx: np.ndarray          # (2,)
    rx: np.ndarray          # (K, 2)
    y: np.ndarray           # complex64 (K, Mc, Ms), sample index fastest
    pos: np.ndarray         # (T, 2) target positions
    vel: np.ndarray         # (T, 2) target velocities
    alpha: np.ndarray       # complex128 (T, K)
    snr_db: float
    grid: Grid
    c: float = C_LIGHT
    centered: int = 1

    @property
    def k(self) -> int:
        return self.rx.shape[0]


# The seeded single-frame workloads, by number: 1 the small frame the oracle
# sweeps whole, 2 the paper-scale frame, 3 the precision workload, 5 the
# differentiation workload (the batching workload is `make_batch`).
WORKLOADS = {
    1: dict(k=3, ms=64, mc=32, targets=1, snr_db=20.0, n=(32, 32, 8, 8)),
    2: dict(k=4, ms=256, mc=128, targets=3, snr_db=10.0, n=(128, 128, 32, 32)),
    3: dict(k=8, ms=64, mc=32, targets=1, snr_db=20.0, n=(256, 256, 32, 32)),
    5: dict(k=8, ms=512, mc=256, targets=8, snr_db=5.0, n=(128, 128, 32, 32), close_pairs=2),
}
F0, BW, TC, PAD = 24e9, 250e6, 256e-6, 4


def default_seed(cfg: int, trial: int = 0) -> int:
    return 230716550 + 1000 * cfg + trial


def full_grid(n) -> Grid:
    return Grid((X_LO[0], X_LO[1], V_LO[0], V_LO[1]), (X_HI[0], X_HI[1], V_HI[0], V_HI[1]), tuple(n))


def draw_receivers(rng, k: int, half_span: float = 10.0, min_gap: float | None = None) -> np.ndarray:
    """k receivers uniform on the 20 m baseline x = 0, at least 1 m apart (closer for k > 8)."""
    if min_gap is None:
        min_gap = 1.0 if k <= 8 else half_span / (2 * k)
    while True:
        ys = rng.uniform(-half_span, half_span, size=k)
        if k < 2 or np.min(np.diff(np.sort(ys))) >= min_gap:
            return np.stack([np.zeros(k), ys], axis=1)


def synthesize(f0, bw, tc, ms, mc, tx, rx, pos, vel, alpha, noise_sigma2, rng, c=C_LIGHT):
    """Forward model of eq. (3) summed over targets, plus complex white noise."""
    k = rx.shape[0]
    s = np.arange(ms, dtype=np.float64)
    m = np.arange(mc, dtype=np.float64)
    y = np.zeros((k, mc, ms), dtype=np.complex128)
    for t in range(pos.shape[0]):
        p, v = pos[t], vel[t]
        d_tx = p - tx
        n_tx = math.hypot(d_tx[0], d_tx[1])
        for q in range(k):
            d_rx = p - rx[q]
            n_rx = math.hypot(d_rx[0], d_rx[1])
            rng_sum = n_tx + n_rx
            rate = float(np.dot(d_tx / n_tx + d_rx / n_rx, v))
            fr = bw * rng_sum / (c * ms)
            fd = f0 * tc * rate / c
            a = np.exp(2j * np.pi * fr * s)
            b = np.exp(2j * np.pi * fd * m)
            y[q] += alpha[t, q] * np.outer(b, a)
    if noise_sigma2 > 0:
        w = rng.standard_normal((k, mc, ms, 2)) * math.sqrt(noise_sigma2 / 2.0)
        y += w[..., 0] + 1j * w[..., 1]
    return y


def make_scene(cfg: int = 1, trial: int = 0, seed: int | None = None, *, snr_db: float | None = None,
               on_grid: bool = False, targets: int | None = None, k: int | None = None,
               ms: int | None = None, mc: int | None = None, n=None, centered: int = 1) -> Scene:
    """Draw a scene of workload `cfg` (keyword arguments override the recipe)."""
    spec = dict(WORKLOADS[cfg])
    for key, val in (("snr_db", snr_db), ("targets", targets), ("k", k), ("ms", ms), ("mc", mc), ("n", n)):
        if val is not None:
            spec[key] = val
    rng = np.random.default_rng(default_seed(cfg, trial) if seed is None else seed)
    tx = np.zeros(2)
    rx = draw_receivers(rng, spec["k"])
    nt = spec["targets"]
    pos = np.empty((nt, 2))
    vel = np.empty((nt, 2))
    for t in range(nt):
        pos[t] = rng.uniform(X_LO, X_HI)
        vel[t] = rng.uniform(V_LO, V_HI)
    # targets 2p + 1 placed within one bistatic range cell (c / B = 1.2 m) of targets 2p
    for pr in range(min(spec.get("close_pairs", 0), nt // 2)):
        ang = rng.uniform(0.0, 2.0 * np.pi)
        dist = rng.uniform(0.3, 0.9)
        cand = pos[2 * pr] + dist * np.array([np.cos(ang), np.sin(ang)])
        pos[2 * pr + 1] = np.clip(cand, X_LO, X_HI)
    alpha = (rng.standard_normal((nt, spec["k"])) + 1j * rng.standard_normal((nt, spec["k"]))) / math.sqrt(2.0)
    grid = full_grid(spec["n"])
    if on_grid:
        axes = [grid.axis(a) for a in range(4)]
        for t in range(nt):
            pos[t] = [axes[0][np.argmin(abs(axes[0] - pos[t, 0]))], axes[1][np.argmin(abs(axes[1] - pos[t, 1]))]]
            vel[t] = [axes[2][np.argmin(abs(axes[2] - vel[t, 0]))], axes[3][np.argmin(abs(axes[3] - vel[t, 1]))]]
    snr = spec["snr_db"]
    sigma2 = 0.0 if snr == math.inf else 10.0 ** (-snr / 10.0)
    y = synthesize(F0, BW, TC, spec["ms"], spec["mc"], tx, rx, pos, vel, alpha, sigma2, rng)
    return Scene(f0=F0, bw=BW, tc=TC, ms=spec["ms"], mc=spec["mc"], pad=PAD, tx=tx, rx=rx,
                 y=y.astype(np.complex64), pos=pos, vel=vel, alpha=alpha, snr_db=snr, grid=grid,
                 centered=centered)


# Batching workload: per frame K in [3, 8], Ms in {128, 256}, Mc in {64, 128},
# 1-5 targets, Nx = Ny in {64, 96, 128, 160, 192}, Nvx = Nvy in {16, 24, 32}
# (SNR 10 dB, the paper-scale scene's).
BATCH = dict(frames=64, k=(3, 8), ms=(128, 256), mc=(64, 128), targets=(1, 5), nxy=(64, 96, 128, 160, 192),
             nv=(16, 24, 32), snr_db=10.0)


def batch_seed(trial: int = 0) -> int:
    return 230716550 + 4000 + trial


def make_batch(trial: int = 0, frames: int | None = None, seed: int | None = None, **over) -> list:
    """Scenes of the batching workload.  The frame shapes are drawn first, in
    frame order, from default_rng(seed): K, Ms, Mc, targets, Nx = Ny, Nvx = Nvy;
    frame f is then make_scene's draw with seed + 1 + f.  Keyword arguments
    replace entries of BATCH (tuples are the choices, (lo, hi) for K and
    targets)."""
    spec = dict(BATCH)
    spec.update(over)
    nf = spec["frames"] if frames is None else frames
    base = batch_seed(trial) if seed is None else seed
    rng = np.random.default_rng(base)
    shapes = []
    for _ in range(nf):
        k = int(rng.integers(spec["k"][0], spec["k"][1] + 1))
        ms = int(rng.choice(spec["ms"]))
        mc = int(rng.choice(spec["mc"]))
        nt = int(rng.integers(spec["targets"][0], spec["targets"][1] + 1))
        nxy = int(rng.choice(spec["nxy"]))
        nv = int(rng.choice(spec["nv"]))
        shapes.append((k, ms, mc, nt, nxy, nv))
    return [make_scene(1, seed=base + 1 + f, k=k, ms=ms, mc=mc, targets=nt, n=(nxy, nxy, nv, nv),
                       snr_db=spec["snr_db"])
            for f, (k, ms, mc, nt, nxy, nv) in enumerate(shapes)]


def direct_grid(scene: Scene, cfg: int) -> Grid:
    """Grid of the direct method: the full grid, except cfg 2's stride-2 subgrid."""
    return scene.grid.decimate(2) if cfg == 2 else scene.grid
