"""One Block-OMP iteration of the oracle (test infrastructure; see the package header).

The paper names Block Orthogonal Matching Pursuit and lists iterative direct
algorithms for several targets as future work (Sec. VI); block-sparse
recovery is the family of its direct-method reference.  One iteration, as
built here:
  1. decision on the current residual (grid hopping on its maps, or direct);
  2. select the grid cell theta of the maximum, excluding cells already in the
     support S; S <- S + [theta];
  3. per receiver q, least squares over the support with the exact atoms of
     eq. (3), A_q(theta) = b(f_d) (x) a(f_r):
        alpha[:, q] = argmin_a || Y_q - sum_t a_t A_q(theta_t) ||^2
     via the normal equations (A^H A) alpha = A^H Y_q;
  4. residual Y_q - sum_t alpha[t, q] A_q(theta_t), in the data domain.
The scattering coefficients are refitted jointly every iteration (the
"orthogonal" step); the number of iterations is fixed by the caller.
"""
from __future__ import annotations

import numpy as np

from . import direct, gh, maps, peaks, radar as rd


def atom(radar: rd.Radar, q: int, point) -> np.ndarray:
    """A_q(theta) of eq. (3) as an (Mc, Ms) matrix: b_m(f_d) a_s(f_r)."""
    fr, fd = rd.sensed_freqs(radar, q, point[0], point[1], point[2], point[3])
    return np.outer(direct.doppler_atom(fd, radar.mc), direct.range_atom(fr, radar.ms))


def decision(resid: np.ndarray, radar: rd.Radar, grid, use_direct: bool, kind: int) -> np.ndarray:
    if use_direct:
        return direct.direct_decision(resid, radar, grid)
    z = maps.rd_maps(resid, radar.pad_r, radar.pad_d, radar.centered)
    return gh.gh_decision(z, radar, grid, kind)


def fit(y: np.ndarray, radar: rd.Radar, grid, support):
    """Least-squares coefficients alpha[t, q] over `support` and the new residual (complex128)."""
    y = np.asarray(y).astype(np.complex128)
    pts = [rd.grid_point(grid, int(c)) for c in support]
    alpha = np.zeros((len(pts), radar.k), dtype=np.complex128)
    resid = np.empty_like(y)
    for q in range(radar.k):
        a = np.stack([atom(radar, q, p).ravel() for p in pts], axis=1)     # (Mc*Ms, T)
        gram = a.conj().T @ a
        rhs = a.conj().T @ y[q].ravel()
        alpha[:, q] = np.linalg.solve(gram, rhs)
        resid[q] = (y[q].ravel() - a @ alpha[:, q]).reshape(y[q].shape)
    return alpha, resid


def bomp_step(y, resid, support, radar: rd.Radar, grid, use_direct: bool = False, kind: int = gh.BILINEAR):
    """One iteration: returns (support + [theta], alpha (T, K), new residual, decision peak value)."""
    d = decision(resid, radar, grid, use_direct, kind)
    value, cell = peaks.global_peak(d, exclude=support)
    support = list(support) + [cell]
    alpha, new_resid = fit(y, radar, grid, support)
    return support, alpha, new_resid, value
