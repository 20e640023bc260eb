"""FP64 oracle of interaction-matrix calibration and the regularised least-squares control
matrix.  TEST INFRASTRUCTURE ONLY (same rules as the rest of this package).

Sec. 2.5: the modes of the chosen modal base are pushed through the sensor model and their
slopes recorded, with or without noise and optionally on top of a turbulence screen; the
reference slopes are saved beside them.  Here the modes are single actuator pokes of a DM grid
(its bilinear interpolation in the projection is the influence function) and each slope column
is a push-pull central difference.

Sec. 2.6: the control matrix is the (pseudo-)inverse of the interaction matrix, i.e. the
least-squares estimator, with a user regularisation coefficient and per-DM weights.  Reading:
R = (D^T D + lambda diag(w))^-1 D^T with lambda = eps * mean(diag(D^T D)), D the interaction
matrix (slopes x actuators).
"""

import numpy as np

from .wfs_oracle import forward


def interaction_matrix(cfg, act_offset, n_act, amplitude, batch, step=0, seed=42, noise=False,
                       base=None):
    """Rows j = (s(base + a e_j) - s(base - a e_j)) / (2 a), j < n_act, where e_j is element
    act_offset + j of one realisation's layer buffer.  Every row is taken about the same
    operating point: the layers (a base screen with wind included) are sampled at time step
    ``step`` for every actuator.  The realisation and noise numbering of a batched
    calibration with ``batch`` realisations per call is kept (actuator j = c h + r,
    h = batch / 2: push in realisation r, pull in realisation h + r, noise drawn with step
    counter step + c), so noisy calibrations draw the same noise as that schedule."""
    stride = int(cfg["layer_stride"])
    x0 = np.zeros(stride) if base is None else np.asarray(base, dtype=np.float64).copy()
    h = batch // 2
    rows = []
    for j in range(n_act):
        c, r = divmod(j, h)
        xp = x0.copy()
        xp[act_offset + j] += amplitude
        xm = x0.copy()
        xm[act_offset + j] -= amplitude
        sp, _ = forward(xp[None], cfg, step, seed, noise, realisations=[r], noise_step=step + c)
        sm, _ = forward(xm[None], cfg, step, seed, noise, realisations=[h + r],
                        noise_step=step + c)
        rows.append((sp[0] - sm[0]) / (2.0 * amplitude))
    return np.array(rows)


def reference_slopes(cfg, step=0, seed=42, noise=False, base=None):
    """Slopes of the unpoked system (realisation 0)."""
    stride = int(cfg["layer_stride"])
    x0 = np.zeros(stride) if base is None else np.asarray(base, dtype=np.float64)
    s, _ = forward(x0[None], cfg, step, seed, noise, realisations=[0])
    return s[0]


def regularised_lse(im, eps, weights=None):
    """Control matrix R [m][n_s] from the interaction matrix im [m][n_s] (row j = slopes of
    actuator j): R = (D^T D + lambda diag(w))^-1 D^T, D = im^T, lambda = eps mean diag(D^T D)."""
    D = np.asarray(im, dtype=np.float64).T
    G = D.T @ D
    m = G.shape[0]
    w = np.ones(m) if weights is None else np.asarray(weights, dtype=np.float64)
    lam = eps * np.trace(G) / m
    return np.linalg.solve(G + lam * np.diag(w), D.T)
