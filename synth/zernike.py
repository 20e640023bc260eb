"""Zernike modes (Noll ordering and normalisation) sampled on a square grid: the input of a
telescope-aberration map (static, or a time series of coefficients).

Z_j(r, theta) = sqrt(n + 1) R_n^m(r) (sqrt(2) cos(m theta) or sqrt(2) sin(m theta), or 1 for
m = 0), with the radial polynomial R_n^m(r) = sum_s (-1)^s (n - s)! / (s! ((n + m)/2 - s)!
((n - m)/2 - s)!) r^(n - 2s); mean of Z_i Z_j over the unit disk = delta_ij.  Noll's index j
orders (n, m) by n, then |m|, even j for cos terms, odd j for sin terms.
"""

import math

import numpy as np


def noll_to_nm(j):
    """Noll index j >= 1 -> (n, m) with m signed (m > 0: cos, m < 0: sin)."""
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    k = j - n * (n + 1) // 2 - 1  # position within radial order n
    ms = [m for m in range(n % 2, n + 1, 2)]
    # each |m| > 0 appears twice; Noll: even j -> cos (m > 0), odd j -> sin (m < 0)
    seq = []
    for m in ms:
        seq += [m] if m == 0 else [m, m]
    m = seq[k]
    if m == 0:
        return n, 0
    return n, (m if j % 2 == 0 else -m)


def radial(n, m, r):
    m = abs(m)
    out = np.zeros_like(r)
    for s in range((n - m) // 2 + 1):
        c = ((-1) ** s * math.factorial(n - s)
             / (math.factorial(s) * math.factorial((n + m) // 2 - s)
                * math.factorial((n - m) // 2 - s)))
        out += c * r ** (n - 2 * s)
    return out


def zernike(j, x, y):
    """Z_j at points (x, y) in units of the pupil radius."""
    n, m = noll_to_nm(j)
    r = np.hypot(x, y)
    t = np.arctan2(y, x)
    R = radial(n, m, r)
    if m == 0:
        return math.sqrt(n + 1) * R
    f = np.cos(m * t) if m > 0 else np.sin(-m * t)
    return math.sqrt(2 * (n + 1)) * R * f


def zernike_grid(n_modes, nx, pitch, radius, first=2):
    """[n_modes][nx * nx] modes first .. first + n_modes - 1 (default: from tip) on an nx x nx
    grid of pitch `pitch` centred like a layer grid (pixel centres (j + 1/2 - nx/2) pitch),
    zero outside the pupil radius."""
    c = (np.arange(nx) + 0.5 - nx / 2.0) * pitch / radius
    X, Y = np.meshgrid(c, c)
    inside = np.hypot(X, Y) <= 1.0
    return np.stack([(zernike(j, X, Y) * inside).ravel()
                     for j in range(first, first + n_modes)])
