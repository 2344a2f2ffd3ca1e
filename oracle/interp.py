"""FP64 oracle of the SPH interpolant (paper, Sec. 2, eq. (interp)).

TEST INFRASTRUCTURE: imported only by the tests.  Nothing here imports the
GPU package.

Q(r) = sum_i m_i Q_i / rho_i W(|r - r_i|, H_i): every particle contributes
inside its own support H_i (the reading for points that are not particles,
which carry no smoothing length of their own), with the minimum-image
distance in the periodic box.  Brute force over all particles, in chunks of
points, float64.
"""
from __future__ import annotations

import math

import numpy as np


def w_cubic(q):
    """Cubic spline w(q) with support 1 (W = 8/(pi H^3) w(r/H))."""
    q = np.asarray(q, dtype=np.float64)
    w = np.where(q <= 0.5, 1.0 - 6.0 * q * q + 6.0 * q ** 3, 2.0 * (1.0 - q) ** 3)
    return np.where(q < 1.0, w, 0.0)


def interpolate(px, py, pz, x, y, z, m, rho, H, Q, box, chunk=256):
    """Q at the points (px, py, pz) from particles (x, y, z, m, rho, H, Q) in
    the periodic box of edges `box`."""
    P = np.stack([np.asarray(px, np.float64), np.asarray(py, np.float64), np.asarray(pz, np.float64)], 1)
    X = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64), np.asarray(z, np.float64)], 1)
    L = np.asarray(box, dtype=np.float64)
    H = np.asarray(H, np.float64)
    coef = np.asarray(m, np.float64) * np.asarray(Q, np.float64) / np.asarray(rho, np.float64)
    out = np.zeros(P.shape[0])
    for s in range(0, P.shape[0], chunk):
        d = P[s:s + chunk, None, :] - X[None, :, :]
        d -= L * np.round(d / L)
        r = np.sqrt(np.sum(d * d, axis=2))
        W = 8.0 / (math.pi * H ** 3) * w_cubic(r / H)
        out[s:s + chunk] = W @ coef
    return out
