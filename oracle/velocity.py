"""Automatic anisotropic velocity estimate from a Radon cube (FP64).  Test infrastructure only.

Section 3, "Automatic Anisotropic Velocity Peaking": the squared slowness at
intercept tau and azimuth theta is the curvature-weighted mean of the Radon
cube, v^-2(tau, theta) = sum_q q M(tau, q, theta) / sum_q M(tau, q, theta),
the integral over q taken as the sum over the uniform curvature samples.

Reading: the paper states the formula for a cube holding only primary energy;
a sparse-inversion cube is signed (Ricker events), so the weights are |M|.
Where sum_q |M| = 0 (no energy) the estimate is reported as 0, and so is the
velocity v = (v^-2)^(-1/2) wherever v^-2 <= 0.
"""
from __future__ import annotations

import numpy as np


def curvature_mean(m: np.ndarray, q: np.ndarray) -> np.ndarray:
    """m [..., nq, ntau] -> sum_l q_l |m_l| / sum_l |m_l|  [..., ntau] (0 where the sum is 0)."""
    a = np.abs(np.asarray(m, dtype=np.float64))
    den = a.sum(axis=-2)
    num = (np.asarray(q, dtype=np.float64)[:, None] * a).sum(axis=-2)
    out = np.zeros_like(den)
    np.divide(num, den, out=out, where=den > 0)
    return out


def velocity(m: np.ndarray, q: np.ndarray):
    """(v^-2, v) per (..., tau): the curvature mean and its inverse square root (0 where <= 0)."""
    qbar = curvature_mean(m, q)
    v = np.zeros_like(qbar)
    np.power(qbar, -0.5, out=v, where=qbar > 0)
    return qbar, v
