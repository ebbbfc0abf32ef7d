"""Oracle-2: conventional time-domain AAHRT (FP64).  Test infrastructure only.

The operator of Section 2.2 (delta along t = sqrt(tau^2 + q (x^2+y^2)) and
along theta = arctan(y/x)) discretised directly as a Riemann sum, with linear
interpolation in time and azimuth (the direct method of Section 5):

  for every model sample (j, l, i) and trace n with azimuth weight w[n, j]:
      t~ = sqrt(tau_i^2 + q_l h_n^2) / dt,  s = floor(t~),  a = t~ - s
      d[n, s]   += w[n, j] (1 - a) M[j, l, i]
      d[n, s+1] += w[n, j] a       M[j, l, i]      (taps at s >= nt are dropped)

The adjoint is the matching gather with the same taps.  A second,
independent discretisation of the same continuous operator as oracle-1.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry


def _taps(geom: Geometry, n: int):
    tau = np.arange(geom.ntau) * geom.dtau
    h2 = geom.x[n] ** 2 + geom.y[n] ** 2
    arg = tau[None, :] ** 2 + geom.q[:, None] * h2           # [nq, ntau]
    valid = arg >= 0.0
    tt = np.sqrt(np.where(valid, arg, 0.0)) / geom.dt
    s = np.floor(tt).astype(np.int64)
    a = tt - s
    return s, a, valid


def forward(m: np.ndarray, geom: Geometry) -> np.ndarray:
    m = np.asarray(m, dtype=np.float64)
    W = geom.W()
    ntr = geom.x.size
    d = np.zeros((ntr, geom.nt))
    for n in range(ntr):
        s, a, valid = _taps(geom, n)
        mw = np.einsum('j,jli->li', W[n], m)                   # azimuth interpolation
        for sh, wt in ((0, 1.0 - a), (1, a)):
            idx = s + sh
            ok = valid & (idx < geom.nt)
            np.add.at(d[n], idx[ok], (wt * mw)[ok])
    return d


def adjoint(d: np.ndarray, geom: Geometry) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    W = geom.W()
    m = np.zeros((geom.ntheta, geom.nq, geom.ntau))
    for n in range(geom.x.size):
        s, a, valid = _taps(geom, n)
        acc = np.zeros((geom.nq, geom.ntau))
        for sh, wt in ((0, 1.0 - a), (1, a)):
            idx = s + sh
            ok = valid & (idx < geom.nt)
            acc[ok] += wt[ok] * d[n, idx[ok]]
        m += W[n][:, None, None] * acc[None]
    return m
