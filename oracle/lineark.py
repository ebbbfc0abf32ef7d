"""The paper's own step 3: bilinear interpolation in (k, theta) (FP64).  Test infrastructure only.

Section 3.4 evaluates step 3 of Algorithm 1 by interpolating the 2-D spectrum
M^(f', k, theta), sampled on a uniform k grid k_i = i dk and on the azimuth grid
theta_j, at k = f'(x^2 + y^2), theta = arctan(y/x), with the four coefficients
A1..A4 of eq. (thli):

    A1 = (k_{i+1} - k)(theta_{j+1} - theta)/(dk dtheta)  = (1 - a)(1 - alpha)
    A2 = -(k_{i+1} - k)(theta_j - theta)/(dk dtheta)     = (1 - a) alpha
    A3 = -(k_i - k)(theta_{j+1} - theta)/(dk dtheta)     = a (1 - alpha)
    A4 = (k_i - k)(theta_j - theta)/(dk dtheta)          = a alpha

with i, j the cells holding (k, theta), a = k/dk - i and alpha = theta/dtheta - j.
No interpolation is needed along f' (it appears on both sides).

Readings taken here (the same as the library's kernel_width = 2 mode):
* The k grid is the DFT of the q axis, zero-padded to mg = sigma nq samples, so
  dk = 1/(mg dq).  Before the transform the curvature axis is centred on
  q_c = q_min + (nq // 2) dq: this is the partial NMO of Section 3.5 that brings the
  curvature range around zero (the paper's q range is symmetric about 0).  With
  q_l - q_c = (l - nq//2) dq the centred spectrum
        Mc(f', k, theta_j) = sum_l M^(f', q_l, theta_j) exp(-2 pi i k (q_l - q_c))
  is periodic in k with period 1/dq = mg dk, so cell indices are taken modulo mg:
        G[j, i, f] = Mc(f', k_i, theta_j) = sum_l M^[j, l, f] exp(-2 pi i (l - nq//2) i / mg).
* After the interpolation the partial NMO is undone by exp(-2 pi i f' q_c h^2), which is
  exact: sum_l M^ exp(-2 pi i f' q_l h^2) = exp(-2 pi i f' q_c h^2) Mc(f', f' h^2).
* The theta part (bin by floor, upper neighbour modulo ntheta, weights 1 - alpha and
  alpha) is the oracle's theta_weights; no deapodisation (the paper applies none).

Steps 1, 2 (tau' half), 4 and 5 are oracle-1's.  The transpose takes the same steps in
reverse, each replaced by its transpose under the real inner product.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry
from . import gfst


def _trace_cells(geom: Geometry, mg: int, f_idx: np.ndarray):
    """For every (frequency, trace): the lower k cell i (mod mg) and the fraction a."""
    dq = (geom.q_max - geom.q_min) / (geom.nq - 1)
    fp = f_idx / (geom.nfft * geom.dt_str)                     # f'
    u = (fp[:, None] * geom.h2[None, :] * dq * mg) % mg          # k / dk, reduced by the period
    i = np.floor(u).astype(np.int64)
    a = u - i
    return i % mg, (i + 1) % mg, a


def _azimuth_cells(geom: Geometry):
    """Lower azimuth bin j_n, upper bin (j_n + 1) mod ntheta and alpha_n of every trace."""
    W = geom.W()
    ntr = W.shape[0]
    jlo = np.zeros(ntr, dtype=np.int64)
    alpha = np.zeros(ntr)
    dth = math.pi / geom.ntheta
    for n in range(ntr):
        if geom.x[n] == 0.0 and geom.y[n] == 0.0:
            th = 0.0
        else:
            th = math.atan2(geom.y[n], geom.x[n]) % math.pi
        u = th / dth
        j = int(math.floor(u))
        a = u - j
        if j >= geom.ntheta:
            j -= geom.ntheta
        jlo[n] = j
        alpha[n] = a
    return jlo, (jlo + 1) % geom.ntheta, alpha


def k_grid(mh: np.ndarray, geom: Geometry, mg: int) -> np.ndarray:
    """Step 2, q half: G[j, i, f] = sum_l Mh[j, l, f] exp(-2 pi i (l - nq//2) i / mg), i < mg."""
    lc = np.arange(geom.nq) - geom.nq // 2
    i = np.arange(mg)
    E = np.exp(-2j * np.pi * np.outer(i, lc) / mg)              # [mg, nq]
    return np.einsum('il,jlf->jif', E, mh)


def q_centre(geom: Geometry) -> float:
    dq = (geom.q_max - geom.q_min) / (geom.nq - 1)
    return geom.q_min + (geom.nq // 2) * dq


def linear_map(mh: np.ndarray, geom: Geometry, mg: int) -> np.ndarray:
    """Step 3 with the A1..A4 interpolation: Mh[theta, q, f] -> Dh[trace, f]."""
    G = k_grid(mh, geom, mg)
    jlo, jhi, alpha = _azimuth_cells(geom)
    f_idx = np.arange(geom.nf)
    i0, i1, a = _trace_cells(geom, mg, f_idx)                    # [nf, ntr]
    fsel = f_idx[:, None]
    A1 = (1 - a) * (1 - alpha)[None, :]
    A2 = (1 - a) * alpha[None, :]
    A3 = a * (1 - alpha)[None, :]
    A4 = a * alpha[None, :]
    dc = (A1 * G[jlo[None, :], i0, fsel] + A2 * G[jhi[None, :], i0, fsel]
          + A3 * G[jlo[None, :], i1, fsel] + A4 * G[jhi[None, :], i1, fsel])   # [nf, ntr]
    fp = f_idx / (geom.nfft * geom.dt_str)
    nmo = np.exp(-2j * np.pi * fp[:, None] * q_centre(geom) * geom.h2[None, :])
    return (nmo * dc).T


def linear_map_T(gh: np.ndarray, geom: Geometry, mg: int) -> np.ndarray:
    """Transpose of linear_map: Gh[trace, f] -> Hh[theta, q, f]."""
    jlo, jhi, alpha = _azimuth_cells(geom)
    f_idx = np.arange(geom.nf)
    i0, i1, a = _trace_cells(geom, mg, f_idx)
    fp = f_idx / (geom.nfft * geom.dt_str)
    nmo_c = np.exp(2j * np.pi * fp[:, None] * q_centre(geom) * geom.h2[None, :])
    v = nmo_c * gh.T                                            # [nf, ntr]
    Gt = np.zeros((geom.ntheta, mg, geom.nf), dtype=np.complex128)
    fsel = np.broadcast_to(f_idx[:, None], i0.shape)
    for jj, ii, cw in ((jlo, i0, (1 - a) * (1 - alpha)[None, :]), (jhi, i0, (1 - a) * alpha[None, :]),
                       (jlo, i1, a * (1 - alpha)[None, :]), (jhi, i1, a * alpha[None, :])):
        np.add.at(Gt, (np.broadcast_to(jj[None, :], ii.shape), ii, fsel), cw * v)
    lc = np.arange(geom.nq) - geom.nq // 2
    i = np.arange(mg)
    Ec = np.exp(2j * np.pi * np.outer(lc, i) / mg)              # [nq, mg], conjugate of k_grid's
    return np.einsum('li,jif->jlf', Ec, Gt)


def forward(m: np.ndarray, geom: Geometry, mg: int) -> np.ndarray:
    """d = L_lin m for one gather: Algorithm 1 with the Section 3.4 step 3 on an mg-point k grid."""
    m = np.asarray(m, dtype=np.float64)
    mh = gfst.spectrum(gfst.stretch(m, geom), geom)
    dh = linear_map(mh, geom, mg)
    return gfst.unstretch(gfst.inverse_spectrum(dh, geom), geom)


def adjoint(d: np.ndarray, geom: Geometry, mg: int) -> np.ndarray:
    """m = L_lin^T d, the exact transpose of forward."""
    d = np.asarray(d, dtype=np.float64)
    gh = gfst.inverse_spectrum_T(gfst.unstretch_T(d, geom), geom)
    hh = linear_map_T(gh, geom, mg)
    return gfst.stretch_T(gfst.spectrum_T(hh, geom), geom)
