"""Algorithm 2 (Section 3.2): the paper's fast velocity stack, with the (x, y)-grid bilinear
interpolation of Section 3.4 (coefficients B1..B4).  FP64.  Test infrastructure only.

Unlike oracle-1's adjoint this is not the transpose of the forward operator: step 3 reads
the data spectrum at the one offset that the GFST relation of Section 3.2 assigns to each
model coefficient, x = sqrt(k/f') cos(theta), y = sqrt(k/f') sin(theta), on a regular
(x_m, y_n) grid.  The five steps, in the paper's order:

1. stretch the data along time by interpolation, D'(t') = D(t = sqrt(t'))  (linear);
2. real DFT along t' (bins f = 0..N/2-1);
3. Mh(f', k_p, theta_j) = B1 Dh(x_m, y_n) + B2 Dh(x_m, y_n+1) + B3 Dh(x_m+1, y_n)
                          + B4 Dh(x_m+1, y_n+1)
   at the point above, for the k grid dual to the uniform q axis, k_p = p/(nq dq),
   p = -nq/2 .. nq/2-1 (FFT order), and f' = f/(N dt');
4. inverse 2-D DFT along f' and k:
       G(f, q_l)  = (1/nq) sum_p Mh(f', k_p) exp(+2 pi i k_p q_l),  q_l = q_min + l dq
       M'(tau'_r) = (1/N) (G(0) + 2 Re sum_{f=1}^{N/2-1} G(f) exp(+2 pi i f r/N))
   (the negative-frequency half is the complex conjugate, as for any real cube);
5. undo the stretch by interpolation, M(tau_i) = M'(tau' = tau_i^2)  (linear).

Readings (where the paper is silent): a point with k < 0 (no real offset), at f' = 0, or
outside the grid gives 0; the grid is x_m = x_0 + m dx, y_n = y_0 + n dy (the paper
writes x_m = m dx, a grid starting at zero offset); a point on the last grid line uses
the last cell.  Only the offset with y >= 0 is read, as the printed relation gives; the
mirror offset (-x, -y) shares the same azimuth and is not read.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, stretch_matrix, unstretch_matrix


def regular_grid(x: np.ndarray, y: np.ndarray, tol: float = 1e-9):
    """(x0, dx, mx, y0, dy, my, node) of a complete regular offset grid, node[n] = (m, k)
    of trace n; ValueError if the traces do not fill such a grid exactly once."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)

    def axis(v):
        u = np.unique(np.round(v / tol) * tol)
        if u.size < 2:
            raise ValueError('a regular grid needs at least two lines per axis')
        step = (u[-1] - u[0]) / (u.size - 1)
        if np.max(np.abs(u - (u[0] + step * np.arange(u.size)))) > 1e-6 * step:
            raise ValueError('offsets are not uniformly spaced')
        return float(u[0]), float(step), int(u.size)

    x0, dx, mx = axis(x)
    y0, dy, my = axis(y)
    m = np.rint((x - x0) / dx).astype(np.int64)
    k = np.rint((y - y0) / dy).astype(np.int64)
    if x.size != mx * my or np.unique(m * my + k).size != x.size:
        raise ValueError('traces do not fill the grid exactly once')
    return x0, dx, mx, y0, dy, my, np.stack([m, k], axis=1)


def stretch_data(d: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 1: [ntr, nt] -> [ntr, nt']."""
    return np.asarray(d, dtype=np.float64) @ stretch_matrix(geom.nt, geom.dt, geom.nt_str, geom.dt_str).T


def data_spectrum(dp: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 2: [..., nt'] -> [..., N/2] complex."""
    return np.fft.rfft(dp, n=geom.nfft, axis=-1)[..., :geom.nf]


def k_axis(geom: Geometry) -> np.ndarray:
    """k_p = p/(nq dq) for p = 0..nq-1 in FFT order (p >= nq/2 stands for p - nq)."""
    dq = (geom.q_max - geom.q_min) / (geom.nq - 1)
    p = np.arange(geom.nq)
    p = np.where(p < (geom.nq + 1) // 2, p, p - geom.nq)
    return p / (geom.nq * dq)


def bilinear(dh_grid: np.ndarray, grid, px: float, py: float) -> np.ndarray:
    """Step 3 at one point: B1..B4 of Section 3.4 applied to dh_grid[m, n, :] (0 outside)."""
    x0, dx, mx, y0, dy, my = grid
    u = (px - x0) / dx
    v = (py - y0) / dy
    if not (0.0 <= u <= mx - 1 and 0.0 <= v <= my - 1):
        return np.zeros(dh_grid.shape[2:], dtype=dh_grid.dtype)
    m = min(int(np.floor(u)), mx - 2)
    n = min(int(np.floor(v)), my - 2)
    xm, xm1 = x0 + m * dx, x0 + (m + 1) * dx
    yn, yn1 = y0 + n * dy, y0 + (n + 1) * dy
    b1 = (xm1 - px) * (yn1 - py) / (dx * dy)
    b2 = -(xm1 - px) * (yn - py) / (dx * dy)
    b3 = -(xm - px) * (yn1 - py) / (dx * dy)
    b4 = (xm - px) * (yn - py) / (dx * dy)
    return (b1 * dh_grid[m, n] + b2 * dh_grid[m, n + 1] + b3 * dh_grid[m + 1, n]
            + b4 * dh_grid[m + 1, n + 1])


def polar_map(dh_grid: np.ndarray, grid, geom: Geometry) -> np.ndarray:
    """Step 3: Dh on the (x_m, y_n) grid [mx, my, N/2] -> Mh [ntheta, nq (FFT order), N/2]."""
    k = k_axis(geom)
    fp = geom.fprime
    theta = np.pi * np.arange(geom.ntheta) / geom.ntheta
    mh = np.zeros((geom.ntheta, geom.nq, geom.nf), dtype=np.complex128)
    for j, th in enumerate(theta):
        for p, kp in enumerate(k):
            if kp < 0.0:
                continue
            for f in range(1, geom.nf):
                r = np.sqrt(kp / fp[f])
                mh[j, p, f] = bilinear(dh_grid[:, :, f:f + 1], grid, r * np.cos(th), r * np.sin(th))[0]
    return mh


def inverse_2d(mh: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 4: Mh [ntheta, nq (FFT order), N/2] -> M' [ntheta, nq, nt']."""
    E = np.exp(2j * np.pi * np.outer(k_axis(geom), geom.q))          # [p, l]
    G = np.einsum('jpf,pl->jlf', mh, E) / geom.nq
    full = np.zeros(G.shape[:2] + (geom.nf + 1,), dtype=np.complex128)
    full[..., :geom.nf] = G
    return np.fft.irfft(full, n=geom.nfft, axis=-1)[..., :geom.nt_str]


def unstretch_model(mp: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 5: M' [..., nt'] -> M [..., ntau], M(tau_i) = M'(tau_i^2)."""
    return mp @ unstretch_matrix(geom.ntau, geom.dtau, geom.nt_str, geom.dt_str).T


def adjoint(d: np.ndarray, geom: Geometry) -> np.ndarray:
    """Algorithm 2 on one gather whose traces fill a regular grid: d [ntr, nt] -> M [ntheta, nq, ntau]."""
    x0, dx, mx, y0, dy, my, node = regular_grid(geom.x, geom.y)
    dh = data_spectrum(stretch_data(d, geom), geom)
    dh_grid = np.zeros((mx, my, geom.nf), dtype=np.complex128)
    dh_grid[node[:, 0], node[:, 1]] = dh
    mh = polar_map(dh_grid, (x0, dx, mx, y0, dy, my), geom)
    return unstretch_model(inverse_2d(mh, geom), geom)
