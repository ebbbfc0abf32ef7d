"""Discrete geometry of the AAHRT (FP64).  Test infrastructure only.

Readings of the paper used here (each is one line of the design notes):
* stretch t' = t^2 and tau' = tau^2 (Section 3.1); the stretched axis has
  nt' = K*nt samples on [0, T^2], T = (nt-1)*dt, so dt' = T^2/(nt'-1), and is
  shared by the model and the data side;
* S and S^-1 are local interpolators (Section 3.4); read as linear
  interpolation, with positions computed in FP64 and taps outside the target
  axis dropped;
* curvature q (squared slowness, Section 2) is the uniformly sampled axis,
  q_l = q_min + l*dq, dq = (q_max-q_min)/(nq-1);
* azimuth theta = arctan(y/x) has period pi; grid theta_j = j*pi/ntheta and a
  trace's weights are the linear ones of the A1..A4 coefficients of
  Section 3.4 restricted to theta, with the bin found by floor and the upper
  neighbour wrapped modulo ntheta; a zero-offset trace takes theta = 0;
* FFT length: the smallest even 2^a 3^b 5^c that is at least nt' plus the
  largest stretched-time shift q*h^2/dt' (both signs), so the circular
  transform does not wrap an event of the cube onto the kept samples.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def is_smooth235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def nfft_rule(nt_str: int, dt_str: float, q_min: float, q_max: float, h2max: float) -> int:
    """Smallest even 2^a3^b5^c >= nt' + ceil(max(q_max,0) h2max/dt') + ceil(max(-q_min,0) h2max/dt')."""
    need = nt_str + math.ceil(max(q_max, 0.0) * h2max / dt_str) \
        + math.ceil(max(-q_min, 0.0) * h2max / dt_str)
    n = max(need, 2)
    while True:
        if n % 2 == 0 and is_smooth235(n):
            return n
        n += 1


def theta_weights(x: np.ndarray, y: np.ndarray, ntheta: int) -> np.ndarray:
    """Dense [ntr, ntheta] matrix of linear azimuth weights w_{n,j}."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.zeros((x.size, ntheta))
    dth = np.pi / ntheta
    for n in range(x.size):
        if x[n] == 0.0 and y[n] == 0.0:
            th = 0.0
        else:
            th = math.atan2(y[n], x[n]) % math.pi
        u = th / dth
        j = int(math.floor(u))
        a = u - j
        if j >= ntheta:          # theta rounded up to pi
            j -= ntheta
        w[n, j] += 1.0 - a
        w[n, (j + 1) % ntheta] += a
    return w


def stretch_matrix(ntau: int, dtau: float, nt_str: int, dt_str: float) -> np.ndarray:
    """S [nt', ntau]: M'(tau'_r) = linear interpolation of M at tau = sqrt(r dt')."""
    S = np.zeros((nt_str, ntau))
    for r in range(nt_str):
        pos = math.sqrt(r * dt_str) / dtau
        i = int(math.floor(pos))
        a = pos - i
        if 0 <= i < ntau:
            S[r, i] += 1.0 - a
        if 0 <= i + 1 < ntau:
            S[r, i + 1] += a
    return S


def unstretch_matrix(nt: int, dt: float, nt_str: int, dt_str: float) -> np.ndarray:
    """U [nt, nt']: d(t_s) = linear interpolation of D' at t' = (s dt)^2."""
    U = np.zeros((nt, nt_str))
    for s in range(nt):
        pos = (s * dt) ** 2 / dt_str
        r = int(math.floor(pos))
        b = pos - r
        if 0 <= r < nt_str:
            U[s, r] += 1.0 - b
        if 0 <= r + 1 < nt_str:
            U[s, r + 1] += b
    return U


@dataclass
class Geometry:
    """Everything the oracle needs for one gather on a given set of axes."""
    nt: int
    dt: float
    ntau: int
    dtau: float
    nq: int
    q_min: float
    q_max: float
    ntheta: int
    stretch: int
    x: np.ndarray
    y: np.ndarray
    nfft: int

    @classmethod
    def build(cls, axes, x, y, nfft: int | None = None, h2max: float | None = None):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        nt_str = axes.stretch * axes.nt
        T = (axes.nt - 1) * axes.dt
        dt_str = T * T / (nt_str - 1)
        if nfft is None:
            if h2max is None:
                h2max = float(np.max(x * x + y * y)) if x.size else 0.0
            nfft = nfft_rule(nt_str, dt_str, axes.q_min, axes.q_max, h2max)
        return cls(axes.nt, axes.dt, axes.ntau, axes.dtau, axes.nq, axes.q_min, axes.q_max,
                   axes.ntheta, axes.stretch, x, y, int(nfft))

    # derived quantities -------------------------------------------------
    @property
    def nt_str(self) -> int:
        return self.stretch * self.nt

    @property
    def dt_str(self) -> float:
        T = (self.nt - 1) * self.dt
        return T * T / (self.nt_str - 1)

    @property
    def nf(self) -> int:
        return self.nfft // 2

    @property
    def q(self) -> np.ndarray:
        dq = (self.q_max - self.q_min) / (self.nq - 1)
        return self.q_min + dq * np.arange(self.nq)

    @property
    def h2(self) -> np.ndarray:
        return self.x * self.x + self.y * self.y

    @property
    def fprime(self) -> np.ndarray:
        """Stretched-axis frequencies f'_f = f/(N dt'), f = 0..N/2-1 (1/s^2)."""
        return np.arange(self.nf) / (self.nfft * self.dt_str)

    def S(self) -> np.ndarray:
        return stretch_matrix(self.ntau, self.dtau, self.nt_str, self.dt_str)

    def U(self) -> np.ndarray:
        return unstretch_matrix(self.nt, self.dt, self.nt_str, self.dt_str)

    def W(self) -> np.ndarray:
        return theta_weights(self.x, self.y, self.ntheta)

    def subset(self, idx) -> 'Geometry':
        idx = np.asarray(idx)
        return Geometry(self.nt, self.dt, self.ntau, self.dtau, self.nq, self.q_min, self.q_max,
                        self.ntheta, self.stretch, self.x[idx], self.y[idx], self.nfft)
