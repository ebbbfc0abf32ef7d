"""Seeded synthetic CMP workloads shared by the oracle, the tests and the benchmark.

This module holds geometry, axes and synthetic data only.  It contains none of
the Radon operator's arithmetic: no stretch, no Fourier transform, no
curvature/azimuth mapping.  Both the FP64 oracle and the HIP path take their
inputs from here, so neither depends on the other.

Units used throughout: time in s, offsets in km, curvature q (squared
slowness) in s^2/km^2.  The configs below mirror the synthetic CMP gathers of
Section 5 of the paper (hyperbolic events whose velocity depends on azimuth;
the paper's own gather is shown only as a figure, so these seeded gathers
stand in for it).

Event model (Section 2.1, elliptical anisotropy): an event with intercept
tau0 and 2x2 SPD slowness matrix W arrives at t^2 = tau0^2 + h^T W h, where
W = R(phi) diag(p1^2, p2^2) R(phi)^T.  Each event is a Ricker wavelet
r(t) = (1 - 2 pi^2 f0^2 t^2) exp(-pi^2 f0^2 t^2) with amplitude N(0,1); white
Gaussian noise is added at SNR = rms(clean) / sigma over the gather.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 250500387


@dataclass(frozen=True)
class Axes:
    """Discrete axes of one operator plan (shared by every gather of a batch)."""
    nt: int            # data time samples, t_s = s*dt
    dt: float          # s
    ntau: int          # model intercept samples, tau_i = i*dtau
    dtau: float        # s
    nq: int            # curvature samples, uniform in [q_min, q_max] inclusive
    q_min: float       # s^2/km^2
    q_max: float       # s^2/km^2
    ntheta: int        # azimuth samples theta_j = j*pi/ntheta
    stretch: int = 2   # nt' = stretch * nt

    @property
    def dq(self) -> float:
        return (self.q_max - self.q_min) / (self.nq - 1)


@dataclass
class Gather:
    x: np.ndarray                 # km, [ntr]
    y: np.ndarray                 # km, [ntr]
    data: Optional[np.ndarray] = None   # [ntr, nt] synthetic observed data
    events: list = field(default_factory=list)


@dataclass
class Workload:
    name: str
    axes: Axes
    gathers: List[Gather]
    n_iter: int
    description: str

    @property
    def batch(self) -> int:
        return len(self.gathers)

    @property
    def trace_ptr(self) -> np.ndarray:
        ptr = np.zeros(self.batch + 1, dtype=np.int64)
        ptr[1:] = np.cumsum([g.x.size for g in self.gathers])
        return ptr

    @property
    def x_all(self) -> np.ndarray:
        return np.concatenate([g.x for g in self.gathers]) if self.gathers else np.zeros(0)

    @property
    def y_all(self) -> np.ndarray:
        return np.concatenate([g.y for g in self.gathers]) if self.gathers else np.zeros(0)

    def data_all(self) -> np.ndarray:
        return np.concatenate([g.data for g in self.gathers], axis=0)


def config_rng(config: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([SEED_BASE, config])


def gather_rngs(config: int, batch: int) -> List[np.random.Generator]:
    return [np.random.default_rng(s) for s in config_rng(config).spawn(batch)]


def ricker(t: np.ndarray, f0: float) -> np.ndarray:
    a = (np.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def _event_matrix(rng, p_lo, p_hi):
    p1, p2 = rng.uniform(p_lo, p_hi, size=2)
    phi = rng.uniform(0.0, np.pi)
    c, s = np.cos(phi), np.sin(phi)
    R = np.array([[c, -s], [s, c]])
    return R @ np.diag([p1 * p1, p2 * p2]) @ R.T


def synth_data(axes: Axes, x, y, events, snr: Optional[float], rng) -> np.ndarray:
    """Sum of Ricker events on t^2 = tau0^2 + h^T W h, plus noise at the given SNR.

    Each wavelet is evaluated on the samples within 1.6/f0 of its arrival time (its
    amplitude there is below 1e-11 of the peak) and is zero elsewhere.
    """
    d = np.zeros((x.size, axes.nt))
    h = np.stack([x, y], axis=1)
    rows = np.arange(x.size)[:, None]
    for ev in events:
        hw = np.einsum('ni,ij,nj->n', h, ev['W'], h)
        tev = np.sqrt(ev['tau0'] ** 2 + hw)
        half = int(np.ceil(1.6 / (ev['f0'] * axes.dt)))
        idx = np.rint(tev / axes.dt).astype(np.int64)[:, None] + np.arange(-half, half + 1)[None, :]
        ok = (idx >= 0) & (idx < axes.nt)
        vals = ev['amp'] * ricker(idx * axes.dt - tev[:, None], ev['f0'])
        rr = np.broadcast_to(rows, idx.shape)
        d[rr[ok], idx[ok]] += vals[ok]
    if snr is not None and d.size:
        rms = np.sqrt(np.mean(d * d))
        d += rng.standard_normal(d.shape) * (rms / snr)
    return d


def disk_offsets(rng, n, radius):
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, n))
    a = rng.uniform(0.0, 2.0 * np.pi, n)
    return r * np.cos(a), r * np.sin(a)


def _events(rng, n, tau_lo, tau_hi, p_lo, p_hi, f_lo, f_hi):
    evs = []
    for _ in range(n):
        evs.append(dict(tau0=rng.uniform(tau_lo, tau_hi), W=_event_matrix(rng, p_lo, p_hi),
                        amp=rng.standard_normal(), f0=rng.uniform(f_lo, f_hi)))
    return evs


def _flat_multiples(rng, n, tau_lo, tau_hi, p_lo, f_lo, f_hi):
    evs = []
    for _ in range(n):
        p = rng.uniform(p_lo, p_lo + 0.05)
        evs.append(dict(tau0=rng.uniform(tau_lo, tau_hi), W=np.eye(2) * p * p,
                        amp=rng.standard_normal(), f0=rng.uniform(f_lo, f_hi)))
    return evs


def config1(with_data: bool = True) -> Workload:
    """Single CMP: nt=256 @ 4 ms, 16x16 regular offsets on [-1,1]^2 km, nq=32, ntheta=8."""
    ax = Axes(nt=256, dt=0.004, ntau=256, dtau=0.004, nq=32,
              q_min=0.25 ** 2, q_max=0.67 ** 2, ntheta=8)
    rng = gather_rngs(1, 1)[0]
    g1 = np.linspace(-1.0, 1.0, 16)
    X, Y = np.meshgrid(g1, g1, indexing='ij')
    g = Gather(x=X.ravel().copy(), y=Y.ravel().copy())
    if with_data:
        g.events = _events(rng, 5, 0.1, 0.9, 0.25, 0.67, 25.0, 25.0)
        g.data = synth_data(ax, g.x, g.y, g.events, 10.0, rng)
    return Workload('cmp_single_nt256', ax, [g], 20,
                    'single CMP, 256 traces on a 16x16 grid, nt=256, nq=32, ntheta=8')


def config2(with_data: bool = True) -> Workload:
    """Realistic CMP: nt=1024 @ 2 ms, 1024 traces in a disk of 3 km, nq=64, ntheta=16."""
    ax = Axes(nt=1024, dt=0.002, ntau=1024, dtau=0.002, nq=64,
              q_min=0.2 ** 2, q_max=0.7 ** 2, ntheta=16)
    rng = gather_rngs(2, 1)[0]
    x, y = disk_offsets(rng, 1024, 3.0)
    g = Gather(x=x, y=y)
    if with_data:
        T = (ax.nt - 1) * ax.dt
        g.events = (_events(rng, 12, 0.1, 0.8 * T, 0.2, 0.7, 20.0, 30.0)
                    + _flat_multiples(rng, 4, 0.1, 0.8 * T, 0.2, 20.0, 30.0))
        g.data = synth_data(ax, g.x, g.y, g.events, 5.0, rng)
    return Workload('cmp_realistic_nt1024', ax, [g], 100,
                    'one CMP, 1024 traces in a 3 km disk, nt=1024, nq=64, ntheta=16')


def config3(with_data: bool = True) -> Workload:
    """Differentiation batch: 8 CMPs on config-1 axes, 512 traces uniform in [-1,1]^2 km."""
    ax = config1(with_data=False).axes
    gs = []
    for rng in gather_rngs(3, 8):
        x = rng.uniform(-1.0, 1.0, 512)
        y = rng.uniform(-1.0, 1.0, 512)
        g = Gather(x=x, y=y)
        if with_data:
            g.events = _events(rng, 5, 0.1, 0.9, 0.25, 0.67, 25.0, 25.0)
            g.data = synth_data(ax, g.x, g.y, g.events, 10.0, rng)
        gs.append(g)
    return Workload('cmp_batch8_nt256', ax, gs, 20,
                    '8 CMPs x 512 irregular traces, config-1 axes')


def config4(with_data: bool = True, batch: int = 256) -> Workload:
    """Batched uneven folds: 256 CMPs, fold ~U[200,1200], disk 3 km, nt=1024 @ 2 ms, nq=64, ntheta=16."""
    ax = config2(with_data=False).axes
    T = (ax.nt - 1) * ax.dt
    gs = []
    for rng in gather_rngs(4, 256)[:batch]:
        fold = int(rng.integers(200, 1201))
        x, y = disk_offsets(rng, fold, 3.0)
        g = Gather(x=x, y=y)
        if with_data:
            g.events = _events(rng, int(rng.integers(5, 16)), 0.1, 0.8 * T, 0.2, 0.7, 20.0, 30.0)
            g.data = synth_data(ax, g.x, g.y, g.events, 5.0, rng)
        gs.append(g)
    return Workload('cmp_batch256_uneven_nt1024', ax, gs, 100,
                    '256 CMPs, fold U[200,1200] in a 3 km disk, nt=1024, nq=64, ntheta=16')


def config5(with_data: bool = True, batch: int = 32) -> Workload:
    """Large: 32 CMPs, nt=2048 @ 1 ms, 4096 traces in a 4 km disk, nq=128, ntheta=36."""
    ax = Axes(nt=2048, dt=0.001, ntau=2048, dtau=0.001, nq=128,
              q_min=0.2 ** 2, q_max=0.7 ** 2, ntheta=36)
    T = (ax.nt - 1) * ax.dt
    gs = []
    for rng in gather_rngs(5, 32)[:batch]:
        x, y = disk_offsets(rng, 4096, 4.0)
        g = Gather(x=x, y=y)
        if with_data:
            g.events = _events(rng, int(rng.integers(5, 16)), 0.1, 0.8 * T, 0.2, 0.7, 20.0, 30.0)
            g.data = synth_data(ax, g.x, g.y, g.events, 10.0, rng)
        gs.append(g)
    return Workload('cmp_batch32_nt2048', ax, gs, 100,
                    '32 CMPs x 4096 traces in a 4 km disk, nt=2048, nq=128, ntheta=36')


def table1(nt: int, nxy: int, np_: int, ntheta: int = 90, with_data: bool = True) -> Workload:
    """Velocity-scan shape of the paper's timing table (Section 5): one CMP on a regular
    nxy x nxy offset grid at 40 m, centred on zero offset, nt samples at 4 ms, np_ curvatures
    uniform in [0.2^2, 0.7^2] s^2/km^2 (the slowness range is not stated; this one is the
    other workloads'), ntheta azimuths.  Data: 8 anisotropic 25 Hz Ricker events without
    noise (the timing of a linear operator does not depend on its input; band-limited data
    make the difference between two discretisations of the adjoint meaningful)."""
    ax = Axes(nt=nt, dt=0.004, ntau=nt, dtau=0.004, nq=np_, q_min=0.2 ** 2, q_max=0.7 ** 2,
              ntheta=ntheta)
    g1 = (np.arange(nxy) - (nxy - 1) / 2.0) * 0.040
    X, Y = np.meshgrid(g1, g1, indexing='ij')
    g = Gather(x=X.ravel().copy(), y=Y.ravel().copy())
    if with_data:
        rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 4000 + nt + nxy + np_]))
        T = (nt - 1) * ax.dt
        g.events = _events(rng, 8, 0.1, 0.8 * T, 0.2, 0.7, 25.0, 25.0)
        g.data = synth_data(ax, g.x, g.y, g.events, None, rng)
    return Workload(f'table1_nt{nt}_grid{nxy}_np{np_}', ax, [g], 0,
                    f'one CMP, {nxy}x{nxy} offsets at 40 m, nt={nt} at 4 ms, nq={np_}, ntheta={ntheta}')


TABLE1_SHAPES = [(512, 128, 128), (512, 128, 256), (512, 256, 128), (512, 256, 256),
                 (1024, 128, 128), (1024, 128, 256), (1024, 256, 128), (1024, 256, 256)]


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def random_model(axes: Axes, batch: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) model cube [batch, ntheta, nq, ntau] in FP64."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 1000 + seed]))
    return rng.standard_normal((batch, axes.ntheta, axes.nq, axes.ntau))


def random_data(ntr: int, nt: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 2000 + seed]))
    return rng.standard_normal((ntr, nt))


def small_case(nt=32, ntr=7, nq=5, ntheta=3, seed=0, q_min=0.05, q_max=0.4,
               radius=1.0, stretch=2, ntau=None, dtau=None, dt=0.02) -> Workload:
    """Tiny random case for brute-force tests."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 3000 + seed]))
    ntau = nt if ntau is None else ntau
    dtau = dt if dtau is None else dtau
    ax = Axes(nt=nt, dt=dt, ntau=ntau, dtau=dtau, nq=nq, q_min=q_min, q_max=q_max,
              ntheta=ntheta, stretch=stretch)
    x, y = disk_offsets(rng, ntr, radius)
    return Workload('tiny', ax, [Gather(x=x, y=y)], 5, 'tiny brute-force case')
