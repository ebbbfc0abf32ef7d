"""Pins for the FP64 oracle: closed forms, invariants, brute force and special cases.

Each test checks the oracle against something other than itself (a second
formula, a hand-derived value, a library routine, or an invariant of the
mathematics), so that a dropped term, a wrong sign, index or scale fails one
of them.  CPU only.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import gfst, timedomain, fista
from oracle.geometry import Geometry, nfft_rule, theta_weights, stretch_matrix, unstretch_matrix
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), 'golden')


def _tiny(seed=0, **kw):
    w = wl.small_case(seed=seed, **kw)
    return w, Geometry.build(w.axes, w.gathers[0].x, w.gathers[0].y)


# ------------------------------------------------------------------ geometry
def test_theta_weights_golden():
    """Hand-derived azimuth weights (Section 3.4, theta part of A1..A4, period pi, wrap)."""
    g = json.load(open(os.path.join(GOLDEN, 'theta_weights.json')))
    nth = g['ntheta']
    for case in g['cases']:
        if 'angle_over_pi' in case:
            a = case['angle_over_pi'] * math.pi
            x, y = 1.7 * math.cos(a), 1.7 * math.sin(a)
        else:
            x, y = case['x'], case['y']
        w = theta_weights(np.array([x]), np.array([y]), nth)[0]
        want = np.zeros(nth)
        for k, v in case['weights'].items():
            want[int(k)] = v
        np.testing.assert_allclose(w, want, atol=1e-12)


def test_theta_weights_hat_functions():
    """Linear azimuth weights equal periodic hat functions max(0, 1 - dist(theta, theta_j)/dtheta)."""
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal(500), rng.standard_normal(500)
    for nth in (1, 3, 8, 16):
        w = theta_weights(x, y, nth)
        dth = np.pi / nth
        th = np.mod(np.arctan2(y, x), np.pi)
        grid = np.arange(nth) * dth
        d = np.abs(th[:, None] - grid[None, :])
        d = np.minimum(d, np.pi - d)                    # circular distance on a period of pi
        hat = np.maximum(0.0, 1.0 - d / dth)
        if nth == 1:
            hat = np.ones_like(hat)
        np.testing.assert_allclose(w, hat, atol=1e-12)
        np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-14)


def test_fft_length_golden():
    g = json.load(open(os.path.join(GOLDEN, 'fft_lengths.json')))
    for c in g['cases']:
        nts = 2 * c['nt']
        T = (c['nt'] - 1) * c['dt']
        dts = T * T / (nts - 1)
        assert abs(c['q_max'] * c['h2max'] / dts - c['shift']) < 0.01
        assert nfft_rule(nts, dts, c['q_min'], c['q_max'], c['h2max']) == c['nfft']


def test_stretch_reproduces_linear_functions():
    """Linear interpolation is exact on linear functions: S maps a + b*tau to a + b*sqrt(tau')."""
    for (ntau, dtau, nts, dts) in [(64, 0.01, 128, 0.63 ** 2 / 127), (256, 0.004, 512, 1.02 ** 2 / 511)]:
        S = stretch_matrix(ntau, dtau, nts, dts)
        m = 0.3 + 2.0 * np.arange(ntau) * dtau
        tau_s = np.sqrt(np.arange(nts) * dts)
        inside = tau_s <= (ntau - 1) * dtau
        np.testing.assert_allclose((S @ m)[inside], (0.3 + 2.0 * tau_s)[inside], atol=1e-12)
        assert np.all(S.sum(1)[inside] > 1 - 1e-12)


def test_unstretch_reproduces_linear_functions():
    """U maps a + b*t' to a + b*t^2 on the whole data axis (t'_max = T^2 is the last stretched sample)."""
    for (nt, dt, K) in [(32, 0.02, 2), (256, 0.004, 2), (100, 0.01, 1), (64, 0.005, 3)]:
        nts = K * nt
        T = (nt - 1) * dt
        dts = T * T / (nts - 1)
        U = unstretch_matrix(nt, dt, nts, dts)
        dp = -1.0 + 0.7 * np.arange(nts) * dts
        t = np.arange(nt) * dt
        np.testing.assert_allclose(U @ dp, -1.0 + 0.7 * t * t, atol=1e-12)


# ------------------------------------------------------------------ oracle-1
def _dot_test(L, Lt, m, d):
    a = np.sum(L(m) * d)
    b = np.sum(m * Lt(d))
    return abs(a - b) / max(abs(a), abs(b))


@pytest.mark.parametrize('seed', [0, 1, 2])
def test_dot_test_gfst(seed):
    w, g = _tiny(seed, ntheta=3 + seed)
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    d = rng.standard_normal((g.x.size, g.nt))
    assert _dot_test(lambda v: gfst.forward(v, g), lambda v: gfst.adjoint(v, g), m, d) < 1e-12


def test_dot_test_gfst_config1():
    w = wl.config1(with_data=False)
    g = Geometry.build(w.axes, w.gathers[0].x, w.gathers[0].y)
    rng = np.random.default_rng(11)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    d = rng.standard_normal((g.x.size, g.nt))
    assert _dot_test(lambda v: gfst.forward(v, g), lambda v: gfst.adjoint(v, g), m, d) < 1e-12


def _dirichlet(x, N):
    """K_N(x) = (1/N)(1 + 2 sum_{f=1}^{N/2-1} cos(2 pi f x/N)) in closed form."""
    F = N // 2
    phi = 2 * np.pi * x / N
    s = np.sin(phi / 2)
    out = np.empty_like(phi)
    small = np.abs(s) < 1e-12
    out[~small] = np.sin((F - 0.5) * phi[~small]) / s[~small]
    out[small] = (2 * F - 1) * np.cos((F - 0.5) * phi[small]) / np.cos(phi[small] / 2)
    return out / N


@pytest.mark.parametrize('seed', [0, 3])
def test_gfst_equals_periodic_sinc_closed_form(seed):
    """Steps 2-4 equal a band-limited periodic-sinc shift by q h^2/dt' on the stretched axis."""
    w, g = _tiny(seed, ntheta=4)
    rng = np.random.default_rng(100 + seed)
    mp = rng.standard_normal((g.ntheta, g.nq, g.nt_str))
    got = gfst.inverse_spectrum(gfst.gfst_map(gfst.spectrum(mp, g), g), g)
    # independent azimuth weights: periodic hat functions
    dth = np.pi / g.ntheta
    th = np.mod(np.arctan2(g.y, g.x), np.pi)
    dist = np.abs(th[:, None] - np.arange(g.ntheta)[None, :] * dth)
    dist = np.minimum(dist, np.pi - dist)
    W = np.maximum(0.0, 1.0 - dist / dth)
    r = np.arange(g.nt_str)
    want = np.zeros_like(got)
    for n in range(g.x.size):
        for l, ql in enumerate(g.q):
            sh = ql * (g.x[n] ** 2 + g.y[n] ** 2) / g.dt_str
            K = _dirichlet(r[:, None] - r[None, :] - sh, g.nfft)      # [r_out, r_in]
            want[n] += (W[n] @ mp[:, l, :]) @ K.T
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-12


def _band_project(v, N):
    """Remove the Nyquist component of a length-N real sequence: v - (1/N)(sum v (-1)^r)(-1)^r."""
    sgn = (-1.0) ** np.arange(N)
    return v - (np.sum(v * sgn) / N) * sgn


def test_zero_offset_trace_is_band_projection():
    """h = 0: no shift; D' is the Nyquist-free part of sum_j w_j sum_l M'."""
    w, g = _tiny(0, ntheta=5)
    g = Geometry(g.nt, g.dt, g.ntau, g.dtau, g.nq, g.q_min, g.q_max, g.ntheta, g.stretch,
                 np.array([0.0, 0.0]), np.array([0.0, 0.0]), g.nfft)
    rng = np.random.default_rng(5)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    mp = m @ g.S().T
    v = np.zeros(g.nfft)
    v[:g.nt_str] = mp[0].sum(0)                    # theta = 0 -> weight 1 on theta_0
    dp = _band_project(v, g.nfft)[:g.nt_str]
    want = g.U() @ dp
    got = gfst.forward(m, g)
    np.testing.assert_allclose(got[0], want, atol=1e-12 * np.abs(want).max())
    np.testing.assert_allclose(got[1], want, atol=1e-12 * np.abs(want).max())


def test_integer_shift_is_pure_circular_shift():
    """If every q_l h_n^2/dt' is an integer, L is a circular sample shift (minus the Nyquist part)."""
    nt, dt = 40, 0.01
    nts = 2 * nt
    T = (nt - 1) * dt
    dts = T * T / (nts - 1)
    h2 = np.array([1.0, 2.0, 3.0])
    ax = wl.Axes(nt=nt, dt=dt, ntau=nt, dtau=dt, nq=4, q_min=2 * dts, q_max=5 * dts, ntheta=2)
    ang = np.array([0.1, 0.7, 2.0])
    g = Geometry.build(ax, np.sqrt(h2) * np.cos(ang), np.sqrt(h2) * np.sin(ang))
    rng = np.random.default_rng(3)
    mp = rng.standard_normal((g.ntheta, g.nq, g.nt_str))
    got = gfst.inverse_spectrum(gfst.gfst_map(gfst.spectrum(mp, g), g), g)
    W = g.W()
    for n in range(3):
        acc = np.zeros(g.nfft)
        for j in range(g.ntheta):
            for l, ql in enumerate(g.q):
                sh = int(round(ql * h2[n] / dts))
                assert abs(ql * h2[n] / dts - sh) < 1e-9
                v = np.zeros(g.nfft)
                v[:g.nt_str] = mp[j, l]
                acc += W[n, j] * np.roll(v, sh)
        np.testing.assert_allclose(got[n], _band_project(acc, g.nfft)[:g.nt_str], atol=1e-11)


@pytest.mark.parametrize('k', [1, 3])
def test_rotation_by_grid_step_rolls_azimuth(k):
    """Rotating all offsets by k*dtheta equals rolling the model's azimuth axis by -k."""
    w, g = _tiny(4, ntheta=6)
    a = k * np.pi / g.ntheta
    xr = g.x * np.cos(a) - g.y * np.sin(a)
    yr = g.x * np.sin(a) + g.y * np.cos(a)
    gr = Geometry(g.nt, g.dt, g.ntau, g.dtau, g.nq, g.q_min, g.q_max, g.ntheta, g.stretch, xr, yr, g.nfft)
    rng = np.random.default_rng(9)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    np.testing.assert_allclose(gfst.forward(m, gr), gfst.forward(np.roll(m, -k, axis=0), g), atol=1e-10)


def test_single_azimuth_is_rotation_invariant():
    """ntheta = 1: the operator is the isotropic parabolic/hyperbolic Radon transform in h^2 only."""
    w, g = _tiny(5, ntheta=1)
    ang = np.random.default_rng(1).uniform(0, 2 * np.pi, g.x.size)
    h = np.sqrt(g.h2)
    g2 = Geometry(g.nt, g.dt, g.ntau, g.dtau, g.nq, g.q_min, g.q_max, 1, g.stretch,
                  h * np.cos(ang), h * np.sin(ang), g.nfft)
    m = np.random.default_rng(2).standard_normal((1, g.nq, g.ntau))
    np.testing.assert_allclose(gfst.forward(m, g), gfst.forward(m, g2), atol=1e-11)


def test_brute_force_matrix_transpose_and_norm():
    """Dense L from unit vectors: the adjoint is its transpose; the power iteration finds sigma_max^2."""
    w, g = _tiny(6, nt=16, ntr=4, nq=3, ntheta=2)
    nm = g.ntheta * g.nq * g.ntau
    nd = g.x.size * g.nt
    L = np.zeros((nd, nm))
    for i in range(nm):
        e = np.zeros(nm)
        e[i] = 1.0
        L[:, i] = gfst.forward(e.reshape(g.ntheta, g.nq, g.ntau), g).ravel()
    Lt = np.zeros((nm, nd))
    for i in range(nd):
        e = np.zeros(nd)
        e[i] = 1.0
        Lt[:, i] = gfst.adjoint(e.reshape(g.x.size, g.nt), g).ravel()
    np.testing.assert_allclose(Lt, L.T, atol=1e-13)
    smax = np.linalg.svd(L, compute_uv=False)[0]
    est = fista.power_norm2(lambda v: L @ v, lambda v: L.T @ v,
                            np.random.default_rng(0).standard_normal(nm), n_iter=500)
    assert abs(est - smax ** 2) / smax ** 2 < 1e-6


def test_sampled_outputs_match_full():
    w, g = _tiny(7, ntr=9)
    rng = np.random.default_rng(1)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    d = rng.standard_normal((g.x.size, g.nt))
    full = gfst.forward(m, g)
    np.testing.assert_allclose(gfst.forward_traces(m, g, [2, 5]), full[[2, 5]], atol=1e-13)
    fa = gfst.adjoint(d, g)
    rows = [(0, 1), (2, 4)]
    np.testing.assert_allclose(gfst.adjoint(d, g, rows=rows), fa[[0, 2], [1, 4]], atol=1e-13)


# ------------------------------------------------------------------ oracle-2
@pytest.mark.parametrize('seed', [0, 1])
def test_dot_test_timedomain(seed):
    w, g = _tiny(seed, ntheta=3)
    rng = np.random.default_rng(seed + 50)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    d = rng.standard_normal((g.x.size, g.nt))
    assert _dot_test(lambda v: timedomain.forward(v, g), lambda v: timedomain.adjoint(v, g), m, d) < 1e-12


def test_spike_maps_to_two_taps_on_the_hyperbola():
    """A model spike lands on t = sqrt(tau0^2 + q0 h^2) with linear weights (hand-derived)."""
    dt = 0.004
    # tau0 = 0.4 s (i0 = 100); target t = 0.501 s = (125 + 0.25) dt  =>  q0 h^2 = 0.501^2 - 0.16
    q0 = 0.25
    h2 = (0.501 ** 2 - 0.16) / q0
    ax = wl.Axes(nt=256, dt=dt, ntau=256, dtau=dt, nq=2, q_min=q0, q_max=q0 + 0.1, ntheta=4)
    g = Geometry.build(ax, np.array([math.sqrt(h2)]), np.array([0.0]))
    m = np.zeros((4, 2, 256))
    m[0, 0, 100] = 1.0
    d = timedomain.forward(m, g)[0]
    nz = np.nonzero(np.abs(d) > 1e-12)[0]
    assert list(nz) == [125, 126]
    np.testing.assert_allclose(d[125:127], [0.75, 0.25], atol=1e-9)


def test_elliptic_event_is_reproduced_per_azimuth():
    """Spikes at q_j = n_j^T W n_j reproduce t^2 = tau0^2 + h^T W h on traces at azimuth theta_j."""
    c, s = math.cos(0.4), math.sin(0.4)
    Rm = np.array([[c, -s], [s, c]])
    W = Rm @ np.diag([0.3 ** 2, 0.6 ** 2]) @ Rm.T
    tau0, dt, nth = 0.5, 0.002, 8
    for j in range(nth):
        th = j * math.pi / nth
        nv = np.array([math.cos(th), math.sin(th)])
        qj = float(nv @ W @ nv)
        ax = wl.Axes(nt=1024, dt=dt, ntau=1024, dtau=dt, nq=2, q_min=qj, q_max=qj + 0.05, ntheta=nth)
        hs = np.array([0.5, 1.3, 2.2])
        g = Geometry.build(ax, hs * nv[0], hs * nv[1])
        m = np.zeros((nth, 2, 1024))
        m[j, 0, int(round(tau0 / dt))] = 1.0
        d = timedomain.forward(m, g)
        for n, h in enumerate(hs):
            hv = h * nv
            t_ev = math.sqrt(tau0 ** 2 + hv @ W @ hv)
            centroid = np.sum(np.arange(1024) * d[n]) / np.sum(d[n])
            assert abs(centroid * dt - t_ev) < 1e-9
            assert abs(np.sum(d[n]) - 1.0) < 1e-12


def test_oracles_agree_on_smooth_models():
    """Oracle-1 vs oracle-2 (parity unpinned; the paper compares them only in a figure).

    The stretched operator of Section 3.1 carries no Jacobian, while the direct
    Riemann sum of the delta along t = sqrt(tau^2 + q h^2) gathers dtau/dt = t/tau
    more energy per data sample.  So the two agree in shape and arrival time,
    and their peak amplitudes differ by about t/tau.
    """
    w = wl.small_case(nt=128, ntr=20, nq=6, ntheta=4, seed=3, dt=0.004)
    g = Geometry.build(w.axes, w.gathers[0].x, w.gathers[0].y)
    tau = np.arange(g.ntau) * g.dtau
    m = np.zeros((g.ntheta, g.nq, g.ntau))
    m[1, 3] = np.exp(-((tau - 0.25) / 0.02) ** 2)
    a = gfst.forward(m, g)
    b = timedomain.forward(m, g)
    seen = 0
    for n in range(g.x.size):
        if np.abs(b[n]).max() < 1e-6:
            continue
        seen += 1
        cc = np.sum(a[n] * b[n]) / np.linalg.norm(a[n]) / np.linalg.norm(b[n])
        assert cc > 0.99
        assert abs(int(np.argmax(a[n])) - int(np.argmax(b[n]))) <= 1
        jac = np.sqrt(0.25 ** 2 + g.q[3] * g.h2[n]) / 0.25
        ratio = np.abs(b[n]).max() / np.abs(a[n]).max()
        assert abs(ratio / jac - 1) < 0.1
    assert seen >= 5


# ------------------------------------------------------------------ oracle-3
def test_fista_betas_golden():
    g = json.load(open(os.path.join(GOLDEN, 'fista_betas.json')))
    np.testing.assert_allclose(fista.fista_betas(4), g['betas'], atol=1e-9)


def test_soft_threshold_matches_paper_form():
    """sign(x) max(|x|-t, 0) equals the paper's x max(1 - t/|x|, 0) for x != 0, and 0 at 0."""
    x = np.array([-3.0, -0.5, 0.0, 0.2, 1.0, 4.0])
    t = 0.7
    paper = np.where(x != 0, x * np.maximum(1 - t / np.where(x != 0, np.abs(x), 1), 0), 0)
    np.testing.assert_allclose(fista.soft(x, t), paper, atol=1e-15)


def _dense_problem(seed=0, nd=60, nm=40):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((nd, nm))
    xt = np.zeros(nm)
    xt[rng.choice(nm, 6, replace=False)] = rng.standard_normal(6) * 3
    b = A @ xt + 0.05 * rng.standard_normal(nd)
    return A, b


def test_fista_matches_coordinate_descent_lasso():
    """Converged FISTA equals scikit-learn's coordinate-descent Lasso (alpha = lambda/n_samples)."""
    from sklearn.linear_model import Lasso
    A, b = _dense_problem()
    lam = 2.0
    norm2 = np.linalg.norm(A, 2) ** 2
    m = fista.solve(lambda v: A @ v, lambda v: A.T @ v, b, lam, 1.0 / norm2, 3000)
    ref = Lasso(alpha=lam / A.shape[0], fit_intercept=False, tol=1e-12, max_iter=200000).fit(A, b).coef_
    np.testing.assert_allclose(m, ref, atol=1e-6)
    assert fista.kkt_residual(lambda v: A @ v, lambda v: A.T @ v, b, m, lam) < 1e-6


def test_fista_zero_above_lambda_max_and_first_iterate():
    A, b = _dense_problem(1)
    L, Lt = (lambda v: A @ v), (lambda v: A.T @ v)
    gam = 1.0 / np.linalg.norm(A, 2) ** 2
    lmax = np.max(np.abs(A.T @ b))
    assert np.all(fista.solve(L, Lt, b, lmax * 1.0001, gam, 25) == 0)
    lam = 0.3 * lmax
    m1 = fista.solve(L, Lt, b, lam, gam, 1)
    np.testing.assert_allclose(m1, fista.soft(gam * (A.T @ b), gam * lam), atol=1e-14)


def test_ista_objective_monotone():
    A, b = _dense_problem(2)
    L, Lt = (lambda v: A @ v), (lambda v: A.T @ v)
    gam = 1.0 / np.linalg.norm(A, 2) ** 2
    lam = 0.1 * np.max(np.abs(A.T @ b))
    prev = np.inf
    hist = {k: None for k in range(1, 41)}
    fista.solve(L, Lt, b, lam, gam, 40, momentum=False, history=hist)
    for k in range(1, 41):
        o = fista.objective(L, b, hist[k], lam)
        assert o <= prev + 1e-12
        prev = o


def test_fista_on_gfst_kkt_decreases():
    """Sparse AAHRT on a tiny gather: the KKT residual shrinks with the iteration count."""
    w, g = _tiny(8, nt=24, ntr=6, nq=4, ntheta=3)
    L = lambda v: gfst.forward(v, g)
    Lt = lambda v: gfst.adjoint(v, g)
    rng = np.random.default_rng(4)
    d = rng.standard_normal((g.x.size, g.nt))
    n2 = fista.power_norm2(L, Lt, rng.standard_normal((g.ntheta, g.nq, g.ntau)), 60)
    gam = fista.step_from_norm2(n2)
    lam = fista.lambda_rule(Lt, d)
    k10 = fista.kkt_residual(L, Lt, d, fista.solve(L, Lt, d, lam, gam, 10), lam)
    k300 = fista.kkt_residual(L, Lt, d, fista.solve(L, Lt, d, lam, gam, 300), lam)
    assert k300 < 0.2 * k10


# ------------------------------------------------------------------ velocity estimate (Section 3)
def test_velocity_single_spike_gives_its_curvature():
    from oracle import velocity
    q = np.linspace(0.04, 0.49, 10)
    m = np.zeros((3, 10, 5))
    m[1, 7, 2] = -2.5                          # sign does not matter (weights |M|)
    qbar, v = velocity.velocity(m, q)
    assert qbar[1, 2] == q[7] and abs(v[1, 2] - q[7] ** -0.5) < 1e-15
    assert np.all(qbar[0] == 0) and np.all(v[0] == 0)   # no energy -> 0


def test_velocity_two_spikes_weighted_mean_and_scale_invariance():
    from oracle import velocity
    q = np.array([0.1, 0.2, 0.3, 0.4])
    m = np.zeros((4, 1))
    m[0, 0], m[3, 0] = 1.0, 3.0
    qbar = velocity.curvature_mean(m, q)
    assert abs(qbar[0] - (0.1 * 1 + 0.4 * 3) / 4) < 1e-15
    assert abs(velocity.curvature_mean(7.0 * m, q)[0] - qbar[0]) < 1e-15


def test_velocity_of_isotropic_event_cube_recovers_slowness():
    """A cube whose energy sits symmetrically about q0 (a line smeared over neighbouring q
    samples) gives v^-2 = q0 exactly."""
    from oracle import velocity
    q = 0.04 + 0.01 * np.arange(21)
    m = np.zeros((21, 3))
    for k, a in zip((-2, -1, 0, 1, 2), (0.1, 0.5, 1.0, 0.5, 0.1)):
        m[10 + k, :] = a
    qbar, v = velocity.velocity(m, q)
    assert np.allclose(qbar, q[10], rtol=0, atol=1e-15)
    assert np.allclose(v, q[10] ** -0.5, rtol=1e-14)


# ------------------------------------------------------------------ deconvolutive AAHRT (Section 4)
def test_deconv_convolution_matches_numpy_full_convolution():
    """W d equals numpy's full linear convolution cut to the trace's samples at origin c."""
    from oracle import deconv
    rng = np.random.default_rng(5)
    d = rng.standard_normal((3, 40))
    for nw, c in ((1, 0), (7, 3), (9, 0), (9, 8), (60, 20)):
        w = rng.standard_normal(nw)
        full = np.stack([np.convolve(row, w) for row in d])      # index s + c of full = output s
        ref = full[:, c:c + d.shape[1]]
        assert np.allclose(deconv.convolve(d, w, c), ref, rtol=0, atol=1e-13)


def test_deconv_delta_wavelet_is_identity_and_shift_is_shift():
    from oracle import deconv
    d = np.random.default_rng(6).standard_normal((2, 30))
    assert np.array_equal(deconv.convolve(d, [1.0], 0), d)
    out = deconv.convolve(d, [0.0, 0.0, 1.0], 0)                   # delay by 2 samples
    assert np.array_equal(out[:, 2:], d[:, :-2]) and np.all(out[:, :2] == 0)


def test_deconv_correlation_is_the_transpose_and_operator_dot_test():
    from oracle import deconv
    rng = np.random.default_rng(7)
    w, c = rng.standard_normal(11), 4
    a, b = rng.standard_normal((4, 50)), rng.standard_normal((4, 50))
    assert abs(np.sum(deconv.convolve(a, w, c) * b) - np.sum(a * deconv.correlate(b, w, c))) < 1e-11
    wk = wl.small_case(nt=32, ntr=6, nq=5, ntheta=3, seed=8)
    g = Geometry.build(wk.axes, wk.gathers[0].x, wk.gathers[0].y)
    m = rng.standard_normal((3, 5, 32))
    d = rng.standard_normal((6, 32))
    lhs = np.sum(deconv.forward(m, g, w, c) * d)
    rhs = np.sum(m * deconv.adjoint(d, g, w, c))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


# ------------------------------------------------------------------ Algorithm 2 (Section 3.2)
def _grid_gather(n=9, step=0.05, shuffle_seed=None):
    g1 = (np.arange(n) - (n - 1) / 2.0) * step
    X, Y = np.meshgrid(g1, g1, indexing='ij')
    x, y = X.ravel(), Y.ravel()
    if shuffle_seed is not None:
        p = np.random.default_rng(shuffle_seed).permutation(x.size)
        x, y = x[p], y[p]
    return x, y


def test_alg2_regular_grid_recovers_the_grid_and_rejects_others():
    from oracle import alg2
    x, y = _grid_gather(7, 0.04, shuffle_seed=1)
    x0, dx, mx, y0, dy, my, node = alg2.regular_grid(x, y)
    assert (mx, my) == (7, 7) and abs(dx - 0.04) < 1e-12 and abs(x0 + 0.12) < 1e-12 and abs(y0 + 0.12) < 1e-12
    assert np.allclose(x0 + dx * node[:, 0], x) and np.allclose(y0 + dy * node[:, 1], y)
    with pytest.raises(ValueError):
        alg2.regular_grid(x[1:], y[1:])                     # one node missing
    with pytest.raises(ValueError):
        alg2.regular_grid(x * (1 + 0.1 * (x > 0)), y)      # uneven spacing


def test_alg2_bilinear_reproduces_bilinear_functions():
    """B1..B4 of Section 3.4 interpolate a + b x + c y + e x y exactly, return the node
    values at nodes, and 0 outside the grid."""
    from oracle import alg2
    grid = (-0.375, 0.125, 7, -0.25, 0.0625, 9)            # binary-exact nodes
    xs = grid[0] + grid[1] * np.arange(7)
    ys = grid[3] + grid[4] * np.arange(9)
    f = lambda x, y: 1.5 - 2.0 * x + 0.7 * y + 3.0 * x * y
    dh = f(xs[:, None], ys[None, :])[:, :, None].astype(np.complex128) * (1 - 2j)
    rng = np.random.default_rng(2)
    for _ in range(50):
        px, py = rng.uniform(xs[0], xs[-1]), rng.uniform(ys[0], ys[-1])
        assert abs(alg2.bilinear(dh, grid, px, py)[0] - f(px, py) * (1 - 2j)) < 1e-12
    assert abs(alg2.bilinear(dh, grid, xs[3], ys[4])[0] - dh[3, 4, 0]) < 1e-13
    assert abs(alg2.bilinear(dh, grid, xs[-1], ys[-1])[0] - dh[-1, -1, 0]) < 1e-12   # last grid line
    assert alg2.bilinear(dh, grid, xs[-1] + 1e-6, 0.0)[0] == 0
    assert alg2.bilinear(dh, grid, 0.0, ys[0] - 1e-6)[0] == 0


def test_alg2_stretch_steps_are_exact_on_linear_signals():
    """Step 1 is exact on data linear in t, step 5 on a model linear in tau'."""
    from oracle import alg2
    w, g = _tiny(nt=40, ntr=3, nq=4, ntheta=2, dt=0.01)
    t = np.arange(g.nt) * g.dt
    d = np.stack([0.3 + 2.0 * t, -1.0 + 0.5 * t, np.ones_like(t)])
    dp = alg2.stretch_data(d, g)
    tr = np.sqrt(np.arange(g.nt_str) * g.dt_str)
    ok = tr <= t[-1]
    assert np.allclose(dp[0, ok], 0.3 + 2.0 * tr[ok], atol=1e-12)
    assert np.allclose(dp[2, ok], 1.0, atol=1e-12)
    tp = np.arange(g.nt_str) * g.dt_str
    mp = np.stack([0.2 - 1.5 * tp, 4.0 + 0 * tp])
    m = alg2.unstretch_model(mp, g)
    tau = np.arange(g.ntau) * g.dtau
    ok = tau ** 2 <= tp[-1]
    assert np.allclose(m[0, ok], 0.2 - 1.5 * tau[ok] ** 2, atol=1e-12)
    assert np.allclose(m[1, ok], 4.0, atol=1e-12)


def test_alg2_inverse_2d_matches_numpy_ffts():
    """Step 4 against numpy's inverse FFT over k (with the q_min shift) and an explicit
    cosine/sine sum over f'."""
    from oracle import alg2
    w, g = _tiny(nt=24, ntr=3, nq=6, ntheta=2, dt=0.02, q_min=-0.1, q_max=0.4)
    rng = np.random.default_rng(3)
    mh = rng.standard_normal((2, 6, g.nf)) + 1j * rng.standard_normal((2, 6, g.nf))
    k = alg2.k_axis(g)
    assert np.allclose(np.sort(k * 6 * (g.q[1] - g.q[0])), np.arange(-3, 3))
    G = np.fft.ifft(mh * np.exp(2j * np.pi * k * g.q_min)[None, :, None], axis=1)
    r = np.arange(g.nt_str)
    f = np.arange(1, g.nf)
    ph = 2 * np.pi * np.outer(f, r) / g.nfft
    ref = (G[..., :1].real + 2 * (np.einsum('jlf,fr->jlr', G[..., 1:].real, np.cos(ph))
                                   - np.einsum('jlf,fr->jlr', G[..., 1:].imag, np.sin(ph)))) / g.nfft
    assert np.allclose(alg2.inverse_2d(mh, g), ref, atol=1e-12)


@pytest.mark.parametrize('Wq', [np.diag([0.25, 0.25]), np.diag([0.16, 0.36])])
def test_alg2_focuses_an_event_at_its_curvature_per_azimuth(Wq):
    """Physics pin: an event t^2 = tau0^2 + h^T W h on a dense regular grid stacks, at every
    azimuth theta, at tau0 and at q(theta) = (cos, sin) W (cos, sin)^T within one q-sample."""
    from oracle import alg2
    ax = wl.Axes(nt=200, dt=0.004, ntau=200, dtau=0.004, nq=32, q_min=0.04, q_max=0.49, ntheta=6)
    x, y = _grid_gather(21, 0.05)
    g = Geometry.build(ax, x, y)
    d = wl.synth_data(ax, x, y, [dict(tau0=0.4, W=Wq, amp=1.0, f0=30.0)], None, None)
    M = alg2.adjoint(d, g)
    dq = g.q[1] - g.q[0]
    for j in range(ax.ntheta):
        th = np.pi * j / ax.ntheta
        c = np.array([np.cos(th), np.sin(th)])
        l, i = np.unravel_index(np.argmax(np.abs(M[j])), M[j].shape)
        assert abs(i * ax.dtau - 0.4) <= ax.dtau
        assert abs(g.q[l] - c @ Wq @ c) <= dq


# ------------------------------------------------------------------ the paper's step 3 (Section 3.4)
def _node_geometry(mg, nfft=240):
    """Tiny axes and traces whose k = f' h^2 falls on a node of the mg-point k grid for every
    frequency (h^2 = c N dt'/(dq mg), c integer) at azimuths on grid lines (0 and pi/2)."""
    ax = wl.Axes(nt=32, dt=0.02, ntau=32, dtau=0.02, nq=8, q_min=0.05, q_max=0.4, ntheta=4)
    T = (ax.nt - 1) * ax.dt
    dts = T * T / (2 * ax.nt - 1)
    unit = nfft * dts / (ax.dq * mg)
    c = np.array([0, 1, 2, 3, 5, 8])
    h = np.sqrt(c * unit)
    x = np.concatenate([h, np.zeros(c.size - 1)])
    y = np.concatenate([np.zeros(c.size), h[1:]])
    return ax, Geometry.build(ax, x, y, nfft=nfft)


@pytest.mark.parametrize('mg', [16, 24, 40])
def test_lineark_is_exact_on_the_k_grid_nodes(mg):
    """Where every k = f'h^2 is a node k_i of the grid and theta a grid azimuth, the A1..A4
    interpolation reads node values only, so it equals the exact sum over q (oracle-1)."""
    from oracle import lineark
    ax, g = _node_geometry(mg)
    rng = np.random.default_rng(mg)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    np.testing.assert_allclose(lineark.forward(m, g, mg), gfst.forward(m, g), atol=1e-11, rtol=0)
    d = rng.standard_normal((g.x.size, g.nt))
    np.testing.assert_allclose(lineark.adjoint(d, g, mg), gfst.adjoint(d, g), atol=1e-11, rtol=0)


def test_lineark_is_linear_in_k_between_nodes():
    """Between two nodes the interpolated spectrum, with the centring phase exp(-2 pi i f' q_c h^2)
    removed, is the straight line between the exact centred values at the nodes (Section 3.4,
    A1..A4 with theta on a grid line); node values from oracle-1's exact sum."""
    from oracle import lineark
    mg = 20
    ax, g0 = _node_geometry(mg)
    rng = np.random.default_rng(3)
    mh = rng.standard_normal((g0.ntheta, g0.nq, g0.nf)) + 1j * rng.standard_normal((g0.ntheta, g0.nq, g0.nf))
    qc = lineark.q_centre(g0)
    for f in (1, 7, 33, 119):
        fp = f / (g0.nfft * g0.dt_str)
        for u in (0.25, 3.6, 11.93):                # k/dk of the trace (not a node)
            i = math.floor(u)
            a = u - i
            h2 = np.array([u, i, i + 1]) / (fp * ax.dq * mg)
            gg = g0.subset([0, 0, 0])
            gg.x = np.sqrt(h2)
            gg.y = np.zeros(3)
            lin = lineark.linear_map(mh, gg, mg)[:, f]
            ex = gfst.gfst_map(mh, gg)[:, f] * np.exp(2j * np.pi * fp * qc * h2)   # centred exact values
            want = (1 - a) * ex[1] + a * ex[2]
            got = lin[0] * np.exp(2j * np.pi * fp * qc * h2[0])
            assert abs(got - want) < 1e-10 * max(1.0, abs(want)), (f, u)


def test_lineark_error_falls_with_the_k_grid_step():
    """Against the exact sum over q the linear interpolation is second order in dk = 1/(mg dq):
    doubling mg cuts the error by about four (config-1 axes, random model)."""
    from oracle import lineark
    w = wl.config1(with_data=False)
    g = Geometry.build(w.axes, w.gathers[0].x[::5], w.gathers[0].y[::5])
    m = np.random.default_rng(5).standard_normal((g.ntheta, g.nq, g.ntau))
    ref = gfst.forward(m, g)
    errs = [np.linalg.norm(lineark.forward(m, g, mg) - ref) / np.linalg.norm(ref) for mg in (64, 128, 256)]
    assert errs[0] < 0.5
    assert 0.15 < errs[1] / errs[0] < 0.35 and 0.15 < errs[2] / errs[1] < 0.35, errs


@pytest.mark.parametrize('mg', [12, 30])
def test_lineark_dot_test(mg):
    from oracle import lineark
    w, g = _tiny(4, ntheta=5, nq=6)
    rng = np.random.default_rng(mg)
    m = rng.standard_normal((g.ntheta, g.nq, g.ntau))
    d = rng.standard_normal((g.x.size, g.nt))
    assert _dot_test(lambda v: lineark.forward(v, g, mg), lambda v: lineark.adjoint(v, g, mg), m, d) < 1e-12
