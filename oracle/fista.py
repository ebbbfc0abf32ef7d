"""Oracle-3: sparse AAHRT by forward-backward splitting (FP64).  Test infrastructure only.

Section 4: minimise 0.5 ||d - L m||^2 + lambda ||m||_1 by the iteration
m^{k+1} = S(m^k + gamma L^T (d - L m^k)) with the soft shrinkage S at
threshold gamma*lambda.  The shrinkage is written as sign(x) max(|x| - gamma
lambda, 0), which equals x max(1 - gamma lambda/|x|, 0) for x != 0 and gives
0 at x = 0.  FISTA adds the Beck-Teboulle momentum:

  y_1 = m_0 = 0, t_1 = 1
  m_k     = S(y_k + gamma L^T (d - L y_k))
  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
  y_{k+1} = m_k + ((t_k - 1)/t_{k+1}) (m_k - m_{k-1})

The step is gamma = 1/(1.05 ||L||^2), with ||L||^2 from 30 power iterations
on L^T L started at a given vector; lambda = 0.05 max |L^T d|.
"""
from __future__ import annotations

import numpy as np


def soft(x: np.ndarray, thr) -> np.ndarray:
    return np.sign(x) * np.maximum(np.abs(x) - thr, 0.0)


def fista_betas(n_iter: int) -> np.ndarray:
    """Momentum weights beta_k = (t_k - 1)/t_{k+1}, k = 1..n_iter."""
    t = 1.0
    out = np.zeros(n_iter)
    for k in range(n_iter):
        tn = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        out[k] = (t - 1.0) / tn
        t = tn
    return out


def solve(apply_L, apply_Lt, d, lam, gamma, n_iter, m0=None, momentum=True, history=None):
    """FISTA (momentum=True) or ISTA.  history: optional dict k -> copy of m_k is filled."""
    m_prev = np.zeros_like(apply_Lt(d)) if m0 is None else np.array(m0, dtype=np.float64)
    y = m_prev.copy()
    betas = fista_betas(n_iter)
    for k in range(n_iter):
        r = d - apply_L(y)
        m = soft(y + gamma * apply_Lt(r), gamma * lam)
        if momentum:
            y = m + betas[k] * (m - m_prev)
        else:
            y = m
        m_prev = m
        if history is not None and (k + 1) in history:
            history[k + 1] = m.copy()
    return m_prev


def objective(apply_L, d, m, lam) -> float:
    r = d - apply_L(m)
    return 0.5 * float(np.sum(r * r)) + lam * float(np.sum(np.abs(m)))


def power_norm2(apply_L, apply_Lt, v0, n_iter=30) -> float:
    """Estimate ||L||^2 = largest eigenvalue of L^T L from a start vector v0."""
    v = v0 / np.linalg.norm(v0)
    est = 0.0
    for _ in range(n_iter):
        w = apply_Lt(apply_L(v))
        est = float(np.linalg.norm(w))
        if est == 0.0:
            return 0.0
        v = w / est
    return est


def step_from_norm2(norm2: float) -> float:
    return 1.0 / (1.05 * norm2)


def lambda_rule(apply_Lt, d, frac=0.05) -> float:
    return frac * float(np.max(np.abs(apply_Lt(d))))


def kkt_residual(apply_L, apply_Lt, d, m, lam) -> float:
    """max over coordinates of the violation of 0 in L^T(Lm - d) + lam d|m|."""
    g = apply_Lt(d - apply_L(m))
    on = m != 0
    v_on = np.abs(g[on] - lam * np.sign(m[on]))
    v_off = np.maximum(np.abs(g[~on]) - lam, 0.0)
    return float(max(v_on.max(initial=0.0), v_off.max(initial=0.0)))
