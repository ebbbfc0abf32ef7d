"""Shared helpers of the GPU tests: build plans from seeded workloads and compare with the oracle."""
from __future__ import annotations

import functools

import numpy as np

import workloads as wl
from oracle import gfst, fista
from oracle.geometry import Geometry

# Relative L2 error bound of an FP32 result against the FP64 oracle: 1e-4, the bound the method
# is held to.  The operators themselves sit near 1e-6: the nonuniform FFT runs at nufft_tol = 1e-6
# (at sigma = 2, width 7 for nq = 64 and width 8 for nq = 32, estimated 9.6e-7 and 5.5e-7 with
# FP32 rounding), and FP32 DFTs of length <= 12000 add a few 1e-7.
TOL = 1e-4


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def geoms(w: wl.Workload):
    """Oracle geometry of every gather, with the batch-wide FFT length rule."""
    h2max = max([float(np.max(g.x ** 2 + g.y ** 2)) for g in w.gathers if g.x.size] + [0.0])
    out = []
    for g in w.gathers:
        out.append(Geometry.build(w.axes, g.x, g.y, h2max=h2max))
    nf = {g.nfft for g in out}
    assert len(nf) == 1
    return out


def make_plan(w: wl.Workload, **kw):
    from paper_2505_00387_amd import plan_from_workload
    return plan_from_workload(w, device=0, **kw)


def to_dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device='cuda:0')


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def split_data(d, trace_ptr):
    return [d[trace_ptr[b]:trace_ptr[b + 1]] for b in range(len(trace_ptr) - 1)]


def oracle_solver_params(geom: Geometry, d: np.ndarray, seed: int = 0):
    """lambda = 0.05 max|L^T d| and gamma = 1/(1.05 ||L||^2) from 30 power iterations (oracle, FP64)."""
    L = lambda v: gfst.forward(v, geom)
    Lt = lambda v: gfst.adjoint(v, geom)
    rng = np.random.default_rng(seed)
    n2 = fista.power_norm2(L, Lt, rng.standard_normal((geom.ntheta, geom.nq, geom.ntau)), 30)
    return fista.lambda_rule(Lt, d), fista.step_from_norm2(n2), n2


# ------------------------------------------------------------------ oracle work in worker processes
# The oracle's work for independent gathers runs in a pool of fresh interpreters (spawned, so they
# hold no GPU state), one BLAS thread each, so that the GPU tests' host time stays bounded.
def _one_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def oracle_pool(fn, cases, workers: int = 8):
    """[fn(*case) for case in cases], computed in up to `workers` spawned processes."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    cases = list(cases)
    if len(cases) <= 1:
        return [fn(*c) for c in cases]
    ctx = mp.get_context('spawn')
    with ProcessPoolExecutor(max_workers=min(workers, len(cases)), mp_context=ctx, initializer=_one_thread) as ex:
        return list(ex.map(fn, *zip(*cases)))


def oracle_pair(geom: Geometry, m: np.ndarray, d: np.ndarray):
    """(L m, L^T d) of one gather by the oracle."""
    return gfst.forward(m, geom), gfst.adjoint(d, geom)


def oracle_fista_case(geom: Geometry, d: np.ndarray, n_iter: int, ista: bool, seed: int = 0):
    """Oracle lambda, gamma and the n_iter-th FISTA (or ISTA) iterate of one gather."""
    lam, gam, _ = oracle_solver_params(geom, d, seed)
    L = lambda v: gfst.forward(v, geom)
    Lt = lambda v: gfst.adjoint(v, geom)
    return lam, gam, fista.solve(L, Lt, d, lam, gam, n_iter, momentum=not ista)
