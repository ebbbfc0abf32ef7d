#!/usr/bin/env python3
"""Write the stored FP64 references of the 100-iteration sparse AAHRT (oracle only).

Section 4 casts the forward transform as argmin 0.5||d - L m||^2 + lambda ||m||_1 and
solves it by forward-backward splitting with soft shrinkage; oracle-3 adds the FISTA
momentum.  For every case below this script runs, in FP64 with the CPU oracle alone:

* lambda_b = 0.05 max|L_b^T d_b| and gamma_b = 1/(1.05 ||L_b||^2), the norm from 30 power
  iterations started at a seeded N(0,1) cube;
* 100 FISTA iterations from m = 0, keeping the iterates m_k at the k of ``KEEP``.

Iterates are sparse (soft shrinkage zeroes most of the cube), so each is stored as the
flat indices of its nonzero entries and their values rounded to FP32 (relative rounding
6e-8, far below the 1e-4 bound the library is held to).  Also stored: a SHA-256 of the
FP64 data the iterates were computed from, so that a test can tell a stale file from a
changed workload generator.

Cases (inputs from ``workloads``; nothing here comes from the HIP library):
* ``config1``  -- the single 256-trace CMP (nt = 256);
* ``config2``  -- the realistic 1024-trace CMP (nt = 1024, nq = 64, ntheta = 16);
* ``config4_bNNN`` -- eight gathers of the 256-gather uneven-fold batch: the smallest, the
  median and the largest fold and five seeded others, each with the batch-wide FFT length.

Run from the repository root (about 35 minutes on 8 cores):
    python tests/golden/make_fista100.py [--jobs 7] [--only config1,config2]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT_DIR = os.path.join(HERE, 'fista100')
KEEP = (1, 10, 50, 100)
N_ITER = 100
POWER_ITERS = 30


def data_sha(d: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(d, dtype=np.float64).tobytes()).hexdigest()


def config4_picks(w) -> list:
    """Smallest, median and largest fold, then five seeded others (sorted, distinct)."""
    folds = np.diff(w.trace_ptr)
    order = np.argsort(folds, kind='stable')
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    rng = np.random.default_rng(np.random.SeedSequence([2505_00387, 4, 100]))
    for b in rng.permutation(w.batch):
        if len(picks) == 8:
            break
        if int(b) not in picks:
            picks.append(int(b))
    return sorted(picks)


def cases() -> list:
    """(name, config, gather index) of every stored reference."""
    import workloads as wl
    out = [('config1', 1, 0), ('config2', 2, 0)]
    w4 = wl.config4(with_data=False)
    out += [(f'config4_b{b:03d}', 4, b) for b in config4_picks(w4)]
    return out


def geometry_of(config: int, b: int):
    import workloads as wl
    from oracle.geometry import Geometry
    w = wl.CONFIGS[config](with_data=False)
    h2max = max(float(np.max(g.x ** 2 + g.y ** 2)) for g in w.gathers if g.x.size)
    # the gathers of a batch draw from their own spawned generators, so the first b + 1
    # gathers with data give gather b exactly as the whole batch would
    wd = wl.config4(with_data=True, batch=b + 1) if config == 4 else wl.CONFIGS[config](with_data=True)
    g = wd.gathers[b]
    assert np.array_equal(g.x, w.gathers[b].x)
    return w, Geometry.build(w.axes, g.x, g.y, h2max=h2max), g.data


def run_case(name: str, config: int, b: int) -> str:
    from threadpoolctl import threadpool_limits
    from oracle import gfst, fista
    t0 = time.perf_counter()
    with threadpool_limits(1):
        w, geom, d = geometry_of(config, b)
        L = lambda v: gfst.forward(v, geom)
        Lt = lambda v: gfst.adjoint(v, geom)
        lam = fista.lambda_rule(Lt, d)
        rng = np.random.default_rng(np.random.SeedSequence([2505_00387, 100 + config, b]))
        v0 = rng.standard_normal((geom.ntheta, geom.nq, geom.ntau))
        norm2 = fista.power_norm2(L, Lt, v0, POWER_ITERS)
        gam = fista.step_from_norm2(norm2)
        hist = {k: None for k in KEEP}
        fista.solve(L, Lt, d, lam, gam, N_ITER, history=hist)
    rec = {'lam': np.float64(lam), 'gamma': np.float64(gam), 'norm2': np.float64(norm2),
           'config': np.int64(config), 'gather': np.int64(b), 'nfft': np.int64(geom.nfft),
           'shape': np.array([geom.ntheta, geom.nq, geom.ntau], dtype=np.int64),
           'keep': np.array(KEEP, dtype=np.int64), 'data_sha': np.array(data_sha(d)),
           'ntraces': np.int64(geom.x.size)}
    for k in KEEP:
        m = hist[k].ravel()
        idx = np.flatnonzero(m)
        rec[f'idx_{k}'] = idx.astype(np.int32)
        rec[f'val_{k}'] = m[idx].astype(np.float32)
        rec[f'norm_{k}'] = np.float64(np.linalg.norm(m))
    os.makedirs(OUT_DIR, exist_ok=True)
    path = os.path.join(OUT_DIR, f'{name}.npz')
    np.savez_compressed(path, **rec)
    nnz = {k: rec[f'idx_{k}'].size for k in KEEP}
    return f'{name}: {geom.x.size} traces, lambda {lam:.6e}, gamma {gam:.6e}, nnz {nnz}, ' \
           f'{time.perf_counter() - t0:.0f} s'


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--jobs', type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument('--only', default='', help='comma-separated case names')
    args = ap.parse_args()
    todo = cases()
    if args.only:
        want = set(args.only.split(','))
        todo = [c for c in todo if c[0] in want]
    # largest first, so the longest job starts at once
    import workloads as wl
    w4 = wl.config4(with_data=False)
    folds = np.diff(w4.trace_ptr)
    cost = {'config1': 1, 'config2': 1024}
    todo.sort(key=lambda c: -(cost.get(c[0]) or int(folds[c[2]])))
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        futs = [ex.submit(run_case, *c) for c in todo]
        for f in futs:
            print(f.result(), flush=True)


if __name__ == '__main__':
    main()
