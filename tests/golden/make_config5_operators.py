#!/usr/bin/env python3
"""Write FP64 oracle references of L and L^T on four gathers of the large workload.

The workload is 32 CMPs of 4096 traces in a 4 km disk, nt = 2048 at 1 ms, nq = 128,
ntheta = 36 (FFT length N = 12000 from the whole batch's offsets).  Four seeded gathers
b each carry their own seeded N(0,1) model ``workloads.random_model(axes, 1, 50 + b)``
and data ``workloads.random_data(4096, nt, 50 + b)``.  For each of them the oracle
(oracle-1, Algorithm 1 with the exact sum over q) gives six seeded traces of L m_b and
four seeded model rows (theta_j, q_l) of L^T d_b, stored in FP32 with their indices in
``config5_operators.npz``.  Nothing here comes from the HIP library.  Run from the
repository root (a few minutes):
    python tests/golden/make_config5_operators.py [--jobs 4]
"""
from __future__ import annotations

import argparse
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, 'config5_operators.npz')
NTRACE = 6
NROW = 4


def picks(batch: int):
    rng = np.random.default_rng(np.random.SeedSequence([2505_00387, 55]))
    return sorted(rng.choice(batch, 4, replace=False).tolist())


def one_gather(b: int):
    from threadpoolctl import threadpool_limits
    import workloads as wl
    from oracle import gfst
    from oracle.geometry import Geometry
    w = wl.config5(with_data=False)
    h2max = max(float(np.max(g.x ** 2 + g.y ** 2)) for g in w.gathers)
    g0 = w.gathers[b]
    rng = np.random.default_rng(np.random.SeedSequence([2505_00387, 56, b]))
    tr = np.sort(rng.choice(g0.x.size, NTRACE, replace=False)).astype(np.int64)
    rows = np.stack([rng.integers(w.axes.ntheta, size=NROW), rng.integers(w.axes.nq, size=NROW)],
                    axis=1).astype(np.int64)
    m = wl.random_model(w.axes, 1, 50 + b)[0]
    d = wl.random_data(g0.x.size, w.axes.nt, 50 + b)
    with threadpool_limits(2):
        g = Geometry.build(w.axes, g0.x, g0.y, h2max=h2max)
        fwd = gfst.forward_traces(m, g, tr)
        adj = gfst.adjoint(d, g, rows=[tuple(r) for r in rows])
    return b, g.nfft, tr, rows, fwd, adj


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--jobs', type=int, default=4)
    args = ap.parse_args()
    import workloads as wl
    w = wl.config5(with_data=False)
    bs = picks(w.batch)
    out = {'gathers': np.array(bs, dtype=np.int64)}
    fwd = np.zeros((4, NTRACE, w.axes.nt), dtype=np.float32)
    adj = np.zeros((4, NROW, w.axes.ntau), dtype=np.float32)
    tri = np.zeros((4, NTRACE), dtype=np.int64)
    rwi = np.zeros((4, NROW, 2), dtype=np.int64)
    nffts = set()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for i, (b, nfft, tr, rows, f, a) in enumerate(ex.map(one_gather, bs)):
            fwd[i], adj[i], tri[i], rwi[i] = f, a, tr, rows
            nffts.add(nfft)
            print(f'gather {b} done', flush=True)
    assert len(nffts) == 1
    np.savez_compressed(OUT, forward=fwd, adjoint=adj, trace_idx=tri, row_idx=rwi,
                        nfft=np.int64(nffts.pop()), **out)
    print('wrote', OUT, os.path.getsize(OUT), 'bytes')


if __name__ == '__main__':
    main()
