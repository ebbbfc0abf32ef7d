#!/usr/bin/env python3
"""Write FP64 oracle references of L and L^T on every gather of the 256-gather workload.

The workload is the uneven-fold batch (fold 200..1200 in a 3 km disk, nt = 1024 at 2 ms,
nq = 64, ntheta = 16, FFT length N = 4320 from the whole batch's offsets).  Inputs are
the seeded N(0,1) model cube and data of ``workloads.random_model(axes, 256, 21)`` and
``workloads.random_data(ntraces, nt, 21)``.  For every gather b the oracle (oracle-1,
Algorithm 1 with the exact sum over q) gives

* two seeded traces of L m_b (forward; each output trace depends on its own offset only),
* two seeded model rows (theta_j, q_l) of L^T d_b (adjoint),

stored in FP32 (relative rounding 6e-8) with their indices, in ``config4_operators.npz``.
Nothing here comes from the HIP library.  Run from the repository root (a few minutes on
8 cores):
    python tests/golden/make_config4_operators.py [--jobs 7]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, 'config4_operators.npz')
SEED = 21
NTRACE = 2
NROW = 2


def picks(b: int, fold: int, ntheta: int, nq: int):
    """Seeded trace indices (within the gather) and (theta, q) rows of gather b."""
    rng = np.random.default_rng(np.random.SeedSequence([2505_00387, 44, b]))
    tr = np.sort(rng.choice(fold, NTRACE, replace=False)).astype(np.int64)
    rows = np.stack([rng.integers(ntheta, size=NROW), rng.integers(nq, size=NROW)], axis=1).astype(np.int64)
    return tr, rows


def one_gather(args):
    b, m_b, d_b, x, y, axes, h2max = args
    from threadpoolctl import threadpool_limits
    from oracle import gfst
    from oracle.geometry import Geometry
    with threadpool_limits(1):
        g = Geometry.build(axes, x, y, h2max=h2max)
        tr, rows = picks(b, x.size, axes.ntheta, axes.nq)
        fwd = gfst.forward_traces(m_b, g, tr)
        adj = gfst.adjoint(d_b, g, rows=[tuple(r) for r in rows])
    return b, g.nfft, tr, rows, fwd, adj


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--jobs', type=int, default=max(1, (os.cpu_count() or 2) - 1))
    args = ap.parse_args()
    import workloads as wl
    w = wl.config4(with_data=False)
    tp = w.trace_ptr
    m = wl.random_model(w.axes, w.batch, SEED)
    d = wl.random_data(int(tp[-1]), w.axes.nt, SEED)
    sha_m = hashlib.sha256(m.tobytes()).hexdigest()
    sha_d = hashlib.sha256(d.tobytes()).hexdigest()
    h2max = max(float(np.max(g.x ** 2 + g.y ** 2)) for g in w.gathers)
    jobs = [(b, m[b], d[tp[b]:tp[b + 1]], w.gathers[b].x, w.gathers[b].y, w.axes, h2max) for b in range(w.batch)]
    fwd = np.zeros((w.batch, NTRACE, w.axes.nt), dtype=np.float32)
    adj = np.zeros((w.batch, NROW, w.axes.ntau), dtype=np.float32)
    tr_idx = np.zeros((w.batch, NTRACE), dtype=np.int64)
    row_idx = np.zeros((w.batch, NROW, 2), dtype=np.int64)
    nffts = set()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for b, nfft, tr, rows, f, a in ex.map(one_gather, jobs, chunksize=4):
            fwd[b], adj[b], tr_idx[b], row_idx[b] = f, a, tr, rows
            nffts.add(nfft)
            if b % 32 == 0:
                print(f'gather {b} done', flush=True)
    assert len(nffts) == 1
    np.savez_compressed(OUT, forward=fwd, adjoint=adj, trace_idx=tr_idx, row_idx=row_idx,
                        nfft=np.int64(nffts.pop()), seed=np.int64(SEED), model_sha=np.array(sha_m),
                        data_sha=np.array(sha_d))
    print('wrote', OUT, os.path.getsize(OUT), 'bytes')


if __name__ == '__main__':
    main()
