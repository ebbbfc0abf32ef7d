#!/usr/bin/env python3
"""Benchmark of the batched sparse AAHRT on one MI355X.

A step is one 100-iteration FISTA solve of the whole batch: the lambda rule
(one L^T pass and a per-gather max) plus 100 iterations of {L, residual, L^T,
shrinkage + momentum}.  The workload is 256 CMP gathers of uneven fold (200 to
1200 traces in a 3 km disk), nt = 1024 at 2 ms, nq = 64, ntheta = 16, seeded
synthetic data (elliptical-moveout Ricker events plus noise).  The step length
gamma_b = 1/(1.05 ||L_b||^2) depends only on the geometry, so it is computed
once per plan (30 power iterations) and reported as setup, like the plan.

Prints one JSON line: metric, value (gathers/s), ms per step, the roofline of
the dominant kernel (algorithmic bytes per launch / its mean HIP-event time),
fwd+adj gather-pairs/s, per-kernel times, and the FP64 oracle timed on host
cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_bytes(plan, name: str) -> float:
    """Algorithmic HBM bytes of one launch of a kernel over the plan's batch."""
    a = plan.axes
    B, ntr, nf = plan.batch, plan.ntraces, plan.info['nfreq']
    rows = B * a.ntheta * a.nq
    return {
        'model_r2c': rows * (4 * a.ntau + 8 * nf),
        'nufft_interp': rows * 8 * nf + ntr * 8 * nf,
        'data_c2r': ntr * (8 * nf + 4 * a.nt),
        'data_r2c': ntr * (4 * a.nt + 8 * nf),
        'nufft_spread': ntr * 8 * nf + rows * 8 * nf,
        'model_c2r': rows * (8 * nf + 4 * a.ntau),
        'residual_r2c': ntr * (16 * nf + 4 * a.nt),
        'model_c2r_update': rows * (8 * nf + 16 * a.ntau),
        'model_update_r2c': rows * (16 * nf + 16 * a.ntau),
    }[name]


def source_hash() -> str:
    """Hash of the kernel sources with comments and blank space removed (comment edits keep it)."""
    import re
    h = hashlib.sha256()
    for f in ('gfst_sweep.hip', 'gfst_res.hip', 'gfst_common.hpp', 'es_poly.hpp', 'rows.hip', 'misc.hip',
              'kernel_common.hpp', 'fft_lds.hpp', 'aahrt_internal.hpp'):
        with open(os.path.join(ROOT, 'paper_2505_00387_amd', 'csrc', f)) as fh:
            text = fh.read()
        text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
        text = re.sub(r'//[^\n]*', '', text)
        h.update(''.join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, gfst: dict):
    """HBM bytes per launch from committed rocprofv3 counter runs, if taken on this kernel source
    (and, for the GFST kernels, on the same autotuned grid setting)."""
    path = os.path.join(ROOT, 'profiles', 'hbm_counters.json')
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get('source_hash') != source_hash() or rec.get('workload') != workload:
        return None
    if kernel.startswith('nufft_'):
        cfg = rec.get('gfst_config', {})
        if any(cfg.get(k) != gfst.get(k) for k in ('grid', 'kernel_width', 'freq_tile', 'freq_tile_adjoint',
                                                    'block_threads', 'block_threads_adjoint')):
            return None
    k = rec.get('kernels', {}).get(kernel)
    return None if k is None else k.get('bytes_per_launch')


def _oracle_iterations(axes, x, y, d, h2max, n_iter):
    """Worker: n_iter FISTA iterations (L, L^T and the shrinkage) of the FP64 oracle on one gather,
    one BLAS thread; returns the seconds per iteration."""
    from threadpoolctl import threadpool_limits
    from oracle import gfst, fista
    from oracle.geometry import Geometry
    with threadpool_limits(1):
        geom = Geometry.build(axes, x, y, h2max=h2max)
        L = lambda v: gfst.forward(v, geom)
        Lt = lambda v: gfst.adjoint(v, geom)
        t0 = time.perf_counter()
        fista.solve(L, Lt, d, 1.0, 1e-3, n_iter)
        return (time.perf_counter() - t0) / n_iter


def cpu_baseline(w, n_iter_sample: int = 2):
    """FP64 oracle on the host cores: one worker process per core (one BLAS thread each), each
    running n_iter_sample FISTA iterations on its own gather, the gathers spread evenly over the
    batch's sorted folds.  The batch's 100-iteration solve on those cores is extrapolated from the
    mean seconds per iteration (plus half an iteration for the lambda rule's L^T), assuming the
    gathers split evenly over the cores."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    folds = np.diff(w.trace_ptr)
    order = np.argsort(folds, kind='stable')
    picks = [int(order[int((i + 0.5) * len(order) / cores)]) for i in range(cores)]
    h2max = max(float(np.max(g.x ** 2 + g.y ** 2)) for g in w.gathers)
    args = [(w.axes, w.gathers[b].x, w.gathers[b].y, w.gathers[b].data, h2max, n_iter_sample) for b in picks]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context('spawn')) as ex:
        per_iter = list(ex.map(_oracle_iterations, *zip(*args)))
    wall = time.perf_counter() - t0
    t_gather = (w.n_iter + 0.5) * float(np.mean(per_iter))
    t_batch = w.batch * t_gather / cores
    return {'value': w.batch / t_batch, 'unit': 'gathers/s', 'cores': cores, 'kind': 'oracle',
            'sample': f'{cores} processes x 1 BLAS thread, each {n_iter_sample} FISTA iterations (L + L^T + '
                      f'shrinkage, FP64 NumPy) on one gather, gathers spread over the sorted folds '
                      f'({int(folds[picks].min())}-{int(folds[picks].max())} traces); mean '
                      f'{np.mean(per_iter):.2f} s per iteration per gather; extrapolated to {w.batch} gathers x '
                      f'{w.n_iter} iterations split over the {cores} cores; sample wall {wall:.1f} s',
            'extrapolated': True}


def cpu_baseline_pair(w):
    """FP64 oracle, one forward + adjoint pair on gather 0, one core."""
    import workloads as wl
    from oracle import gfst
    from oracle.geometry import Geometry
    from threadpoolctl import threadpool_limits
    g0 = w.gathers[0]
    geo = Geometry.build(w.axes, g0.x, g0.y)
    mo = wl.random_model(w.axes, 1, 0)[0]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        gfst.adjoint(gfst.forward(mo, geo), geo)
        t = time.perf_counter() - t0
    return {'pair_s': round(t, 2), 'pairs_per_s': round(1.0 / t, 4), 'cores': 1, 'kind': 'oracle',
            'sample': f'one L + L^T pair on gather 0 ({g0.x.size} traces), FP64 NumPy, 1 thread'}


class PlainOperator:
    """Plain per-gather FP32 operator on the GPU with torch ops, for the speed-up comparison.

    The same discrete L and L^T as the library (linear stretch, real FFT of length N,
    GFST map, inverse FFT, unstretch), but the map is the direct nonuniform DFT over
    q (phases reduced modulo 1 in FP64, exponentials and sums in FP32) and every
    gather is processed on its own.
    """

    def __init__(self, w, nfft, dev):
        import numpy as np
        import torch
        a = w.axes
        self.a, self.N, self.F, self.dev = a, nfft, nfft // 2, dev
        self.nts = a.stretch * a.nt
        T = (a.nt - 1) * a.dt
        self.dts = T * T / (self.nts - 1)
        S = np.zeros((self.nts, a.ntau))
        for r in range(self.nts):
            pos = np.sqrt(r * self.dts) / a.dtau
            i = int(np.floor(pos))
            f = pos - i
            if i < a.ntau:
                S[r, i] += 1 - f
            if i + 1 < a.ntau:
                S[r, i + 1] += f
        U = np.zeros((a.nt, self.nts))
        for t in range(a.nt):
            pos = (t * a.dt) ** 2 / self.dts
            i = int(np.floor(pos))
            f = pos - i
            if i < self.nts:
                U[t, i] += 1 - f
            if i + 1 < self.nts:
                U[t, i + 1] += f
        self.S = torch.tensor(S, dtype=torch.float32, device=dev)
        self.U = torch.tensor(U, dtype=torch.float32, device=dev)
        self.q = torch.tensor(a.q_min + a.dq * np.arange(a.nq), dtype=torch.float64, device=dev)
        self.f = torch.arange(self.F, dtype=torch.float64, device=dev) / (nfft * self.dts)

    def gather(self, g):
        import numpy as np
        import torch
        th = np.mod(np.arctan2(g.y, g.x), np.pi)
        u = th / (np.pi / self.a.ntheta)
        j = np.floor(u).astype(np.int64) % self.a.ntheta
        fr = u - np.floor(u)
        W = np.zeros((g.x.size, self.a.ntheta))
        W[np.arange(g.x.size), j] += 1 - fr
        W[np.arange(g.x.size), (j + 1) % self.a.ntheta] += fr
        h2 = torch.tensor(g.x ** 2 + g.y ** 2, dtype=torch.float64, device=self.dev)
        return torch.tensor(W, dtype=torch.complex64, device=self.dev), h2

    def _phase(self, h2, f0, f1):
        import torch
        ph = torch.frac(self.f[f0:f1, None, None] * h2[None, :, None] * self.q[None, None, :])
        return torch.exp((-2j * torch.pi) * ph.to(torch.float32))          # [fc, n, nq]

    def forward(self, m, W, h2, fc=64):
        import torch
        mh = torch.fft.rfft(m @ self.S.T, n=self.N)[..., :self.F]            # [ntheta, nq, F]
        dh = torch.empty((h2.numel(), self.F), dtype=torch.complex64, device=self.dev)
        for f0 in range(0, self.F, fc):
            f1 = min(f0 + fc, self.F)
            A = torch.einsum('nj,jlf->fnl', W, mh[:, :, f0:f1])
            dh[:, f0:f1] = torch.sum(A * self._phase(h2, f0, f1), dim=2).T
        pad = torch.zeros((h2.numel(), self.F + 1), dtype=torch.complex64, device=self.dev)
        pad[:, :self.F] = dh
        return torch.fft.irfft(pad, n=self.N)[:, :self.nts] @ self.U.T

    def adjoint(self, d, W, h2, fc=64):
        import torch
        c = torch.full((self.F,), 2.0 / self.N, device=self.dev)
        c[0] = 1.0 / self.N
        gh = torch.fft.rfft(d @ self.U, n=self.N)[:, :self.F] * c
        hh = torch.empty((self.a.ntheta, self.a.nq, self.F), dtype=torch.complex64, device=self.dev)
        for f0 in range(0, self.F, fc):
            f1 = min(f0 + fc, self.F)
            B = torch.conj(self._phase(h2, f0, f1)) * gh[:, f0:f1].T[:, :, None]
            hh[:, :, f0:f1] = torch.einsum('nj,fnl->jlf', torch.conj(W), B)
        pad = torch.zeros((self.a.ntheta, self.a.nq, self.N), dtype=torch.complex64, device=self.dev)
        pad[..., :self.F] = hh
        return (torch.fft.ifft(pad).real * self.N)[..., :self.nts] @ self.S


def plain_comparison(w, plan, lib_pair_s, n_sample, dev):
    """Time the plain per-gather operator pair on n_sample gathers and scale to the batch."""
    import torch
    op = PlainOperator(w, plan.info['nfft'], dev)
    gs = [op.gather(g) for g in w.gathers[:n_sample]]
    ms = [torch.randn((w.axes.ntheta, w.axes.nq, w.axes.ntau), device=dev) for _ in range(n_sample)]
    op.adjoint(op.forward(ms[0], *gs[0]), *gs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(n_sample):
        op.adjoint(op.forward(ms[b], *gs[b]), *gs[b])
    torch.cuda.synchronize()
    t_sample = time.perf_counter() - t0
    folds = [g.x.size for g in w.gathers]
    scale = sum(folds) / sum(folds[:n_sample])
    t_batch = t_sample * scale
    # the plain operator and the library compute the same L: compare on gather 0
    mb = torch.zeros(plan.model_shape, device=dev)
    mb[0] = ms[0]
    d_lib = plan.forward(mb)[: w.gathers[0].x.size]
    d_pl = op.forward(ms[0], *gs[0])
    diff = (torch.linalg.norm(d_lib - d_pl) / torch.linalg.norm(d_pl)).item()
    return {'plain_pair_s_batch': round(t_batch, 3), 'plain_sample_gathers': n_sample,
            'plain_pair_ms_per_gather': round(1e3 * t_sample / n_sample, 3),
            'speedup_vs_plain': round(t_batch / lib_pair_s, 1), 'plain_vs_library_rel_diff': diff}


# seconds printed in the paper's timing table (Section 5) for (nt, nx = ny, np): direct sum, proposed
TIMING_TABLE_SECONDS = {(512, 128, 128): (218, 0.87), (512, 128, 256): (421, 1.14), (512, 256, 128): (915, 3.80),
                (512, 256, 256): (1685, 3.98), (1024, 128, 128): (497, 1.97), (1024, 128, 256): (875, 2.78),
                (1024, 256, 128): (1806, 8.57), (1024, 256, 256): (3416, 8.82)}


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def table1_scan(reps: int):
    """Velocity scan (the adjoint, data -> (tau, q, theta)) at the shapes of the paper's timing
    table: the GFST adjoint of the library against the GPU time-domain direct sum, one CMP on a
    regular offset grid at 40 m, 90 azimuths.  One JSON line per shape."""
    import torch
    import workloads as wl
    from paper_2505_00387_amd import plan_from_workload
    dev = torch.device('cuda:0')
    for nt, nxy, np_ in wl.TABLE1_SHAPES:
        w = wl.table1(nt, nxy, np_)
        t0 = time.perf_counter()
        plan = plan_from_workload(w, device=0)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        d = torch.tensor(w.gathers[0].data, dtype=torch.float32, device=dev)
        m_g = torch.empty(plan.model_shape, dtype=torch.float32, device=dev)
        m_d = torch.empty(plan.model_shape, dtype=torch.float32, device=dev)
        t_gfst = _timed(lambda: plan.adjoint(d, m_g), reps)
        plan.profile(True)
        plan.adjoint(d, m_g)
        torch.cuda.synchronize()
        prof = {k: round(ms / n, 4) for k, (ms, n) in plan.profile_read().items() if n}
        plan.profile(False)
        t_direct = _timed(lambda: plan.adjoint_direct(d, m_d), max(1, reps // 5))
        m_a = torch.empty(plan.model_shape, dtype=torch.float32, device=dev)
        t_grid = _timed(lambda: plan.adjoint_grid(d, m_a), reps)
        # Algorithm 2 is not the transpose of L (its step 3 reads one offset per (f', k, theta),
        # without the Jacobian of the polar change of variables): compared by correlation
        corr = (torch.sum(m_a * m_g) / (torch.linalg.norm(m_a) * torch.linalg.norm(m_g))).item()
        diff = (torch.linalg.norm(m_g - m_d) / torch.linalg.norm(m_d)).item()
        # the t^2 stretch at twice nt samples undersamples the first few hundred ms (the
        # stretched spacing in t is dt'/2t), so the two discretisations part mostly there
        i0 = int(round(0.4 / w.axes.dtau))
        diff_late = (torch.linalg.norm(m_g[..., i0:] - m_d[..., i0:]) / torch.linalg.norm(m_d[..., i0:])).item()
        paper = TIMING_TABLE_SECONDS[(nt, nxy, np_)]
        out = {'metric': 'velocity scan seconds (adjoint, one CMP)', 'workload': w.name,
               'nt': nt, 'nx': nxy, 'ny': nxy, 'np': np_, 'ntheta': w.axes.ntheta, 'traces': plan.ntraces,
               'gfst_adjoint_s': round(t_gfst, 6), 'direct_adjoint_s': round(t_direct, 6),
               'speedup_direct_over_gfst': round(t_direct / t_gfst, 1),
               'algorithm2_adjoint_s': round(t_grid, 6), 'algorithm2_corr_with_gfst_adjoint': round(corr, 4),
               'gfst_vs_direct_rel_diff': round(diff, 4), 'gfst_vs_direct_rel_diff_tau_ge_0.4s': round(diff_late, 4),
               'paper_direct_s': paper[0], 'paper_proposed_s': paper[1],
               'paper_speedup': round(paper[0] / paper[1], 1),
               'gfst_adjoint_kernel_ms': prof,
               'plan_s': round(t_plan, 3), 'nfft': plan.info['nfft'], 'grid': plan.info['grid_size'],
               'kernel_width': plan.info['kernel_width'], 'dtype': 'f32', 'data': 'synthetic'}
        print(json.dumps(out), flush=True)
        plan.close()
        del d, m_g, m_d, m_a
        torch.cuda.empty_cache()


def configs_scan(pairs: int, oracle: bool):
    """Forward + adjoint pairs on the other workloads (single CMP, realistic CMP, 8-CMP batch,
    32-CMP large batch with each q-grid storage type): pair time, algorithmic GB/s, per-kernel
    times, the plain per-gather FP32 operator and, for the single and realistic CMP, the FP64
    oracle's pair on one core.  One JSON line per (workload, storage)."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2505_00387_amd import plan_from_workload
    dev = torch.device('cuda:0')
    for c in (1, 2, 3, 5):
        w = wl.CONFIGS[c](with_data=False)
        a = w.axes
        for gd in ((0, 1, 2) if c == 5 else (0,)):
            plan = plan_from_workload(w, device=0, grid_dtype=gd)
            m = torch.randn(plan.model_shape, dtype=torch.float32, device=dev)
            dd = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
            ma = torch.empty(plan.model_shape, dtype=torch.float32, device=dev)

            def pair():
                plan.forward(m, dd)
                plan.adjoint(dd, ma)
            t_pair = _timed(pair, pairs)
            plan.profile(True)
            pair()
            torch.cuda.synchronize()
            prof = {k: round(ms / n, 4) for k, (ms, n) in plan.profile_read().items() if n}
            plan.profile(False)
            nf = plan.info['nfreq']
            rows = w.batch * a.ntheta * a.nq
            bop = 4 * rows * a.ntau + 16 * rows * nf + 16 * plan.ntraces * nf + 4 * plan.ntraces * a.nt
            out = {'metric': 'fwd+adj pair', 'workload': w.name, 'gathers': w.batch, 'traces': plan.ntraces,
                   'grid_dtype': ('f32', 'f16', 'bf16')[gd], 'pair_ms': round(1e3 * t_pair, 4),
                   'pairs_per_s': round(w.batch / t_pair, 1), 'alg_GBs': round(2 * bop / t_pair / 1e9, 1),
                   'hbm_frac': round(2 * bop / t_pair / 1e9 / HBM_PEAK_GBS, 4), 'kernel_ms': prof,
                   'nfft': plan.info['nfft'], 'grid': plan.info['grid_size'],
                   'kernel_width': plan.info['kernel_width'], 'freq_tile': plan.info['freq_tile']}
            if gd == 0 and c in (1, 2, 3):
                out['plain_per_gather_fp32'] = plain_comparison(w, plan, t_pair, min(w.batch, 16), dev)
            if gd == 0 and c in (1, 2) and oracle:
                out['cpu_baseline'] = cpu_baseline_pair(w)
            print(json.dumps(out), flush=True)
            plan.close()
            del m, dd, ma
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--iters', type=int, default=0, help='FISTA iterations per solve (0: workload default, 100)')
    ap.add_argument('--no-cpu', action='store_true', help='skip the oracle CPU-baseline leg')
    ap.add_argument('--pairs', type=int, default=5, help='timed fwd+adj pairs')
    ap.add_argument('--plain-sample', type=int, default=16, help='gathers of the plain-operator comparison (0: skip)')
    ap.add_argument('--configs', action='store_true',
                    help='instead of the solve: fwd+adj pairs on the other workloads')
    ap.add_argument('--table1', action='store_true',
                    help='instead of the solve: the velocity-scan timing at the paper\'s table shapes')
    ap.add_argument('--gfst', default='',
                    help='GFST setting as JSON (keys sigma, kernel_width, freq_tile, freq_tile_adjoint, '
                         'block_threads, block_threads_adjoint) instead of autotuning it, e.g. to take '
                         'counters on the setting a timed run chose')
    args = ap.parse_args()
    if args.gpus != 1:
        print('bench.py runs on one GPU only: the batched solve shards by gather, and this bench '
              'measures one GPU\'s share (use --gpus 1).', file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl
    from paper_2505_00387_amd import plan_from_workload

    assert torch.cuda.is_available(), 'bench.py needs a GPU'
    if args.table1:
        table1_scan(max(args.steps, 5))
        return
    if args.configs:
        configs_scan(max(args.pairs, 5), not args.no_cpu)
        return
    dev = torch.device('cuda:0')
    t0 = time.perf_counter()
    w = wl.config4(with_data=True)
    t_gen = time.perf_counter() - t0
    n_iter = args.iters or w.n_iter
    print(f'# workload {w.name}: {w.batch} gathers, {int(w.trace_ptr[-1])} traces, generated in {t_gen:.1f} s',
          file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    pinned = json.loads(args.gfst) if args.gfst else {}
    allowed = {'sigma', 'kernel_width', 'freq_tile', 'freq_tile_adjoint', 'block_threads', 'block_threads_adjoint'}
    if set(pinned) - allowed:
        raise SystemExit(f'--gfst: unknown keys {sorted(set(pinned) - allowed)}')
    plan = plan_from_workload(w, device=0, **pinned)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    d = torch.tensor(w.data_all(), dtype=torch.float32, device=dev)
    m = torch.zeros(plan.model_shape, dtype=torch.float32, device=dev)

    t0 = time.perf_counter()
    n2 = plan.operator_norm2(30)
    gam = (1.0 / (1.05 * n2)).contiguous()
    torch.cuda.synchronize()
    t_power = time.perf_counter() - t0
    print(f'# plan {t_plan:.2f} s, power iteration {t_power:.2f} s, info {plan.info}', file=sys.stderr, flush=True)

    def step():
        m.zero_()
        plan.sparse_solve(d, n_iter, m=m, step=gam, graph=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        print(f'# step {i + 1}/{args.steps} done at {time.perf_counter() - t0:.2f} s', file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    ms_step = 1000.0 * elapsed / args.steps
    gathers_per_s = w.batch / (elapsed / args.steps)

    # forward + adjoint pairs over the batch
    mr = torch.randn(plan.model_shape, dtype=torch.float32, device=dev)
    dd = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    ma = torch.empty(plan.model_shape, dtype=torch.float32, device=dev)
    plan.forward(mr, dd)
    plan.adjoint(dd, ma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.pairs):
        plan.forward(mr, dd)
        plan.adjoint(dd, ma)
    torch.cuda.synchronize()
    t_pair = (time.perf_counter() - t0) / args.pairs
    pairs_per_s = w.batch / t_pair

    # deconvolutive operator pair L_w = W L (Section 4), a 25 Hz Ricker wavelet of 65 taps
    half = int(np.ceil(1.6 / (25.0 * w.axes.dt)))
    tt = w.axes.dt * np.arange(-half, half + 1)
    plan.set_wavelet(wl.ricker(tt, 25.0), half)
    plan.forward(mr, dd)
    plan.adjoint(dd, ma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.pairs):
        plan.forward(mr, dd)
        plan.adjoint(dd, ma)
    torch.cuda.synchronize()
    t_pair_w = (time.perf_counter() - t0) / args.pairs
    plan.set_wavelet(None)

    # the paper's linear k-interpolation (kernel width 2, sigma 2) on the same batch
    plan_lin = plan_from_workload(w, device=0, kernel_width=2, sigma=2.0)
    plan_lin.forward(mr, dd)
    plan_lin.adjoint(dd, ma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.pairs):
        plan_lin.forward(mr, dd)
        plan_lin.adjoint(dd, ma)
    torch.cuda.synchronize()
    t_pair_lin = (time.perf_counter() - t0) / args.pairs
    plan_lin.close()

    # velocity estimate of the solved cube (Section 3): one read of the model, two small outputs
    plan.velocity(m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.velocity(m)
    torch.cuda.synchronize()
    t_vel = (time.perf_counter() - t0) / 5
    vel_bytes = 4 * w.batch * w.axes.ntheta * w.axes.ntau * (w.axes.nq + 2)

    # the same solve as a captured hipGraph (the library's default): capture, then one timed replay
    m.zero_()
    plan.sparse_solve(d, n_iter, m=m, step=gam, graph=True)
    torch.cuda.synchronize()
    m.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.sparse_solve(d, n_iter, m=m, step=gam, graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    a = w.axes
    nf = plan.info['nfreq']
    rows = w.batch * a.ntheta * a.nq
    bop = 4 * rows * a.ntau + 16 * rows * nf + 16 * plan.ntraces * nf + 4 * plan.ntraces * a.nt
    pair_gbs = 2 * bop / t_pair / 1e9

    plain = None
    if args.plain_sample > 0:
        print('# timing the plain per-gather FP32 operator', file=sys.stderr, flush=True)
        plain = plain_comparison(w, plan, t_pair, args.plain_sample, dev)

    kernels = {}
    for name, (ms, n) in prof.items():
        if n == 0:
            continue
        avg = ms / n
        byt = kernel_bytes(plan, name)
        kernels[name] = {'launches': n, 'avg_ms': round(avg, 4), 'total_ms': round(ms, 2),
                         'alg_GBs': round(byt / (avg * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]['total_ms'])
    avg = kernels[dom]['avg_ms']
    ach = kernel_bytes(plan, dom) / (avg * 1e-3) / 1e9
    gfst = {'grid': plan.info['grid_size'], 'kernel_width': plan.info['kernel_width'],
            'freq_tile': plan.info['freq_tile'], 'freq_tile_adjoint': plan.info['freq_tile_adjoint'],
            'block_threads': plan.info['block_threads'], 'block_threads_adjoint': plan.info['block_threads_adjoint']}
    traffic = load_traffic(dom, w.name, gfst)
    roofline = {'bound': 'hbm', 'achieved': round(ach, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
                'frac': round(ach / HBM_PEAK_GBS, 4), 'traffic': traffic, 'kernel': dom,
                'alg_bytes_per_launch': int(kernel_bytes(plan, dom)), 'avg_ms': avg}

    cpu = None
    if not args.no_cpu:
        print('# timing the FP64 oracle on the host cores (about 30-40 s)', file=sys.stderr, flush=True)
        cpu = cpu_baseline(w)

    out = {
        'metric': 'CMP gathers/s, 100-iter sparse AAHRT at <=1e-4 rel err',
        'value': round(gathers_per_s, 2), 'unit': 'gathers/s', 'n_gpus': 1, 'steps': args.steps,
        'warmup': args.warmup, 'ms_per_step': round(ms_step, 2), 'higher_is_better': True,
        'scaling': 'weak', 'vs_baseline': None, 'dtype': 'f32', 'data': 'synthetic',
        'config': {'workload': w.name, 'gathers': w.batch, 'traces': plan.ntraces, 'nt': a.nt,
                   'nq': a.nq, 'ntheta': a.ntheta, 'fista_iters': n_iter, 'nfft': plan.info['nfft'],
                   'kernel_width': plan.info['kernel_width'], 'grid': plan.info['grid_size'],
                   'sigma': plan.info['sigma'], 'freq_tile': plan.info['freq_tile'],
                   'freq_tile_adjoint': plan.info['freq_tile_adjoint'],
                   'block_threads': plan.info['block_threads'],
                   'block_threads_adjoint': plan.info['block_threads_adjoint']},
        'roofline': roofline,
        'cpu_baseline': cpu,
        'secondary': {'graph_solve_ms': round(1e3 * t_graph, 2), 'graph_gathers_per_s': round(w.batch / t_graph, 2),
                      'velocity_estimate_ms': round(1e3 * t_vel, 3),
                      'deconvolutive_fwd_adj_pair_ms': round(1e3 * t_pair_w, 3),
                      'deconvolutive_wavelet_taps': 2 * half + 1,
                      'linear_k_interp_fwd_adj_pair_ms': round(1e3 * t_pair_lin, 3),
                      'velocity_estimate_GBs': round(vel_bytes / t_vel / 1e9, 1),
                      'fwd_adj_pairs_per_s': round(pairs_per_s, 1), 'fwd_adj_pair_ms': round(1e3 * t_pair, 3),
                      'fwd_adj_alg_GBs': round(pair_gbs, 1), 'setup_plan_s': round(t_plan, 3),
                      'setup_autotune_s': round(plan.info['autotune_seconds'], 3),
                      'autotune_candidates': plan.info['autotune_candidates'],
                      'setup_power_iteration_s': round(t_power, 3), 'plain_per_gather_fp32': plain},
        'kernels': kernels,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == '__main__':
    main()
