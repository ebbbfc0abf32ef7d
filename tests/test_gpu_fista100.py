"""100-iteration sparse AAHRT on the GPU against stored FP64 oracle iterates (Section 4).

The references in tests/golden/fista100/ were written by tests/golden/make_fista100.py,
which calls only the oracle: per case lambda_b, gamma_b and the FISTA iterates m_k at
k = 1, 10, 50 and 100.  Each test runs aahrt_sparse_solve with the oracle's lambda_b and
gamma_b for k iterations from m = 0 and holds the k-th iterate to a relative L2 error of
1e-4 per gather, the bound the method is held to in FP32.  The error at every stored k is
printed: the error-versus-iteration curve of the solve.
"""
import hashlib
import os

import numpy as np
import pytest

import workloads as wl

from gpu_common import TOL, rel, make_plan, to_dev, to_host

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), 'golden', 'fista100')


def load_reference(name):
    """Stored lambda, gamma and dense iterates {k: m_k} of one case."""
    z = np.load(os.path.join(GOLD, f'{name}.npz'), allow_pickle=False)
    shape = tuple(int(v) for v in z['shape'])
    size = int(np.prod(shape))
    its = {}
    for k in z['keep']:
        k = int(k)
        m = np.zeros(size)
        m[z[f'idx_{k}']] = z[f'val_{k}']
        its[k] = m.reshape(shape)
    return {'lam': float(z['lam']), 'gamma': float(z['gamma']), 'nfft': int(z['nfft']),
            'gather': int(z['gather']), 'sha': str(z['data_sha']), 'its': its}


def data_sha(d):
    return hashlib.sha256(np.ascontiguousarray(d, dtype=np.float64).tobytes()).hexdigest()


def config4_cases():
    return sorted(f[:-4] for f in os.listdir(GOLD) if f.startswith('config4_b') and f.endswith('.npz'))


def _solve_curve(plan, d, lam, gam, keep):
    """Iterate k of the solve for every k in keep (each a fresh solve from m = 0)."""
    out = {}
    for k in keep:
        x, _ = plan.sparse_solve(to_dev(d), k, lam=to_dev(lam), step=to_dev(gam))
        out[k] = to_host(x)
    return out


@pytest.mark.parametrize('config', [1, 2])
def test_fista100_single_cmp(config):
    """Configs 1 and 2 (the realistic 1024-trace CMP), 100 iterations."""
    ref = load_reference(f'config{config}')
    w = wl.CONFIGS[config](with_data=True)
    d = w.gathers[0].data
    assert data_sha(d) == ref['sha'], 'stored reference is stale: rerun tests/golden/make_fista100.py'
    plan = make_plan(w)
    assert plan.info['nfft'] == ref['nfft']
    got = _solve_curve(plan, d, np.array([ref['lam']]), np.array([ref['gamma']]), sorted(ref['its']))
    errs = {k: rel(got[k][0], ref['its'][k]) for k in sorted(ref['its'])}
    print(f'config {config} sigma {plan.info["sigma"]} w {plan.info["kernel_width"]}: error by iteration',
          {k: f'{e:.2e}' for k, e in errs.items()})
    plan.close()
    for k, e in errs.items():
        assert e < TOL, (k, e)


def test_fista100_uneven_batch_subset():
    """Eight gathers of the 256-gather workload (smallest, median and largest fold among them)
    solved together as one batch of uneven folds, with the whole batch's FFT length."""
    names = config4_cases()
    assert len(names) == 8
    refs = [load_reference(n) for n in names]
    picks = [r['gather'] for r in refs]
    w4 = wl.config4(with_data=True)
    w = wl.Workload('cmp_batch256_uneven_nt1024_subset', w4.axes, [w4.gathers[b] for b in picks], 100, 'subset')
    for r, b in zip(refs, picks):
        assert data_sha(w4.gathers[b].data) == r['sha'], 'stored reference is stale'
    plan = make_plan(w, nfft=refs[0]['nfft'])
    lam = np.array([r['lam'] for r in refs])
    gam = np.array([r['gamma'] for r in refs])
    d = w.data_all()
    got = _solve_curve(plan, d, lam, gam, sorted(refs[0]['its']))
    worst = 0.0
    for i, (r, b) in enumerate(zip(refs, picks)):
        errs = {k: rel(got[k][i], r['its'][k]) for k in sorted(r['its'])}
        print(f'gather {b} fold {w4.gathers[b].x.size}: error by iteration', {k: f'{e:.2e}' for k, e in errs.items()})
        worst = max(worst, max(errs.values()))
    plan.close()
    assert worst < TOL, worst


def test_fista100_full_batch_as_benchmarked():
    """The benchmark's launch configuration: all 256 gathers in one autotuned plan, one captured
    100-iteration solve.  The eight stored gathers take the oracle's lambda and gamma, the others
    the library's own (0.05 max|L^T d| and the power iteration); the eight are checked."""
    import torch
    names = config4_cases()
    refs = [load_reference(n) for n in names]
    w = wl.config4(with_data=True)
    plan = make_plan(w)
    assert plan.info['nfft'] == refs[0]['nfft']
    d = to_dev(w.data_all())
    lam = plan.lambda_max(d) * 0.05
    gam = 1.0 / (1.05 * plan.operator_norm2(30))
    for r in refs:
        lam[r['gather']] = r['lam']
        gam[r['gather']] = r['gamma']
    m = torch.zeros(plan.model_shape, dtype=torch.float32, device='cuda:0')
    plan.sparse_solve(d, 100, m=m, lam=lam.contiguous(), step=gam.contiguous(), graph=True)
    x = to_host(m)
    worst = 0.0
    for r in refs:
        b = r['gather']
        e = rel(x[b], r['its'][100])
        print(f'full batch, gather {b}: error at iteration 100 {e:.2e}')
        worst = max(worst, e)
    print('plan', {k: plan.info[k] for k in ('sigma', 'kernel_width', 'freq_tile', 'freq_tile_adjoint',
                                              'nufft_error_estimate')})
    plan.close()
    assert worst < TOL, worst
