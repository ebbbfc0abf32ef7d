"""aahrt_adjoint_noalloc (the adjoint that allocates nothing) against aahrt_adjoint, through the C ABI.

Both entry points run the same kernels, the second with its intermediates in the library's
static device array; the spreading accumulates in fixed point, so the two agree bit for bit.
Two calls in a row, the second on a smaller plan (the array keeps the first call's contents),
then the first plan again; a plan whose intermediates exceed the array is refused.
"""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import gfst

from gpu_common import TOL, rel, geoms, make_plan, to_dev, to_host

pytestmark = pytest.mark.gpu


def _call(lib, name, plan, d, m):
    import torch
    rc = getattr(lib, name)(plan._h, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


def _both(lib, plan, seed):
    import torch
    d = to_dev(wl.random_data(plan.ntraces, plan.axes.nt, seed))
    m_ref = torch.empty(plan.model_shape, dtype=torch.float32, device='cuda:0')
    m_na = torch.full(plan.model_shape, float('nan'), dtype=torch.float32, device='cuda:0')
    assert _call(lib, 'aahrt_adjoint', plan, d, m_ref) == 0, lib.aahrt_last_error()
    assert _call(lib, 'aahrt_adjoint_noalloc', plan, d, m_na) == 0, lib.aahrt_last_error()
    torch.cuda.synchronize()
    return d, m_ref, m_na


def test_noalloc_adjoint_equals_adjoint_on_consecutive_calls():
    import torch
    from paper_2505_00387_amd import _lib
    lib = _lib.load()
    w_big = wl.config3(with_data=False)        # 8 gathers x 512 traces, 23.6 MB of intermediates
    w_small = wl.config1(with_data=False)      # 1 gather x 256 traces
    p_big = make_plan(w_big, sigma=2.0, freq_tile=16)
    p_small = make_plan(w_small, sigma=2.0, freq_tile=16)
    d1, r1, n1 = _both(lib, p_big, 61)
    print('first call (8 gathers): max |diff|', float((n1 - r1).abs().max()))
    assert torch.equal(n1, r1)
    d2, r2, n2 = _both(lib, p_small, 62)
    print('second call (1 gather): max |diff|', float((n2 - r2).abs().max()))
    assert torch.equal(n2, r2)
    # the smaller call against the oracle too (the bound every FP32 result is held to)
    g = geoms(w_small)[0]
    assert rel(to_host(n2)[0], gfst.adjoint(to_host(d2), g)) < TOL
    # and the larger plan once more after the smaller one
    _, r3, n3 = _both(lib, p_big, 63)
    assert torch.equal(n3, r3)
    p_big.close()
    p_small.close()


def test_noalloc_adjoint_refuses_a_plan_larger_than_its_array():
    import torch
    from paper_2505_00387_amd import _lib
    lib = _lib.load()
    ax = wl.config2(with_data=False).axes
    x, y = wl.disk_offsets(np.random.default_rng(9), 4096, 3.0)      # (1024 + 4096) x 2160 x 8 B > 64 MiB
    w = wl.Workload('too_large', ax, [wl.Gather(x=x, y=y)], 0, 'one CMP of 4096 traces')
    plan = make_plan(w, sigma=2.0, freq_tile=16)
    d = torch.zeros(plan.data_shape, dtype=torch.float32, device='cuda:0')
    m = torch.zeros(plan.model_shape, dtype=torch.float32, device='cuda:0')
    rc = _call(lib, 'aahrt_adjoint_noalloc', plan, d, m)
    msg = lib.aahrt_last_error().decode()
    print(rc, msg)
    assert rc == _lib.AAHRT_E_UNSUPPORTED and 'scratch' in msg
    plan.close()
