"""Python face of the C ABI: a Plan object and the operator calls on torch device tensors.

PyTorch supplies device memory and the stream only; the arithmetic runs in
libaahrt.so.  Names follow include/aahrt.h.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib
from ._lib import check


@dataclass
class Axes:
    nt: int
    dt: float
    ntau: int
    dtau: float
    nq: int
    q_min: float
    q_max: float
    ntheta: int
    stretch: int = 2


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Plan:
    """A batch of CMP gathers on one set of axes (aahrt_plan_create)."""

    def __init__(self, axes, trace_ptr, x_km, y_km, nfft: int = 0, nufft_tol: float = 0.0,
                 sigma: float = 0.0, kernel_width: int = 0, freq_tile: int = 0, grid_dtype: int = 0,
                 gfst_kind: int = 0, block_threads: int = 0, freq_tile_adjoint: int = 0,
                 block_threads_adjoint: int = 0, device: int = 0):
        lib = _lib.load()
        self._lib = lib
        p = _lib.Params(nt=axes.nt, dt=axes.dt, ntau=axes.ntau, dtau=axes.dtau, nq=axes.nq,
                        q_min=axes.q_min, q_max=axes.q_max, ntheta=axes.ntheta,
                        stretch=getattr(axes, 'stretch', 2), nfft=nfft, nufft_tol=nufft_tol,
                        sigma=sigma, kernel_width=kernel_width, freq_tile=freq_tile,
                        grid_dtype=grid_dtype, gfst_kind=gfst_kind, block_threads=block_threads,
                        freq_tile_adjoint=freq_tile_adjoint, block_threads_adjoint=block_threads_adjoint)
        tp = np.ascontiguousarray(trace_ptr, dtype=np.int64)
        xs = np.ascontiguousarray(x_km, dtype=np.float64)
        ys = np.ascontiguousarray(y_km, dtype=np.float64)
        self.axes = axes
        self.batch = int(tp.size - 1)
        self.trace_ptr = tp
        self.device = device
        self._params = p
        h = ctypes.c_void_p()
        check(lib.aahrt_plan_create(ctypes.byref(h), ctypes.byref(p), self.batch,
                                    tp.ctypes.data, xs.ctypes.data, ys.ctypes.data, device))
        self._h = h
        info = _lib.PlanInfo()
        check(lib.aahrt_plan_query(h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in _lib.PlanInfo._fields_}

    @property
    def ntraces(self) -> int:
        return int(self.trace_ptr[-1])

    @property
    def model_shape(self):
        a = self.axes
        return (self.batch, a.ntheta, a.nq, a.ntau)

    @property
    def data_shape(self):
        return (self.ntraces, self.axes.nt)

    def gfst_setting(self) -> dict:
        """The GFST setting this plan runs (autotuned or requested), as keyword arguments that
        re-create it on another Plan without timing it again."""
        i = self.info
        return {'sigma': i['sigma'], 'kernel_width': i['kernel_width'], 'freq_tile': i['freq_tile'],
                'freq_tile_adjoint': i['freq_tile_adjoint'], 'block_threads': i['block_threads'],
                'block_threads_adjoint': i['block_threads_adjoint']}

    def close(self):
        if getattr(self, '_h', None) is not None and self._h.value:
            self._lib.aahrt_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ operators
    def _check(self, t, shape, name):
        import torch
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f'{name} must be a contiguous float32 device tensor')
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f'{name} has shape {tuple(t.shape)}, expected {tuple(shape)}')

    def forward(self, m, d=None, stream=None):
        """d = L m."""
        import torch
        self._check(m, self.model_shape, 'm')
        if d is None:
            d = torch.empty(self.data_shape, dtype=torch.float32, device=m.device)
        self._check(d, self.data_shape, 'd')
        check(self._lib.aahrt_forward(self._h, m.data_ptr(), d.data_ptr(), _stream(stream)))
        return d

    def adjoint(self, d, m=None, stream=None):
        """m = L^T d."""
        import torch
        self._check(d, self.data_shape, 'd')
        if m is None:
            m = torch.empty(self.model_shape, dtype=torch.float32, device=d.device)
        self._check(m, self.model_shape, 'm')
        check(self._lib.aahrt_adjoint(self._h, d.data_ptr(), m.data_ptr(), _stream(stream)))
        return m

    def adjoint_direct(self, d, m=None, stream=None):
        """Time-domain direct-summation adjoint (aahrt_adjoint_direct), for timing comparison."""
        import torch
        self._check(d, self.data_shape, 'd')
        if m is None:
            m = torch.empty(self.model_shape, dtype=torch.float32, device=d.device)
        self._check(m, self.model_shape, 'm')
        check(self._lib.aahrt_adjoint_direct(self._h, d.data_ptr(), m.data_ptr(), _stream(stream)))
        return m

    def adjoint_grid(self, d, m=None, stream=None):
        """Algorithm 2 of Section 3.2 on regular offset grids (aahrt_adjoint_grid)."""
        import torch
        self._check(d, self.data_shape, 'd')
        if m is None:
            m = torch.empty(self.model_shape, dtype=torch.float32, device=d.device)
        self._check(m, self.model_shape, 'm')
        check(self._lib.aahrt_adjoint_grid(self._h, d.data_ptr(), m.data_ptr(), _stream(stream)))
        return m

    def lambda_max(self, d, stream=None):
        import torch
        self._check(d, self.data_shape, 'd')
        out = torch.empty(self.batch, dtype=torch.float32, device=d.device)
        check(self._lib.aahrt_lambda_max(self._h, d.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def set_wavelet(self, w=None, center=0):
        """Deconvolutive operator L_w = W L (aahrt_set_wavelet); w None or empty: plain L."""
        import numpy as np
        if w is None or len(w) == 0:
            check(self._lib.aahrt_set_wavelet(self._h, None, 0, 0))
            self._wavelet = None
            return
        wa = np.ascontiguousarray(w, dtype=np.float32)
        check(self._lib.aahrt_set_wavelet(self._h, wa.ctypes.data, int(wa.size), int(center)))
        self._wavelet = (wa, int(center))

    def velocity(self, m, stream=None):
        """Automatic anisotropic velocity estimate (aahrt_velocity): returns (qbar, v), each
        [batch, ntheta, ntau]; qbar = v^-2 in s^2/km^2, v in km/s."""
        import torch
        self._check(m, self.model_shape, 'm')
        a = self.axes
        qbar = torch.empty((self.batch, a.ntheta, a.ntau), dtype=torch.float32, device=m.device)
        v = torch.empty_like(qbar)
        check(self._lib.aahrt_velocity(self._h, m.data_ptr(), qbar.data_ptr(), v.data_ptr(), _stream(stream)))
        return qbar, v

    def reconstruct(self, m, x_km, y_km, stream=None):
        """Data of the model m on another trace geometry (one gather per model gather):
        L (L_w when a wavelet is set) applied through a plan on the new offsets (x_km, y_km
        lists of per-gather arrays)."""
        import numpy as np
        tp = np.concatenate([[0], np.cumsum([len(x) for x in x_km])]).astype(np.int64)
        other = Plan(self.axes, tp, np.concatenate(x_km), np.concatenate(y_km), nfft=0,
                     nufft_tol=self._params.nufft_tol, sigma=self.info['sigma'],
                     kernel_width=self._params.kernel_width, gfst_kind=self._params.gfst_kind,
                     block_threads=self._params.block_threads,
                     block_threads_adjoint=self._params.block_threads_adjoint, device=self.device)
        try:
            if getattr(self, '_wavelet', None) is not None:
                other.set_wavelet(*self._wavelet)
            return other.forward(m, stream=stream)
        finally:
            other.close()

    def operator_norm2(self, n_iter=30, stream=None):
        import torch
        out = torch.empty(self.batch, dtype=torch.float32, device=f'cuda:{self.device}')
        check(self._lib.aahrt_operator_norm2(self._h, int(n_iter), out.data_ptr(), _stream(stream)))
        return out

    def profile(self, enable: bool = True):
        check(self._lib.aahrt_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} since the last profile(True)."""
        out = {}
        for k, name in enumerate(_lib.KERNELS):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            check(self._lib.aahrt_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def sparse_solve(self, d, n_iter, m=None, lam=None, step=None, ista=False, graph=True,
                     objective=False, stream=None):
        """FISTA (or ISTA) sparse AAHRT; returns (m, objective or None)."""
        import torch
        self._check(d, self.data_shape, 'd')
        if m is None:
            m = torch.zeros(self.model_shape, dtype=torch.float32, device=d.device)
        self._check(m, self.model_shape, 'm')
        for v, nm in ((lam, 'lam'), (step, 'step')):
            if v is not None:
                self._check(v, (self.batch,), nm)
        obj = torch.empty((n_iter, self.batch), dtype=torch.float32, device=d.device) if objective else None
        flags = (_lib.SOLVE_ISTA if ista else 0) | (0 if graph else _lib.SOLVE_NO_GRAPH)
        check(self._lib.aahrt_sparse_solve(self._h, d.data_ptr(), m.data_ptr(), _ptr(lam), _ptr(step),
                                           int(n_iter), flags, _ptr(obj), _stream(stream)))
        return m, obj


def plan_from_workload(w, device=0, **kw) -> Plan:
    """Plan for a workloads.Workload (offsets already in km)."""
    return Plan(w.axes, w.trace_ptr, w.x_all, w.y_all, device=device, **kw)
