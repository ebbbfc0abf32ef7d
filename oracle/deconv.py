"""Deconvolutive AAHRT (FP64).  Test infrastructure only.

Section 4, "Deconvolutive AAHRT": the basis functions carry the seismic
wavelet w(t) instead of a delta in time, which amounts to R_w^-1 = W R^-1 with
W the linear convolution of every trace with the wavelet along t.

Reading: the wavelet is given by taps w[0..nw-1] with origin at index c, and W
keeps the nt samples of the trace (zero outside):
  (W d)[s] = sum_j w[j] d[s - (j - c)],
its transpose is the correlation
  (W^T r)[s] = sum_j w[j] r[s + (j - c)],
and the operator pair is L_w = W L, L_w^T = L^T W^T.
"""
from __future__ import annotations

import numpy as np

from . import gfst


def convolve(d: np.ndarray, w: np.ndarray, c: int) -> np.ndarray:
    """W d for d [..., nt] (direct sum over the taps)."""
    d = np.asarray(d, dtype=np.float64)
    nt = d.shape[-1]
    out = np.zeros_like(d)
    for j, wj in enumerate(np.asarray(w, dtype=np.float64)):
        k = j - c                       # output s takes d[s - k]
        if k >= 0:
            if k < nt:
                out[..., k:] += wj * d[..., :nt - k]
        else:
            if -k < nt:
                out[..., :nt + k] += wj * d[..., -k:]
    return out


def correlate(r: np.ndarray, w: np.ndarray, c: int) -> np.ndarray:
    """W^T r for r [..., nt]."""
    r = np.asarray(r, dtype=np.float64)
    nt = r.shape[-1]
    out = np.zeros_like(r)
    for j, wj in enumerate(np.asarray(w, dtype=np.float64)):
        k = j - c                       # output s takes r[s + k]
        if k >= 0:
            if k < nt:
                out[..., :nt - k] += wj * r[..., k:]
        else:
            if -k < nt:
                out[..., -k:] += wj * r[..., :nt + k]
    return out


def forward(m, geom, w, c):
    return convolve(gfst.forward(m, geom), w, c)


def adjoint(d, geom, w, c, rows=None):
    return gfst.adjoint(correlate(d, w, c), geom, rows=rows)
