"""Oracle-1: the GFST operator pair with direct nonuniform DFTs (FP64).  Test infrastructure only.

Forward operator L (model m[theta, q, tau] -> data d[trace, t]); it follows
Algorithm 1 of Section 3.1 and the factorisation R^-1 = S^-1 F1^-1 P F2 S of
Section 4:

1. S (stretch, Section 3.4):  M'[j,l,r] = sum_i S[r,i] M[j,l,i]
2. F along tau' (the tau'-half of step 2; the q-half is folded into step 3):
       Mh[j,l,f] = sum_{r<nt'} M'[j,l,r] exp(-2 pi i f r / N),  f = 0..N/2-1
3. P, the GFST relation of Section 3.1 (k_q = f'(x^2+y^2), theta = arctan(y/x)),
   evaluated exactly: the q-Fourier transform of Mh at k_q is summed directly,
   and theta is interpolated linearly between its two grid neighbours:
       Dh[n,f] = sum_j w[n,j] sum_l Mh[j,l,f] exp(-2 pi i f'_f q_l h_n^2),
       f'_f = f/(N dt')
4. F1^-1 along t':  D'[n,r] = (1/N) (Re Dh[n,0] + 2 Re sum_{f=1}^{N/2-1} Dh[n,f] exp(2 pi i f r/N)),
   r < nt'  (the Nyquist bin is not carried)
5. S^-1 (unstretch):  d[n,s] = sum_r U[s,r] D'[n,r]

The adjoint is the exact transpose of these five steps, taken in reverse
order (the real inner product is used on every complex intermediate).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry

_FCHUNK = 32


def _phase(geom: Geometry, f_idx: np.ndarray, h2: np.ndarray, q=None) -> np.ndarray:
    """exp(-2 pi i f'_f q_l h_n^2) as [len(f_idx), ntr, nq] (or [len(f_idx), ntr, len(q)] for
    the curvatures q given)."""
    fp = f_idx / (geom.nfft * geom.dt_str)
    qv = geom.q if q is None else np.asarray(q, dtype=np.float64)
    arg = fp[:, None, None] * h2[None, :, None] * qv[None, None, :]
    return np.exp(-2j * np.pi * arg)


# ---------------------------------------------------------------- forward
def stretch(m: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 1: [..., ntau] -> [..., nt']."""
    return m @ geom.S().T


def spectrum(mp: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 2 (time half): [..., nt'] -> [..., N/2] complex."""
    return np.fft.rfft(mp, n=geom.nfft, axis=-1)[..., :geom.nf]


def gfst_map(mh: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 3: Mh[theta, q, f] -> Dh[trace, f] by the direct nonuniform DFT."""
    W = geom.W()
    h2 = geom.h2
    ntr = h2.size
    dh = np.zeros((ntr, geom.nf), dtype=np.complex128)
    for f0 in range(0, geom.nf, _FCHUNK):
        fi = np.arange(f0, min(f0 + _FCHUNK, geom.nf))
        E = _phase(geom, fi, h2)                        # [fc, n, l]
        A = np.einsum('nj,jlf->fnl', W, mh[:, :, fi])    # sum over the two theta neighbours
        dh[:, fi] = np.einsum('fnl,fnl->nf', A, E)       # sum over q
    return dh


def inverse_spectrum(dh: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 4: [..., N/2] -> [..., nt'] (inverse real DFT with a zero Nyquist bin)."""
    pad = np.zeros(dh.shape[:-1] + (geom.nf + 1,), dtype=np.complex128)
    pad[..., :geom.nf] = dh
    return np.fft.irfft(pad, n=geom.nfft, axis=-1)[..., :geom.nt_str]


def unstretch(dp: np.ndarray, geom: Geometry) -> np.ndarray:
    """Step 5: [..., nt'] -> [..., nt]."""
    return dp @ geom.U().T


def forward(m: np.ndarray, geom: Geometry) -> np.ndarray:
    """d = L m for one gather.  m: [ntheta, nq, ntau] -> d: [ntr, nt]."""
    m = np.asarray(m, dtype=np.float64)
    mh = spectrum(stretch(m, geom), geom)
    dh = gfst_map(mh, geom)
    return unstretch(inverse_spectrum(dh, geom), geom)


def forward_traces(m: np.ndarray, geom: Geometry, idx) -> np.ndarray:
    """Rows idx of L m (each output trace depends only on its own offset)."""
    return forward(m, geom.subset(idx))


# ---------------------------------------------------------------- adjoint
def unstretch_T(g: np.ndarray, geom: Geometry) -> np.ndarray:
    return g @ geom.U()


def inverse_spectrum_T(gp: np.ndarray, geom: Geometry) -> np.ndarray:
    """Transpose of step 4: [..., nt'] -> [..., N/2] complex, weights c_f/N (c_0 = 1, else 2)."""
    c = np.full(geom.nf, 2.0)
    c[0] = 1.0
    return np.fft.rfft(gp, n=geom.nfft, axis=-1)[..., :geom.nf] * (c / geom.nfft)


def gfst_map_T(gh: np.ndarray, geom: Geometry, rows=None) -> np.ndarray:
    """Transpose of step 3: Gh[trace, f] -> Hh[theta, q, f] (or only the (j, l) pairs in rows)."""
    W = geom.W()
    h2 = geom.h2
    if rows is None:
        out = np.zeros((geom.ntheta, geom.nq, geom.nf), dtype=np.complex128)
    else:
        out = np.zeros((len(rows), geom.nf), dtype=np.complex128)
    for f0 in range(0, geom.nf, _FCHUNK):
        fi = np.arange(f0, min(f0 + _FCHUNK, geom.nf))
        if rows is None:
            Ec = np.conj(_phase(geom, fi, h2))          # [fc, n, l]
            B = Ec * gh[:, fi].T[:, :, None]             # [fc, n, l]
            out[:, :, fi] = np.einsum('nj,fnl->jlf', W, B)
        else:
            # only the curvatures of the requested rows: the same phases, fewer of them
            for k, (j, l) in enumerate(rows):
                Ec = np.conj(_phase(geom, fi, h2, q=geom.q[l:l + 1]))[:, :, 0]   # [fc, n]
                out[k, fi] = W[:, j] @ (Ec * gh[:, fi].T).T
    return out


def spectrum_T(hh: np.ndarray, geom: Geometry) -> np.ndarray:
    """Transpose of step 2: [..., N/2] -> [..., nt'], Re sum_f Hh[f] exp(+2 pi i f r/N)."""
    pad = np.zeros(hh.shape[:-1] + (geom.nfft,), dtype=np.complex128)
    pad[..., :geom.nf] = hh
    return (np.fft.ifft(pad, axis=-1).real * geom.nfft)[..., :geom.nt_str]


def stretch_T(hp: np.ndarray, geom: Geometry) -> np.ndarray:
    return hp @ geom.S()


def adjoint(d: np.ndarray, geom: Geometry, rows=None) -> np.ndarray:
    """m = L^T d for one gather.  d: [ntr, nt] -> m: [ntheta, nq, ntau] (or [len(rows), ntau])."""
    d = np.asarray(d, dtype=np.float64)
    gh = inverse_spectrum_T(unstretch_T(d, geom), geom)
    hh = gfst_map_T(gh, geom, rows)
    return stretch_T(spectrum_T(hh, geom), geom)


# ---------------------------------------------------------------- batches
def forward_batch(m: np.ndarray, geoms) -> list:
    return [forward(m[b], g) for b, g in enumerate(geoms)]


def adjoint_batch(ds, geoms) -> np.ndarray:
    return np.stack([adjoint(d, g) for d, g in zip(ds, geoms)])
