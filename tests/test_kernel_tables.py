"""Host-side checks of the constants compiled into the GFST kernels.  CPU only.

The kernel taps at the sigma = 2 shape come from literal polynomial coefficients in
csrc/es_poly.hpp, written by csrc/gen_es_poly.py.  These tests regenerate the header and
compare, and evaluate the committed coefficients (as the kernel does: tap t < w/2 is
E_t(y^2) + y O_t(y^2), tap w-1-t is E_t(y^2) - y O_t(y^2), the middle tap of an odd w is
E(y^2)) against the exponential-of-semicircle kernel itself, exp(beta (sqrt(1 - z^2) - 1)) with
beta = 0.98 pi (1 - 1/(2 sigma)) w at sigma = 2 (Barnett, Magland and af Klinteberg, SIAM J.
Sci. Comput. 41, 2019), at the tap distances of a point x in [0, 1) of a cell.
"""
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, 'paper_2505_00387_amd', 'csrc')
HEADER = os.path.join(CSRC, 'es_poly.hpp')


def _parse(w: int):
    src = open(HEADER).read()
    blk = src[src.index(f'struct EsPoly<{w}> {{'):]
    blk = blk[:blk.index('\n};') + 3]
    de = int(re.search(r'DE = (\d+);', blk).group(1))
    do = int(re.search(r'DO = (\d+);', blk).group(1))

    def rows(name):
        body = re.search(name + r'\[\d+\]\[\d+\] = \{(.*?)\n  \};', blk, re.S).group(1)
        return [[float(x.strip().rstrip('f')) for x in r.split(',') if x.strip()]
                for r in re.findall(r'\{([^{}]*)\}', body)]
    e, o = rows('e'), rows('o')
    assert all(len(r) == de + 1 for r in e) and all(len(r) == do + 1 for r in o)
    return e, o


def _stated_error(w: int) -> float:
    src = open(HEADER).read()
    return float(re.search(rf'// w = {w}, beta = [0-9.]+: degree \d+, fit error ([0-9.e+-]+)', src).group(1))


def test_header_matches_its_generator():
    out = subprocess.run([sys.executable, os.path.join(CSRC, 'gen_es_poly.py')], capture_output=True, text=True,
                         check=True, cwd=CSRC).stdout
    assert out.strip() == open(HEADER).read().strip(), 'es_poly.hpp is stale: rerun gen_es_poly.py'


@pytest.mark.parametrize('w', list(range(5, 13)))
def test_tap_polynomials_match_the_kernel(w):
    """Every tap, including the mirrored ones, is the kernel to within the fit error the header
    states (rounded up by the FP32 coefficients), at 4001 points of the cell."""
    e, o = _parse(w)
    beta = 0.98 * math.pi * (1.0 - 1.0 / (2.0 * 2.0)) * w
    x = np.linspace(0.0, 1.0, 4001)
    y = 2.0 * x - 1.0
    y2 = y * y
    worst = 0.0
    for t in range(w):
        z = 2.0 * (x + w / 2.0 - 1.0 - t) / w
        exact = np.where(np.abs(z) <= 1.0, np.exp(beta * (np.sqrt(np.maximum(1.0 - z * z, 0.0)) - 1.0)), 0.0)
        if 2 * t + 1 == w:
            got = np.polyval(e[t], y2)
        elif t < w // 2:
            got = np.polyval(e[t], y2) + y * np.polyval(o[t], y2)
        else:
            s = w - 1 - t
            got = np.polyval(e[s], y2) - y * np.polyval(o[s], y2)
        worst = max(worst, float(np.max(np.abs(got - exact))))
    assert worst <= 1.2 * _stated_error(w) + 1e-9, (w, worst)
    # the coefficients' magnitudes bound the FP32 Horner rounding the generator states (about 1e-7)
    assert max(sum(abs(c) for c in r) for r in e + o) < 2.0


def test_radix_butterflies_match_a_direct_dft(tmp_path):
    """Every radix butterfly of the LDS FFTs (2, 3, 4, 5, 8, 9, 15, 16; forward and inverse sign),
    built for the host from the same header, against a direct DFT in double."""
    import shutil
    hipcc = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(hipcc):
        pytest.skip('hipcc not available')
    exe = tmp_path / 'dft_check'
    src = os.path.join(ROOT, 'tests', 'host', 'dft_check.cpp')
    subprocess.run([hipcc, '-O2', '-std=c++17', '-x', 'hip', '--offload-arch=gfx950', '-I', CSRC, src, '-o',
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split('\n')
    rows = [ln.split() for ln in out if ln.strip()]
    assert len(rows) == 16
    for r, inv, err in rows:
        # a few FP32 roundings of magnitude-sqrt(R) sums of N(0,1) values
        assert float(err) < 2e-5 * int(r), (r, inv, err)
