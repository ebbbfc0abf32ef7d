"""Build the gfx950 HIP library libaahrt.so in-tree with hipcc.

Each source is compiled to an object of its own, in parallel, under _build/ (ignored by
git), and the objects are linked into paper_2505_00387_amd/libaahrt.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'libaahrt.so')
OBJ_DIR = os.path.join(os.path.dirname(HERE), '_build')

SOURCES = ['plan.cpp', 'rows.hip', 'gfst_sweep.hip', 'gfst_res.hip', 'misc.hip', 'noalloc.hip']
FLAGS = [
    '-O3', '-std=c++17', '-fPIC', '--offload-arch=gfx950',
    # packed FP32 instructions are kept out of every kernel
    '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
    '-munsafe-fp-atomics', '-Wall', '-Wno-unused-function',
]


def hipcc() -> str:
    for cand in (shutil.which('hipcc'), '/opt/rocm/bin/hipcc'):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError('hipcc not found')


def _run(cmd, verbose):
    if verbose:
        print(' '.join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError('hipcc failed: ' + ' '.join(cmd[-3:]))
    return r


def build(verbose: bool = False, extra=None, jobs: int = 0) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    cmds = []
    for s in SOURCES:
        obj = os.path.join(OBJ_DIR, os.path.splitext(s)[0] + '.o')
        objs.append(obj)
        cmds.append([cc] + FLAGS + list(extra or []) + ['-c', os.path.join(CSRC, s), '-o', obj])
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + '.tmp'
    _run([cc, '-shared', '-fPIC', '--offload-arch=gfx950'] + objs + ['-o', tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose=True))
