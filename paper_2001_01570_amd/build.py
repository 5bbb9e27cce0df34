"""Build the HIP library libcgks.so in-tree for gfx950 (hipcc)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, 'libcgks.so')
SRC = [os.path.join(PKG, 'csrc', 'cgks.hip')]
HEADERS = [os.path.join(PKG, 'csrc', 'cgks_device.h'), os.path.join(ROOT, 'include', 'cgks.h')]

HIPCC_FLAGS = [
    '--offload-arch=gfx950', '-O3', '-std=c++17', '-fPIC', '-shared',
    # no packed FP32 instructions anywhere in the device code
    '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
]


def hipcc() -> str:
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', 'hipcc'):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return 'hipcc'


def build(verbose: bool = False, extra=()) -> str:
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + ['-I', os.path.join(ROOT, 'include'), '-I',
                                                    os.path.join(PKG, 'csrc')] + SRC + ['-o', LIB + '.tmp']
    if verbose:
        print(' '.join(cmd), file=sys.stderr, flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + '.tmp', LIB)
    return LIB


if __name__ == '__main__':
    build(verbose=True, extra=sys.argv[1:])
