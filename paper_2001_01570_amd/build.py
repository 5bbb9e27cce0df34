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


FLOPS_JSON = os.path.join(PKG, 'flops.json')


def code_tokens(text: str) -> str:
    """C/C++ source with comments removed and whitespace runs collapsed (string
    and character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in '"\'':
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == '\\' else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith('//', i):
            j = text.find('\n', i)
            i = n if j < 0 else j
        elif text.startswith('/*', i):
            j = text.find('*/', i + 2)
            i = n if j < 0 else j + 2
            out.append(' ')
        else:
            out.append(c)
            i += 1
    return ' '.join(''.join(out).split())


def source_digest() -> str:
    """Digest of the code of the HIP sources (comments and layout excluded):
    measured or tuned figures are valid only for the kernels they were taken
    on."""
    import hashlib
    h = hashlib.sha256()
    for path in (os.path.join(PKG, 'csrc', 'cgks.hip'), os.path.join(PKG, 'csrc', 'cgks_device.h')):
        with open(path, encoding='utf-8') as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]
OPCOUNT_SRC = os.path.join(PKG, 'csrc', 'opcount.cpp')


def count_operations(verbose: bool = False) -> str:
    """Compile the device arithmetic for the host with a counting scalar and
    write the algorithmic operation counts per unit to flops.json."""
    exe = os.path.join(PKG, 'csrc', 'opcount.bin')
    cmd = ['g++', '-std=c++17', '-O1', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include', '-I',
           os.path.join(PKG, 'csrc'), '-I', os.path.join(ROOT, 'include'), OPCOUNT_SRC, '-o', exe]
    if verbose:
        print(' '.join(cmd), file=sys.stderr, flush=True)
    subprocess.check_call(cmd)
    out = subprocess.check_output([exe])
    os.remove(exe)
    with open(FLOPS_JSON + '.tmp', 'wb') as f:
        f.write(out)
    os.replace(FLOPS_JSON + '.tmp', FLOPS_JSON)
    return FLOPS_JSON


RUN_SRC = os.path.join(PKG, 'csrc', 'cgks_run.c')
RUN_EXE = os.path.join(PKG, 'cgks_run')


def build_driver(verbose: bool = False) -> str:
    """Compile cgks_run, the plain-C driver of the C ABI, against libcgks.so."""
    cmd = ['gcc', '-std=c11', '-O2', '-Wall', '-I', os.path.join(ROOT, 'include'), RUN_SRC, '-L', PKG, '-lcgks',
           '-Wl,-rpath,$ORIGIN', '-Wl,-rpath,/opt/rocm/lib', '-o', RUN_EXE + '.tmp']
    if verbose:
        print(' '.join(cmd), file=sys.stderr, flush=True)
    subprocess.check_call(cmd)
    os.replace(RUN_EXE + '.tmp', RUN_EXE)
    return RUN_EXE


def build(verbose: bool = False, extra=(), out: str = None) -> str:
    """Compile libcgks.so (out: alternative path, used for tuning variants)."""
    target = out or LIB
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + ['-I', os.path.join(ROOT, 'include'), '-I',
                                                    os.path.join(PKG, 'csrc')] + SRC + ['-o', target + '.tmp']
    if verbose:
        print(' '.join(cmd), file=sys.stderr, flush=True)
    subprocess.check_call(cmd)
    os.replace(target + '.tmp', target)
    if out is None:
        count_operations(verbose)
        build_driver(verbose)
    return target


if __name__ == '__main__':
    build(verbose=True, extra=sys.argv[1:])
