"""The C-ABI library loads on the host and exports every function include/*.h
declares (no compute calls: there may be no GPU here)."""
import ctypes
import glob
import os
import re

from paper_2001_01570_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, 'include', '*.h')):
        text = open(h).read()
        text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
        for m in re.finditer(r'^\s*(?:const\s+)?[a-z_][a-z0-9_ ]*\s*\**\s*(cgks_[a-z0-9_]+)\s*\(', text, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ('cgks_create', 'cgks_set_state', 'cgks_step', 'cgks_advance_to', 'cgks_get_state', 'cgks_destroy',
              'cgks_batch_create', 'cgks_batch_admit', 'cgks_batch_run', 'cgks_batch_poll', 'cgks_batch_read',
              'cgks_batch_release', 'cgks_batch_destroy'):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(B.LIB):
        B.build()
    lib = ctypes.CDLL(B.LIB)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_is_host_only_and_total():
    if not os.path.exists(B.LIB):
        B.build()
    lib = ctypes.CDLL(B.LIB)
    lib.cgks_strerror.restype = ctypes.c_char_p
    for code in range(-7, 1):
        assert lib.cgks_strerror(code)


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        return
    from paper_2001_01570_amd.cgks import Solver
    from paper_2001_01570_amd import inputs as I
    try:
        Solver(I.sine_wave_1d(8))
    except RuntimeError as e:
        assert 'GPU' in str(e)
    else:
        raise AssertionError('the HIP binding must not run without a GPU')
