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


def test_create_rejects_invalid_configurations_before_touching_the_device():
    """cgks_create validates the configuration first and returns CGKS_EINVAL
    (no device call is made for a rejected configuration)."""
    import dataclasses
    from paper_2001_01570_amd import inputs as I
    from paper_2001_01570_amd.cgks import make_config, CGKS_FP32_STORAGE
    if not os.path.exists(B.LIB):
        B.build()
    lib = ctypes.CDLL(B.LIB)
    lib.cgks_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    EINVAL = -1
    base = I.acoustic_pulse_2d(8, seed=1)

    def rc(prob, storage=0, **fix):
        cfg = make_config(prob, storage)
        for k, v in fix.items():
            if k == 'bc':
                for s in range(4):
                    cfg.bc[s] = v[s]
            else:
                setattr(cfg, k, v)
        h = ctypes.c_void_p()
        r = lib.cgks_create(ctypes.addressof(cfg), None, ctypes.byref(h))
        assert not h.value
        return r

    assert rc(base, nx=0) == EINVAL
    assert rc(base, gauss_points=3) == EINVAL                       # two or four points only
    assert rc(I.sine_wave_1d(16), gauss_points=4) == EINVAL         # 2D only
    assert rc(I.uniform_2d(2, 8, bc=(I.WALL,) * 4), gauss_points=4) == EINVAL   # walls: 3 cells across
    assert rc(base, ny=0) == EINVAL
    assert rc(base, dim=3) == EINVAL
    assert rc(base, nx=65536, ny=65536) == EINVAL                 # beyond the index range
    assert rc(base, gamma=1.0) == EINVAL
    assert rc(base, x1=-1.0) == EINVAL
    assert rc(base, cfl=0.0, fixed_dt=0.0) == EINVAL
    assert rc(base, weno_eps=0.0) == EINVAL
    assert rc(base, tau_eps=0.0) == EINVAL
    assert rc(base, tau_C=-1.0) == EINVAL
    assert rc(base, mu=-1e-3) == EINVAL
    assert rc(base, mu=float('nan')) == EINVAL
    assert rc(base, bc=(5, 5, 0, 0)) == EINVAL                    # unknown boundary kind
    assert rc(base, bc=(0, 1, 0, 0)) == EINVAL                    # periodic on one side only
    assert rc(base, storage=7) == EINVAL
    assert rc(base, recon_vars=2) == EINVAL                       # conservative or characteristic
    assert rc(base, recon_vars=-1) == EINVAL
    assert rc(base, side_slopes=1) != EINVAL                      # the side-slope variant: 1D and 2D
    assert rc(dataclasses.replace(base, gauss_points=4), side_slopes=1) != EINVAL
    assert rc(base, side_slopes=1, recon_vars=1) == EINVAL
    assert rc(base, tang_weno=1) != EINVAL                        # the tangential-WENO variant: 2D
    assert rc(base, tang_weno=2) == EINVAL
    assert rc(dataclasses.replace(base, gauss_points=4), tang_weno=1) != EINVAL
    assert rc(base, tang_weno=1, recon_vars=1) == EINVAL
    assert rc(base, tang_weno=1, side_slopes=1) == EINVAL
    assert rc(I.sine_wave_1d(16), tang_weno=1) == EINVAL
    assert rc(I.sine_wave_1d(16), side_slopes=2) == EINVAL
    assert rc(I.sine_wave_1d(16), side_slopes=1, recon_vars=1) == EINVAL
    assert rc(I.sine_wave_1d(8), storage=CGKS_FP32_STORAGE) == EINVAL   # FP32 storage is 2D only
    walled = dataclasses.replace(base, bc=(I.WALL, I.WALL, I.NOSLIP, I.NOSLIP))
    assert rc(walled, nx=1) == EINVAL                             # a wall needs 2 cells to mirror
    assert rc(walled, ny=1) == EINVAL
    inflow = dataclasses.replace(base, bc=(I.INFLOW, I.FREE, I.PERIODIC, I.PERIODIC),
                                 inflow_prim=((-1.0, 0.0, 0.0, 1.0),) + ((1.0, 0.0, 0.0, 1.0),) * 3)
    assert rc(inflow) == EINVAL                                   # non-physical inflow state
