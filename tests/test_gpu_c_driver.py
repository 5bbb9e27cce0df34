"""The C ABI used from plain C: cgks_run (paper_2001_01570_amd/csrc/cgks_run.c,
no Python and no torch, the null stream, default tile shapes) advances a
state from a raw file; the result is bitwise the Python binding's."""
import dataclasses
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2001_01570_amd import build as B
from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


def write_config(prob, path):
    d = prob.config_dict()
    vals = [d['dim'], d['nx'], d['ny'], d['x0'], d['x1'], d['y0'], d['y1'], d['gamma'], d['cfl']] + list(d['bc'])
    vals += [v for side in d['inflow_prim'] for v in side]
    vals += [d['weno_eps'], d['tau_eps'], d['tau_C'], d['fixed_dt'], d['mu'], d['gauss_points'], d['recon_vars'],
             d['side_slopes'], d['tang_weno']]
    with open(path, 'w') as f:
        f.write(' '.join(repr(float(v)) if isinstance(v, float) else str(v) for v in vals) + '\n')


@pytest.mark.parametrize('name,mk,steps', [
    ('pulse_2d', lambda: I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21), 30),
    ('shock_vortex_2d', lambda: I.shock_vortex_2d(64, 32, Rc=0.12), 12),
    ('shock_entropy_1d', lambda: I.shock_entropy_1d(400), 40),
    ('diagonal_4_points', lambda: dataclasses.replace(I.diagonal_wave_2d(24), gauss_points=4), 10),
    ('shock_vortex_characteristic', lambda: dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), recon_vars=1), 12),
    ('shock_tube_side_slopes', lambda: dataclasses.replace(I.shock_tube_1d(100), side_slopes=1), 30),
    ('shock_vortex_side_slopes', lambda: dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), side_slopes=1), 12),
    ('shock_vortex_tang_weno', lambda: dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), tang_weno=1), 12),
])
def test_c_driver_equals_the_binding(tmp_path, name, mk, steps):
    from paper_2001_01570_amd.cgks import Solver
    assert os.path.exists(B.RUN_EXE), 'build the library first (it builds cgks_run)'
    p = mk()
    cfg, sin, sout = tmp_path / 'cfg.txt', tmp_path / 'in.bin', tmp_path / 'out.bin'
    write_config(p, cfg)
    np.ascontiguousarray(p.fields, dtype=np.float64).tofile(sin)
    r = subprocess.run([B.RUN_EXE, str(cfg), str(sin), str(steps), str(sout)], capture_output=True, text=True,
                       timeout=120)
    print(name, r.stdout.strip(), r.stderr.strip(), file=sys.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    c = np.fromfile(sout, dtype=np.float64).reshape(p.fields.shape)
    s = Solver(p)
    s.run_steps(steps)
    g, t, n = s.get_state()
    assert n == steps and r.stdout.split()[3] == str(steps)
    assert float(r.stdout.split()[1]) == t
    assert np.array_equal(c, g)


def test_c_driver_reports_library_errors(tmp_path):
    p = I.acoustic_pulse_2d(16, seed=1, amp=0.05, half_width=0.3)
    bad = p.fields.copy()
    bad[0, 2, 3] = -1.0                      # a non-physical cell: set_state refuses it
    cfg, sin, sout = tmp_path / 'cfg.txt', tmp_path / 'in.bin', tmp_path / 'out.bin'
    write_config(p, cfg)
    bad.tofile(sin)
    r = subprocess.run([B.RUN_EXE, str(cfg), str(sin), '3', str(sout)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and 'non-physical' in r.stderr
