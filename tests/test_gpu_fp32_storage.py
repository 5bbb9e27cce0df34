"""FP32 storage of the cell-averaged gradients (2D): averages, arithmetic and
accumulation stay FP64.  The round trip rounds only the gradients; one step
and many steps stay within stated bounds of the FP64 path (itself pinned to
the oracle at 1e-12), measured relative to the perturbation amplitude."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_to_amplitude(a, b, amp):
    """max |a - b| per field group, relative to the perturbation amplitude
    (gradients scaled by the cell width, i.e. as differences across a cell)"""
    return np.abs(a - b).reshape(12, -1).max(axis=1) / amp


def test_round_trip_rounds_only_the_gradients():
    from paper_2001_01570_amd.cgks import Solver, CGKS_FP32_STORAGE
    p = I.acoustic_pulse_2d(40, seed=2, amp=1e-3, half_width=0.2, ny=24)
    s = Solver(p, storage=CGKS_FP32_STORAGE)
    g = s.get_state()[0]
    assert np.array_equal(g[:4], p.fields[:4])
    assert np.array_equal(g[4:], p.fields[4:].astype(np.float32).astype(np.float64))


def _viscous_box():
    p = I.acoustic_pulse_2d(40, seed=4, amp=0.05, half_width=0.3, ny=24)
    p.fields[1] += 0.2 * p.fields[0]
    p.fields[3] += 0.02 * p.fields[0]
    p.fields[5] += 0.2 * p.fields[4]
    p.fields[9] += 0.2 * p.fields[8]
    return dataclasses.replace(p, mu=0.01, bc=(I.NOSLIP,) * 4)


@pytest.mark.parametrize('mk,amp', [(lambda: I.acoustic_pulse_2d(64, seed=3, amp=1e-3, half_width=0.2), 1e-3),
                                    (lambda: I.shock_vortex_2d(64, 32, Rc=0.12), 0.3),
                                    (_viscous_box, 0.125),    # its largest perturbation (energy)
                                    (lambda: dataclasses.replace(I.acoustic_pulse_2d(64, seed=3, amp=1e-3,
                                                                                     half_width=0.2),
                                                                 gauss_points=4), 1e-3),
                                    (lambda: dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12),
                                                                 gauss_points=4), 0.3)],
                         ids=['pulse', 'shock_vortex', 'viscous_noslip', 'pulse_four_points',
                              'shock_vortex_four_points'])
def test_fp32_storage_error_against_fp64(mk, amp):
    from paper_2001_01570_amd.cgks import Solver, CGKS_FP32_STORAGE
    p = mk()
    dx = p.dx
    a = Solver(p)
    b = Solver(p, storage=CGKS_FP32_STORAGE)
    o = O.Oracle(p, threads=8)
    dt = a.step()
    b.step(dt)
    o.step(dt)
    one = rel_to_amplitude(b.state, o.state, amp)
    one[4:] *= dx
    say('one step, FP32 storage vs oracle / amplitude:', one)
    assert one[:4].max() < 1e-6 and one[4:].max() < 1e-6
    a.run_steps(49)
    b.run_steps(49)
    many = rel_to_amplitude(b.state, a.state, amp)
    many[4:] *= dx
    say('50 steps, FP32 storage vs FP64 / amplitude:', many)
    assert many.max() < 1e-4
