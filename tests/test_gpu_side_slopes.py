"""The evaluated side-slope variant (side_slopes = 1; 1D, and 2D with two
or four Gauss points): the two non-equilibrium sides take the WENO-weighted
slopes of their candidate polynomials instead of the linear
reconstruction's derivative (in 2D each line's slopes taken to the Gauss
point like the normal derivative).  The HIP path against the oracle with the same option:
single steps (smooth flow, the Sec. 4.4 shock tube, a pressure-ratio-300
tube where the guards fire; 2D shock-vortex with walls and inflow, a
near-vacuum expansion, no-slip walls, FP32 gradient storage), whole runs
with each side's own steps, runs where the guards fire, and a
pressure-ratio-800 tube that only this variant carries to its end time."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I
from tests.parity import field_errors, field_scales, scaled_errors
from tests.test_gpu_parity_runs import _guard_case, own_dt_run

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def side(p):
    return dataclasses.replace(p, side_slopes=1)


# (name, problem, steps before, smallest change against the linear side slopes:
# in smooth flow the WENO-weighted slopes approach the linear derivative and
# enter with a weight of about tau/dt, so one step moves by rounding size)
CASES = [
    ('smooth_wave', lambda: I.sine_wave_1d(100, eps=0.2, t_end=2.0, cfl=0.3), 0, 1e-15),
    ('shock_tube', lambda: I.shock_tube_1d(100), 6, 1e-10),
    ('pressure_ratio_300', lambda: I.riemann_1d((1.0, 0.0, 30.0), (0.125, 0.0, 0.1), 100), 3, 1e-10),
    ('shock_entropy_inflow', lambda: I.shock_entropy_1d(400, t_end=1.8), 4, 1e-10),
]


@pytest.mark.parametrize('name,mk,before,min_change', CASES, ids=[c[0] for c in CASES])
def test_single_step(name, mk, before, min_change):
    """One step from the oracle's state after `before` steps: within 1e-12 of
    the oracle's step with the same option, and different from the step
    with the linear side slopes (the option is in effect)."""
    from paper_2001_01570_amd.cgks import Solver
    p = side(mk())
    o = O.Oracle(p)
    for _ in range(before):
        o.step()
    st, t, _ = o.get_state()
    s = Solver(p)
    s.set_state(st, t)
    dt = s.step()
    o.step(dt)
    r = Solver(dataclasses.replace(p, side_slopes=0))
    r.set_state(st, t)
    r.step(dt)
    e = field_errors(s.state, o.state)
    change = (np.abs(s.state - r.state).max(axis=1) / field_scales(o.state)).max()
    say(name, 'errors', e.max(), 'change against the linear side slopes', change)
    assert e.max() < TOL, e
    assert change > min_change


def test_shock_tube_whole_run_each_side_its_own_dt():
    p = side(I.shock_tube_1d(100))
    s, o, _ = own_dt_run(p, t_end=0.16, threads=1)
    err = scaled_errors(s.state, o.state, p.dx)
    say('side slopes, shock tube to t = 0.16:', o.counters()['steps'], 'steps, scaled errors', err)
    assert s.t == o.t == 0.16
    assert err.max() < TOL, err


def test_table1_row_12_with_the_variant():
    """Table 1's N = 12 run (14,400 steps of dt = 0.5 dx^2 to t = 200): the
    GPU run agrees with the oracle's to the rounding of that many steps, and
    both land on the variant's own error (above the printed R3 value)."""
    from paper_2001_01570_amd.cgks import Solver
    n = 12
    dx = 2.0 / n
    p = side(I.sine_wave_1d(n, eps=1e-4, t_end=200.0, fixed_dt=0.5 * dx * dx))
    s, o = Solver(p), O.Oracle(p, threads=1)
    assert s.advance_to(200.0) == o.advance_to(200.0)
    d = np.abs(s.state[0] - o.state[0]).max()
    eg, eo = I.density_errors(s.state, p.exact(200.0)), I.density_errors(o.state, p.exact(200.0))
    say('side slopes, Table 1 N = 12: GPU', eg, 'oracle', eo, 'max density difference', d)
    assert d < 1e-12 * 1e-4 * 1e3
    assert eg[0] == pytest.approx(eo[0], rel=1e-6)


@pytest.mark.parametrize('pr', [300.0, 800.0])
def test_strong_tubes_guard_counts_and_states(pr):
    """Pressure ratios 300 and 800 (Sod-like, t = 0.1 / sqrt(p_L)): step by
    step and over the run, the guard counts equal the oracle's and the
    states meet the parity bar (or, near a vacuum, 3x the oracle's own
    1-ulp spread)."""
    L, R = (1.0, 0.0, pr / 10.0), (0.125, 0.0, 0.1)
    t_end = 0.1 / math.sqrt(pr / 10.0)
    _guard_case(side(I.riemann_1d(L, R, 100, t_end=t_end)), t_end=t_end, min_w0=0, min_weno=0)


def moving_pulse():
    p = I.acoustic_pulse_2d(40, seed=4, amp=0.05, half_width=0.3, ny=24)
    f = p.fields
    f[1] += 0.2 * f[0]
    f[2] += 0.1 * f[0]
    f[3] += 0.5 * 0.05 * f[0]
    return p


CASES_2D = [
    ('shock_vortex_walls_inflow', lambda: I.shock_vortex_2d(64, 32, Rc=0.12), 3, 1e-10),
    ('expansion_near_vacuum', lambda: I.expansion_2d(32, 28, U=1.25, amp=0.1), 2, 1e-10),
    ('viscous_shock_vortex_noslip', lambda: dataclasses.replace(I.shock_vortex_2d(48, 24, Rc=0.12), mu=1e-3,
                                                                bc=(I.INFLOW, I.FREE, I.NOSLIP, I.NOSLIP)), 2, 1e-10),
    ('moving_pulse_noslip', lambda: dataclasses.replace(moving_pulse(), bc=(I.NOSLIP,) * 4), 0, 1e-15),
]


def _step_pair_2d(p, before, storage=0):
    from paper_2001_01570_amd.cgks import Solver
    o = O.Oracle(p, threads=8)
    for _ in range(before):
        o.step()
    st, t, _ = o.get_state()
    if storage:
        st[4:] = st[4:].astype(np.float32).astype(np.float64)
        o.set_state(st, t)
    s = Solver(p, storage=storage)
    s.set_state(st, t)
    dt = s.step()
    o.step(dt)
    r = Solver(dataclasses.replace(p, side_slopes=0), storage=storage)
    r.set_state(st, t)
    r.step(dt)
    e = field_errors(s.state, o.state)
    change = (np.abs(s.state - r.state).reshape(12, -1).max(axis=1) / field_scales(o.state)).max()
    return e, change


@pytest.mark.parametrize('gp', [2, 4])
@pytest.mark.parametrize('name,mk,before,min_change', CASES_2D, ids=[c[0] for c in CASES_2D])
def test_2d_single_step(name, mk, before, min_change, gp):
    """2D, two and four Gauss points: one step from the oracle's state after
    `before` steps, within 1e-12 of the oracle's step with the same option,
    and different from the step with the linear side slopes."""
    p = side(dataclasses.replace(mk(), gauss_points=gp))
    say('2d side slopes single step', name, p.nx, p.ny, 'gauss points', gp)
    e, change = _step_pair_2d(p, before)
    say(name, 'errors', e.max(), 'change against the linear side slopes', change)
    assert e.max() < TOL, e
    assert change > min_change


@pytest.mark.parametrize('gp', [2, 4])
def test_2d_fp32_storage_single_step(gp):
    """FP32 gradient storage: the averages within 1e-8 of their field scale,
    the gradients within their FP32 rounding (as for the other options)."""
    from paper_2001_01570_amd.cgks import CGKS_FP32_STORAGE
    p = side(dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp))
    e, change = _step_pair_2d(p, 3, CGKS_FP32_STORAGE)
    say('2d side slopes, fp32 storage: averages', e[:4].max(), 'gradients', e[4:].max(), 'change', change)
    assert e[:4].max() < 1e-8, e
    assert e[4:].max() < 4 * 2.0 ** -24, e
    assert change > 1e-10


@pytest.mark.parametrize('gp', [2, 4])
def test_2d_forty_steps_each_side_its_own_dt(gp):
    p = side(dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp))
    s, o, rel = own_dt_run(p, steps=40)
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    say('2d side slopes, 40 steps: dt rel', rel.max(), 'scaled errors', err)
    assert rel.max() < 1e-13
    assert err.max() < TOL, err


def test_2d_guards_fire_with_the_variant():
    """The curved expansion to near-vacuum: both fallbacks fire (a side that
    falls back to its cell average takes the linear slope); guard counts
    equal the oracle's step by step and over the run."""
    _guard_case(side(I.expansion_2d(32, 28, U=1.25, amp=0.1)), steps=12, min_w0=1, min_weno=1)
    _guard_case(side(I.expansion_2d(32, 28, U=1.25, amp=0.1, gauss_points=4)), steps=8, min_w0=1, min_weno=1)


def test_batch_side_slope_kinds_equal_separate_contexts():
    """Side-slope slots of every Gauss-point count and storage next to
    conservative and characteristic ones in one batch: bitwise equal to
    separate contexts on every replay, and a side-slope slot within 1e-12 of
    the oracle."""
    from paper_2001_01570_amd.cgks import Batch, CGKS_FP32_STORAGE, Solver
    g4 = lambda p: dataclasses.replace(p, gauss_points=4)
    kinds = [(side(I.shock_vortex_2d(64, 32, Rc=0.12)), 0),
             (side(g4(I.shock_vortex_2d(40, 24, Rc=0.12))), 0),
             (side(I.expansion_2d(32, 28, U=1.0, amp=0.1)), CGKS_FP32_STORAGE),
             (side(g4(dataclasses.replace(moving_pulse(), bc=(I.NOSLIP,) * 4))), CGKS_FP32_STORAGE),
             (I.shock_vortex_2d(64, 32, Rc=0.12), 0),
             (dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), recon_vars=1), 0)]
    b = Batch(1 << 30, max_slots=8)
    slots = [b.admit_storage(p, st, max_steps=6) for p, st in kinds]
    refs = [Solver(p, storage=st) for p, st in kinds]
    for rnd in range(2):
        b.run(3)
        for r in refs:
            r.run_steps(3)
        for (p, st), s, r in zip(kinds, slots, refs):
            g = b.read(s)
            e, te, ne = r.get_state()
            assert b.poll(s)[2] == ne == 3 * (rnd + 1)
            assert np.array_equal(g, e), (p.name, p.gauss_points, st, rnd, np.abs(g - e).max())
    assert np.abs(b.read(slots[0]) - b.read(slots[4])).max() > 1e-8
    b.close()
    p = kinds[0][0]
    o = O.Oracle(p, threads=8)
    b = Batch(1 << 28, max_slots=2)
    s = b.admit(p, max_steps=1)
    b.run(1)
    o.step(b.poll(s)[1])
    e = field_errors(b.read(s), o.state)
    say('side-slope batch slot vs oracle', e.max())
    assert e.max() < TOL
    b.close()


@pytest.mark.parametrize('gp', [2, 4])
def test_guards_fire_next_to_noslip_walls(gp):
    """The flow leaves every no-slip wall (the 2D expansion with velocity 1.0
    towards the curve): both fallbacks fire along the walls (the WENO
    fallback takes the cells beside the face through the boundary rule);
    guard counts and states follow the oracle step by step and over 30
    steps."""
    p = side(dataclasses.replace(I.expansion_2d(32, 28, U=-1.0, amp=0.1, gauss_points=gp), bc=(I.NOSLIP,) * 4))
    _guard_case(p, steps=30, min_w0=1, min_weno=1)
