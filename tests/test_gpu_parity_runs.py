"""Parity of whole runs (each side choosing its own time steps) and of runs in
which the positivity guards fire; the GPU path against the paper's accuracy
tables at resolutions the oracle needs minutes for."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I
from tests.conftest import golden
from tests.parity import field_errors, scaled_errors

pytestmark = pytest.mark.gpu

TOL = 1e-12


def solver(prob):
    from paper_2001_01570_amd.cgks import Solver
    return Solver(prob)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def own_dt_run(p, steps=None, t_end=None, threads=8):
    """Both sides advance with their own CFL steps (advance_to, last step
    clamped) for `steps` steps or to t_end; returns GPU and oracle solvers
    and the per-step relative differences of the step sizes."""
    s, o = solver(p), O.Oracle(p, threads=threads)
    if t_end is not None:
        ns, no = s.advance_to(t_end), o.advance_to(t_end)
        assert ns == no, (ns, no)
        return s, o, None
    rel = []
    for _ in range(steps):
        assert s.advance_to(1e30, 1) == 1 and o.advance_to(1e30, 1) == 1
        dg, do = s.counters()['last_dt'], o.counters()['last_dt']
        rel.append(abs(dg - do) / do)
    return s, o, np.array(rel)


# ---------------------------------------------------------------- runs with their own time steps

RUNS_2D = [
    ('pulse_periodic', lambda: I.acoustic_pulse_2d(48, seed=6, amp=1e-2, half_width=0.25, ny=40)),
    ('shock_vortex_walls_inflow', lambda: I.shock_vortex_2d(64, 32, Rc=0.12)),
]


@pytest.mark.parametrize('gp', [2, 4])
@pytest.mark.parametrize('name,mk', RUNS_2D, ids=[r[0] for r in RUNS_2D])
def test_2d_hundred_steps_each_side_its_own_dt(name, mk, gp):
    """100 CFL steps with each side's own reduction: the step sizes agree to
    a few ulp of rounding of the states (bound 1e-13 relative: the CFL
    maximum is exact, the per-cell (|U| + c)/dx differs by the states'
    rounding), the times agree, and the states meet the multi-step bar."""
    p = dataclasses.replace(mk(), gauss_points=gp)
    say('own-dt run', name, p.nx, p.ny, 'gauss points', gp)
    s, o, rel = own_dt_run(p, steps=100)
    say(name, gp, 'max relative dt difference', rel.max(), 'first', rel[0])
    assert rel[0] < 4e-16, rel[0]
    assert rel.max() < 1e-13, rel.max()
    assert s.t == pytest.approx(o.t, rel=1e-13)
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    say(name, gp, '100-step scaled errors', err)
    assert err.max() < TOL, err


@pytest.mark.parametrize('gp', [2, 4])
def test_2d_advance_to_lands_on_the_same_step_count(gp):
    p = dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp)
    o0 = O.Oracle(p)
    t_end = 60.5 * o0.cfl_dt()
    s, o, _ = own_dt_run(p, t_end=t_end)
    assert s.t == o.t == t_end
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    say('advance_to', gp, 'steps', o.counters()['steps'], 'scaled errors', err)
    assert err.max() < TOL, err


# ---------------------------------------------------------------- the positivity guards

def _oracle_spread(p, steps=None, t_end=None, trials=4):
    """The oracle's own conditioning: the largest multi-step difference
    between its run and runs from inputs moved by +-1 ulp (random signs)."""
    o = O.Oracle(p, threads=8)
    o.advance_to(t_end) if t_end is not None else o.advance_to(1e30, steps)
    ref = o.state
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(trials):
        f = p.fields * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=p.fields.shape))
        q = O.Oracle(dataclasses.replace(p, fields=f), threads=8)
        q.advance_to(t_end) if t_end is not None else q.advance_to(1e30, steps)
        worst = max(worst, scaled_errors(q.state, ref, p.dx, p.dy).max())
    return worst


def _oracle_step_spread(p, st, t, dt, ref, trials=4):
    """The oracle's own conditioning of one step: the largest single-step
    difference between its step from st and steps from st moved by +-1 ulp."""
    rng = np.random.default_rng(13)
    worst = 0.0
    for _ in range(trials):
        f = st * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=st.shape))
        q = O.Oracle(p, threads=8)
        q.set_state(f, t)
        q.step(dt)
        worst = max(worst, field_errors(q.state, ref).max())
    return worst


def _guard_case(p, steps=None, t_end=None, min_w0=1, min_weno=1):
    """(1) Every step of the run from identical input: the step's guard
    counts are equal and every field is within 1e-12 (single-step metric),
    or, on the few steps where a fallback near a vacuum makes the step itself
    that sensitive, within 3x the oracle's own single-step spread under
    1-ulp input changes (measured at that state and printed).
    (2) The whole run with each side's own steps: equal step and guard
    counts; the states within 1e-12, or within 3x the oracle's own spread
    under 1-ulp input changes where fallbacks near a vacuum make the run
    that sensitive (the spread is measured and printed)."""
    s, o = solver(p), O.Oracle(p, threads=8)
    n = 0
    while (steps is None or n < steps) and (t_end is None or o.t < t_end):
        st, t, _ = o.get_state()
        s.set_state(st, t)
        g0, c0 = s.counters(), o.counters()
        assert o.advance_to(t_end if t_end is not None else 1e30, 1) == 1
        dt = o.counters()['last_dt']
        s.step(dt)
        g1, c1 = s.counters(), o.counters()
        for k in ('guard_w0', 'guard_weno'):
            assert g1[k] - g0[k] == c1[k] - c0[k], (n, k, g1[k] - g0[k], c1[k] - c0[k])
        e = field_errors(s.state, o.state)
        if e.max() >= TOL:
            spread = _oracle_step_spread(p, st, t, dt, o.state)
            say(p.name, 'step', n, 'single-step error', e.max(), "oracle's 1-ulp single-step spread", spread)
            assert e.max() < 3.0 * spread, (n, e, spread)
        n += 1
    s, o, _ = own_dt_run(p, steps=steps, t_end=t_end)
    cs, co = s.counters(), o.counters()
    say(p.name, 'steps', n, 'guards GPU', cs['guard_w0'], cs['guard_weno'], 'oracle', co['guard_w0'], co['guard_weno'])
    assert co['guard_w0'] >= min_w0 and co['guard_weno'] >= min_weno, co
    assert cs['guard_w0'] == co['guard_w0'] and cs['guard_weno'] == co['guard_weno']
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    say(p.name, 'whole-run scaled errors', err)
    if err.max() >= TOL:
        spread = _oracle_spread(p, steps, t_end)
        say(p.name, "oracle's 1-ulp spread", spread)
        assert err.max() < 3.0 * spread, (err, spread)


def test_1d_guards_strong_expansion():
    """Double rarefaction to near-vacuum plus colliding streams (U = 1.5
    against c = 0.75): both guards fire; counts equal.  Near the vacuum a
    step is ill-conditioned: from the state after 15 steps the oracle's own
    single-step spread under 1-ulp input changes is 5e-12..1e-11, and over
    the whole run (38 steps) ~1e-11; the GPU stays inside both."""
    _guard_case(I.expansion_1d(100, 1.5), t_end=0.05, min_w0=30, min_weno=4)


def test_1d_guards_stronger_expansion_twelve_steps():
    _guard_case(I.expansion_1d(100, 1.75), steps=12, min_w0=30, min_weno=10)


def test_1d_guards_pressure_ratio_300_tube():
    L, R = (1.0, 0.0, 30.0), (0.125, 0.0, 0.1)
    t_end = 0.1 / math.sqrt(30.0)
    _guard_case(I.riemann_1d(L, R, 100, t_end=t_end), t_end=t_end, min_w0=60, min_weno=1)


@pytest.mark.parametrize('gp', [2, 4])
def test_2d_guards_curved_expansion(gp):
    """The expansion across the curve x = 1/2 + 0.1 sin 2 pi y on a ragged
    grid: hundreds of equilibrium and WENO fallbacks over 30 steps."""
    p = I.expansion_2d(32, 28, U=1.25, amp=0.1, gauss_points=gp)
    _guard_case(p, steps=30, min_w0=100, min_weno=100)


# ---------------------------------------------------------------- the paper's accuracy tables on the GPU path

def _table_run(n, mode):
    dx = 2.0 / n
    if mode == 'dt':
        p = I.sine_wave_1d(n, eps=1e-4, t_end=200.0, fixed_dt=0.5 * dx * dx)
    else:
        p = I.sine_wave_1d(n, eps=1e-4, t_end=200.0, cfl=0.8)
    s = solver(p)
    s.advance_to(200.0)
    st, t, _ = s.get_state()
    assert t == 200.0
    assert s.counters()['guard_w0'] == 0
    return I.density_errors(st, p.exact(t)), s


def test_table3_rows_96_and_192_on_the_gpu_path():
    """Table 3 (CFL 0.8, t = 200) at N = 96 and 192 (26,200 and 52,399
    steps): L1 and L2 within 1 % of the printed values, Linf within 3 %
    (the oracle's Linf at N = 192 is 1.7 % below the printed one), order 4.00; at
    N = 96 the oracle's own run (26 s on one core) agrees with the GPU's to
    the rounding of 26,200 steps."""
    rows = {int(r[0]): r[1:] for r in golden('table3_compact8_cfl08.txt')}
    errs = {}
    for n in (96, 192):
        errs[n], s = _table_run(n, 'cfl')
        say('table 3 N=%d' % n, errs[n], 'paper', rows[n])
        for e, ref, tol in zip(errs[n], rows[n], (0.01, 0.01, 0.03)):
            assert abs(e / ref - 1.0) < tol, (n, e, ref)
        if n == 96:
            p = I.sine_wave_1d(96, eps=1e-4, t_end=200.0, cfl=0.8)
            o = O.Oracle(p, threads=1)
            assert o.advance_to(200.0) == s.counters()['steps']
            d = np.abs(o.state[0] - s.state[0]).max()
            say('N=96 GPU - oracle density', d)
            assert d < 1e-12 * 1e-4 * 1e3     # 1e-3 of the perturbation's 1e-12 bar per step, over 26,200 steps
    assert math.log2(errs[96][0] / errs[192][0]) == pytest.approx(4.0, abs=0.02)


def test_table1_row_48_on_the_gpu_path():
    """Table 1 (dt = 0.5 dx^2, t = 200) at N = 48: 230,401 steps.  The printed
    L1 6.44e-14 of a 1e-4 wave is at the rounding floor of that many steps
    (its order 8.6 exceeds the scheme's 8); both implementations land at the
    same floor, a few 1e-13, below the N = 24 row by more than 2^6."""
    rows = {int(r[0]): r[1:] for r in golden('table1_compact8_dt05dx2.txt')}
    e48, _ = _table_run(48, 'dt')
    say('table 1 N=48', e48, 'paper', rows[48])
    assert e48[0] < 5e-13
    assert rows[24][0] / e48[0] > 2 ** 6
