"""Parity of the reconstruction in characteristic variables (Sec. 3.2: the
WENO-Z states of each stencil line from the eigenvector coordinates of the
normal flux Jacobian at the mean of the two cells beside the face) on the
HIP path against the oracle: single steps and whole runs in 1D and 2D (two
and four Gauss points, walls and inflow, FP32 gradient storage), a run in
which the positivity guards fire, and batch slots of the characteristic
kinds beside conservative ones."""
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
GiB = 1 << 30


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def chv(p):
    return dataclasses.replace(p, recon_vars=1)


def solver(prob, **kw):
    from paper_2001_01570_amd.cgks import Solver
    return Solver(prob, **kw)


def step_pair(p, steps_before):
    """The oracle advanced `steps_before` steps; one GPU step and one oracle
    step of the same size from that state, and one GPU step of the same size
    with conservative variables (to show that the option changes the
    result).  Returns (errors against the oracle, relative change against
    the conservative step)."""
    o = O.Oracle(p, threads=8)
    for _ in range(steps_before):
        o.step()
    st, t, _ = o.get_state()
    s = solver(p)
    s.set_state(st, t)
    dt = s.step()
    o.step(dt)
    sc = solver(dataclasses.replace(p, recon_vars=0))
    sc.set_state(st, t)
    sc.step(dt)
    change = (np.abs(s.state - sc.state).reshape(s.state.shape[0], -1).max(axis=1) / field_scales(o.state)).max()
    return field_errors(s.state, o.state), change


CASES_1D = [
    ('shock_tube', lambda: I.shock_tube_1d(100), 6),
    ('shock_entropy', lambda: I.shock_entropy_1d(400, t_end=1.8), 4),
    ('pressure_ratio_300', lambda: I.riemann_1d((1.0, 0.0, 30.0), (0.125, 0.0, 0.1), 100), 3),
]


@pytest.mark.parametrize('name,mk,before', CASES_1D, ids=[c[0] for c in CASES_1D])
def test_1d_single_step(name, mk, before):
    p = chv(mk())
    say('1d characteristic single step', name, p.nx)
    e, change = step_pair(p, before)
    say(name, 'errors', e.max(), 'change against conservative variables', change)
    assert e.max() < TOL, e
    assert change > 1e-8


def test_1d_shock_tube_whole_run_each_side_its_own_dt():
    p = chv(I.shock_tube_1d(100))
    s, o, _ = own_dt_run(p, t_end=0.16)
    err = scaled_errors(s.state, o.state, p.dx)
    say('1d characteristic shock tube to t = 0.16', o.counters()['steps'], 'steps, scaled errors', err)
    assert s.t == o.t == 0.16
    assert err.max() < TOL, err


CASES_2D = [
    ('shock_vortex_walls_inflow', lambda: I.shock_vortex_2d(64, 32, Rc=0.12), 3),
    ('expansion_near_vacuum', lambda: I.expansion_2d(32, 28, U=1.25, amp=0.1), 2),
    ('viscous_shock_vortex_noslip', lambda: dataclasses.replace(I.shock_vortex_2d(48, 24, Rc=0.12), mu=1e-3,
                                                                bc=(I.INFLOW, I.FREE, I.NOSLIP, I.NOSLIP)), 2),
]


@pytest.mark.parametrize('gp', [2, 4])
@pytest.mark.parametrize('name,mk,before', CASES_2D, ids=[c[0] for c in CASES_2D])
def test_2d_single_step(name, mk, before, gp):
    p = chv(dataclasses.replace(mk(), gauss_points=gp))
    say('2d characteristic single step', name, p.nx, p.ny, 'gauss points', gp)
    e, change = step_pair(p, before)
    say(name, gp, 'errors', e.max(), 'change against conservative variables', change)
    assert e.max() < TOL, e
    assert change > 1e-8


@pytest.mark.parametrize('gp', [2, 4])
def test_2d_forty_steps_each_side_its_own_dt(gp):
    p = chv(dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp))
    s, o, rel = own_dt_run(p, steps=40)
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    say('2d characteristic 40 steps, gauss points', gp, 'dt rel', rel.max(), 'scaled errors', err)
    assert rel.max() < 1e-13
    assert err.max() < TOL, err


def moving_pulse():
    """The acoustic pulse carried by a mean flow (0.2, 0.1): both momenta
    are non-zero next to every wall."""
    p = I.acoustic_pulse_2d(40, seed=4, amp=0.05, half_width=0.3, ny=24)
    f = p.fields
    f[1] += 0.2 * f[0]
    f[2] += 0.1 * f[0]
    f[3] += 0.5 * 0.05 * f[0]
    return p


@pytest.mark.parametrize('gp', [2, 4])
@pytest.mark.parametrize('walls', ['x', 'y', 'all'])
def test_noslip_walls_repeatable_and_at_parity(walls, gp):
    """No-slip walls mirror both momenta, so the ghost cells of a wall normal
    to the face direction enter the characteristic projection with every
    component changed: three contexts from one state give bitwise equal steps,
    and each is within 1e-12 of the oracle's (a regression test: the ghost
    values of that pass were once wrong and varied from run to run)."""
    N, P = I.NOSLIP, I.PERIODIC
    bc = {'x': (N, N, P, P), 'y': (P, P, N, N), 'all': (N, N, N, N)}[walls]
    p = dataclasses.replace(moving_pulse(), recon_vars=1, bc=bc, gauss_points=gp)
    say('characteristic variables, no-slip walls', walls, 'gauss points', gp)
    o = O.Oracle(p, threads=8)
    st, t, _ = o.get_state()
    o.step(1e-3)
    outs = []
    for _ in range(3):
        s = solver(p)
        s.set_state(st, t)
        s.step(1e-3)
        assert s.counters()['guard_weno'] == o.counters()['guard_weno'] == 0
        outs.append(s.state.copy())
        s.close()
    for x in outs[1:]:
        assert np.array_equal(x, outs[0])
    e = field_errors(outs[0], o.state)
    say('no-slip', walls, gp, 'errors', e.max())
    assert e.max() < TOL, e


@pytest.mark.parametrize('rv,steps', [(0, 30), (1, 12)], ids=['conservative', 'characteristic'])
def test_guards_fire_next_to_noslip_walls(rv, steps):
    """The flow leaves every wall (the 2D expansion with velocity 1.0 towards
    the curve, no-slip walls on all sides): the gas thins out along the
    walls, the equilibrium and WENO fallbacks fire there (the WENO fallback
    takes the cells beside the face through the boundary rule), and the
    guard counts and states follow the oracle step by step and over the run
    (with characteristic variables the oracle meets a vacuum at step 13)."""
    p = dataclasses.replace(I.expansion_2d(32, 28, U=-1.0, amp=0.1), bc=(I.NOSLIP,) * 4, recon_vars=rv)
    _guard_case(p, steps=steps, min_w0=1, min_weno=1)


def test_2d_guards_fire_with_characteristic_variables():
    """The curved expansion to near-vacuum: equilibrium and WENO fallbacks
    fire; the guard counts equal the oracle's step by step and over the run."""
    _guard_case(chv(I.expansion_2d(32, 28, U=1.25, amp=0.1)), steps=20, min_w0=1, min_weno=1)


@pytest.mark.parametrize('gp', [2, 4])
def test_fp32_storage_single_step(gp):
    """FP32 gradient storage: from a state whose gradients are FP32 values,
    one step against the oracle's.  The gradients of the intermediate state
    are stored in FP32 as well and reach the averages through the second
    stage's fluxes, so the averages are within 1e-8 of their field scale (the
    FP64 path: 1e-12) and the gradients within their FP32 rounding (2^-24 of
    the field scale, with a margin of 4)."""
    from paper_2001_01570_amd.cgks import CGKS_FP32_STORAGE
    p = chv(dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp))
    o = O.Oracle(p, threads=8)
    for _ in range(3):
        o.step()
    st, t, _ = o.get_state()
    st[4:] = st[4:].astype(np.float32).astype(np.float64)
    s = solver(p, storage=CGKS_FP32_STORAGE)
    s.set_state(st, t)
    o.set_state(st, t)
    dt = s.step()
    o.step(dt)
    e = field_errors(s.state, o.state)
    say('fp32 storage, characteristic, gauss points', gp, 'averages', e[:4].max(), 'gradients', e[4:].max())
    assert e[:4].max() < 1e-8, e
    assert e[4:].max() < 4 * 2.0 ** -24, e


def test_batch_characteristic_kinds_equal_separate_contexts():
    """Characteristic slots of every Gauss-point count and storage next to
    conservative ones in one batch (walls, inflow, no-slip walls on every
    side): bitwise equal to separate contexts on every replay, and one
    characteristic slot within 1e-12 of the oracle."""
    from paper_2001_01570_amd.cgks import Batch, CGKS_FP32_STORAGE
    g4 = lambda p: dataclasses.replace(p, gauss_points=4)
    kinds = [(chv(I.shock_vortex_2d(64, 32, Rc=0.12)), 0),
             (chv(g4(I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21))), 0),
             (chv(I.vortex_translation_2d(24)), CGKS_FP32_STORAGE),
             (chv(g4(I.shock_vortex_2d(40, 24, Rc=0.12))), CGKS_FP32_STORAGE),
             (I.shock_vortex_2d(64, 32, Rc=0.12), 0),
             (chv(dataclasses.replace(moving_pulse(), bc=(I.NOSLIP,) * 4)), 0),
             (chv(g4(dataclasses.replace(moving_pulse(), bc=(I.NOSLIP,) * 4))), 0)]
    say('characteristic batch', [(p.name, p.gauss_points, st, p.recon_vars) for p, st in kinds])
    b = Batch(1 * GiB, max_slots=8)
    slots = [b.admit_storage(p, st, max_steps=6) for p, st in kinds]
    refs = [solver(p, storage=st) for p, st in kinds]
    for rnd in range(2):
        b.run(3)
        for r in refs:
            r.run_steps(3)
        for (p, st), s, r in zip(kinds, slots, refs):
            g = b.read(s)
            e, te, ne = r.get_state()
            assert b.poll(s)[2] == ne == 3 * (rnd + 1)
            assert np.array_equal(g, e), (p.name, p.gauss_points, st, rnd, np.abs(g - e).max())
    # the characteristic and the conservative shock-vortex slots differ
    assert np.abs(b.read(slots[0]) - b.read(slots[4])).max() > 1e-8
    b.close()
    p = kinds[0][0]
    o = O.Oracle(p, threads=8)
    b = Batch(GiB // 4, max_slots=2)
    s = b.admit(p, max_steps=1)
    b.run(1)
    o.step(b.poll(s)[1])
    e = field_errors(b.read(s), o.state)
    say('characteristic batch slot vs oracle', e.max())
    assert e.max() < TOL
    b.close()
