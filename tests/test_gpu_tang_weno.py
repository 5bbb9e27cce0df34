"""The tangential-WENO variant of the 2D assembly (tang_weno = 1; an
evaluated variant): the two WENO-Z states at each Gauss point come from a
WENO-Z of the three average-interpolating quadratics on the five nearest
face segments.  The HIP path (two points: face kernels with a 5-segment
halo; four points: the middle five of the seven segments) against the
oracle with the same option: single steps with walls,
inflow, no-slip walls, a near vacuum and a ragged grid, FP32 gradient
storage, tiny grids, 40-step runs with each side's own steps, a run where
both guards fire, the Mach 2 shock-vortex run whose WENO-state fallbacks
the variant removes, batch slots, the configurations it refuses, and which
options carry the strong shock-vortex case."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I
from tests.parity import field_errors, field_scales, scaled_errors
from tests.test_gpu_parity import _tiny, TINY, TINY4
from tests.test_gpu_parity_runs import _guard_case, own_dt_run

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def tw(p):
    return dataclasses.replace(p, tang_weno=1)


def moving_pulse():
    p = I.acoustic_pulse_2d(40, seed=4, amp=0.05, half_width=0.3, ny=24)
    f = p.fields
    f[1] += 0.2 * f[0]
    f[2] += 0.1 * f[0]
    f[3] += 0.5 * 0.05 * f[0]
    return p


CASES = [
    ('shock_vortex_walls_inflow', lambda: I.shock_vortex_2d(64, 32, Rc=0.12), 3, 1e-10),
    ('expansion_near_vacuum', lambda: I.expansion_2d(32, 28, U=1.25, amp=0.1), 2, 1e-10),
    ('viscous_shock_vortex_noslip', lambda: dataclasses.replace(I.shock_vortex_2d(48, 24, Rc=0.12), mu=1e-3,
                                                                bc=(I.INFLOW, I.FREE, I.NOSLIP, I.NOSLIP)), 2, 1e-10),
    ('moving_pulse_noslip', lambda: dataclasses.replace(moving_pulse(), bc=(I.NOSLIP,) * 4), 0, 1e-12),
    ('pulse_ragged', lambda: I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21), 0, 1e-12),
]


def _step_pair(p, before, storage=0):
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
    r = Solver(dataclasses.replace(p, tang_weno=0), storage=storage)
    r.set_state(st, t)
    r.step(dt)
    e = field_errors(s.state, o.state)
    change = (np.abs(s.state - r.state).reshape(12, -1).max(axis=1) / field_scales(o.state)).max()
    return e, change


@pytest.mark.parametrize('gp', [2, 4])
@pytest.mark.parametrize('name,mk,before,min_change', CASES, ids=[c[0] for c in CASES])
def test_single_step(name, mk, before, min_change, gp):
    p = tw(dataclasses.replace(mk(), gauss_points=gp))
    say('tangential WENO single step', name, p.nx, p.ny, 'gauss points', gp)
    e, change = _step_pair(p, before)
    say(name, 'errors', e.max(), 'change against the quintic states', change)
    assert e.max() < TOL, e
    assert change > min_change


@pytest.mark.parametrize('gp', [2, 4])
def test_fp32_storage_single_step(gp):
    from paper_2001_01570_amd.cgks import CGKS_FP32_STORAGE
    e, change = _step_pair(tw(dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp)), 3, CGKS_FP32_STORAGE)
    say('tangential WENO, fp32 storage: averages', e[:4].max(), 'gradients', e[4:].max())
    assert e[:4].max() < 1e-8, e
    assert e[4:].max() < 4 * 2.0 ** -24, e


TINY_TW = [t + (2,) for t in TINY] + [t + (4,) for t in TINY4]


@pytest.mark.parametrize('nx,ny,kind,gp', TINY_TW, ids=['g%d_%dx%d-%s' % (t[3], t[0], t[1], t[2]) for t in TINY_TW])
def test_tiny_grids(nx, ny, kind, gp):
    """Grids smaller than the five-segment stencil (ghosts wrap onto or
    mirror the same few cells)."""
    _tiny(nx, ny, kind, gp, tang_weno=1)


@pytest.mark.parametrize('gp', [2, 4])
def test_forty_steps_each_side_its_own_dt(gp):
    p = tw(dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=gp))
    s, o, rel = own_dt_run(p, steps=40)
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    say('tangential WENO, 40 steps: dt rel', rel.max(), 'scaled errors', err)
    assert rel.max() < 1e-13
    assert err.max() < TOL, err


def test_guards_fire_with_the_variant():
    _guard_case(tw(I.expansion_2d(32, 28, U=1.25, amp=0.1)), steps=12, min_w0=1, min_weno=0)
    _guard_case(tw(I.expansion_2d(32, 28, U=1.25, amp=0.1, gauss_points=4)), steps=8, min_w0=1, min_weno=0)


def test_mach2_shock_vortex_run_without_weno_fallbacks():
    """M_s = 2, M_v = 0.5, 64 x 32, CFL 0.3 to t = 0.3 with each side's own
    steps: equal step and guard counts, no WENO-state fallback (the scheme as
    read takes 5 in the oracle), states within 1e-12."""
    p = tw(I.shock_vortex_2d(64, 32, Ms=2.0, Mv=0.5, cfl=0.3))
    s, o, _ = own_dt_run(p, t_end=0.3)
    cs, co = s.counters(), o.counters()
    say('tangential WENO, Mach 2 shock-vortex:', co['steps'], 'steps, guards GPU', cs['guard_w0'], cs['guard_weno'],
        'oracle', co['guard_w0'], co['guard_weno'])
    assert cs['steps'] == co['steps'] and cs['guard_weno'] == co['guard_weno'] == 0
    assert cs['guard_w0'] == co['guard_w0']
    err = scaled_errors(s.state, o.state, p.dx, p.dy)
    assert err.max() < TOL, err


def test_batch_slots_equal_separate_contexts():
    """Tangential-WENO slots (both storages) beside the other kinds in one
    batch: bitwise equal to separate contexts on every replay; one slot
    within 1e-12 of the oracle."""
    from paper_2001_01570_amd.cgks import Batch, CGKS_FP32_STORAGE, Solver
    kinds = [(tw(I.shock_vortex_2d(64, 32, Rc=0.12)), 0),
             (tw(dataclasses.replace(moving_pulse(), bc=(I.NOSLIP,) * 4)), CGKS_FP32_STORAGE),
             (tw(dataclasses.replace(I.shock_vortex_2d(40, 24, Rc=0.12), gauss_points=4)), 0),
             (tw(dataclasses.replace(I.shock_vortex_2d(40, 24, Rc=0.12), gauss_points=4)), CGKS_FP32_STORAGE),
             (I.shock_vortex_2d(64, 32, Rc=0.12), 0),
             (dataclasses.replace(I.shock_vortex_2d(48, 24, Rc=0.12), side_slopes=1), 0),
             (dataclasses.replace(I.shock_vortex_2d(48, 24, Rc=0.12), recon_vars=1, gauss_points=4), 0)]
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
            assert np.array_equal(g, e), (p.name, st, rnd, np.abs(g - e).max())
    assert np.abs(b.read(slots[0]) - b.read(slots[4])).max() > 1e-8
    b.close()
    p = kinds[0][0]
    o = O.Oracle(p, threads=8)
    b = Batch(1 << 28, max_slots=2)
    s = b.admit(p, max_steps=1)
    b.run(1)
    o.step(b.poll(s)[1])
    e = field_errors(b.read(s), o.state)
    say('tangential-WENO batch slot vs oracle', e.max())
    assert e.max() < TOL
    b.close()


def test_refused_with_other_options():
    from paper_2001_01570_amd.cgks import CgksError, CGKS_EINVAL, Solver
    for bad in (dict(recon_vars=1), dict(side_slopes=1)):
        with pytest.raises(CgksError) as ei:
            Solver(dataclasses.replace(tw(I.shock_vortex_2d(32, 16, Rc=0.12)), **bad))
        assert ei.value.code == CGKS_EINVAL


@pytest.mark.parametrize('Ms,gp,kw,reaches', [
    (2.0, 2, {}, False), (2.0, 2, dict(recon_vars=1), True), (2.0, 2, dict(tang_weno=1), True),
    (2.5, 2, {}, False), (2.5, 2, dict(recon_vars=1), False), (2.5, 2, dict(side_slopes=1), False),
    (2.5, 2, dict(tang_weno=1), True), (2.5, 4, {}, False), (2.5, 4, dict(recon_vars=1), True),
    (2.5, 4, dict(tang_weno=1), True), (3.0, 2, dict(tang_weno=1), False), (3.0, 4, dict(recon_vars=1), False)],
    ids=['Ms2-as_read', 'Ms2-characteristic', 'Ms2-tang_weno', 'Ms2.5-as_read', 'Ms2.5-characteristic',
         'Ms2.5-side_slopes', 'Ms2.5-tang_weno', 'Ms2.5-g4-as_read', 'Ms2.5-g4-characteristic',
         'Ms2.5-g4-tang_weno', 'Ms3-tang_weno', 'Ms3-g4-characteristic'])
def test_strong_shock_vortex_which_options_carry_it(Ms, gp, kw, reaches):
    """The shock-vortex case at 256 x 128 (M_v = 0.5, CFL 0.3) to t = 0.3 on
    the GPU path: the scheme as read stops at a non-physical state for
    M_s >= 2 (t = 0.17 at M_s = 2, 0.08 at 2.5); characteristic variables
    carry M_s = 2 and, with four Gauss points, 2.5; the tangential WENO
    carries M_s = 2.5 with two and four points (with two, characteristic
    variables stop at t = 0.285, the side slopes at 0.037); at M_s = 3 every
    option stops (t < 0.14)."""
    from paper_2001_01570_amd.cgks import CgksError, CGKS_ENONPHYS, Solver
    p = dataclasses.replace(I.shock_vortex_2d(256, 128, Ms=Ms, Mv=0.5, cfl=0.3), gauss_points=gp, **kw)
    s = Solver(p)
    try:
        s.advance_to(0.3)
        ok = True
    except CgksError as e:
        assert e.code == CGKS_ENONPHYS
        ok = False
    say('shock-vortex M_s', Ms, 'gauss points', gp, kw, 'reaches t = 0.3' if ok else 'stops at t = %.3f' % s.t)
    assert ok == reaches
    if not ok:
        assert s.t < 0.29
    s.close()


@pytest.mark.parametrize('gp', [2, 4])
def test_guards_fire_next_to_noslip_walls(gp):
    """The flow leaves every no-slip wall (the 2D expansion with velocity 1.0
    towards the curve): both fallbacks fire along the walls (the WENO
    fallback takes the cells beside the face through the boundary rule);
    guard counts and states follow the oracle step by step and over 30
    steps."""
    p = tw(dataclasses.replace(I.expansion_2d(32, 28, U=-1.0, amp=0.1, gauss_points=gp), bc=(I.NOSLIP,) * 4))
    _guard_case(p, steps=30, min_w0=1, min_weno=1)
