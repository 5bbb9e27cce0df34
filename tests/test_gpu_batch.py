"""The batch (serving) API through the C ABI: several independent problems of
different sizes and boundary conditions advanced by shared launches (one HIP
graph per run) must give, slot by slot, exactly the states of separate
contexts advanced eagerly — every replay checked, with eager work and
synchronisation between replays — and the admission, end and release rules."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I
from tests.parity import field_errors

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def problems():
    return [I.acoustic_pulse_2d(48, seed=5, amp=1e-3, half_width=0.2, ny=33),
            I.shock_vortex_2d(64, 32, Rc=0.12),
            I.vortex_translation_2d(24),
            I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21),
            dataclasses.replace(I.shear_wave_2d(29, 0.01, A=0.05, ny=19, U=0.3, rho=1.2, p=0.7), mu=0.01)]


def test_batch_replays_equal_separate_contexts():
    from paper_2001_01570_amd.cgks import Batch, Solver, SLOT_RUNNING, SLOT_DONE
    probs = problems()
    say('batch of', [(p.name, p.nx, p.ny) for p in probs])
    b = Batch(1 * GiB, max_slots=8)
    slots = [b.admit(p, max_steps=7) for p in probs]
    refs = [Solver(p) for p in probs]
    done = 0
    for rnd in range(3):           # 3 + 3 + 1 steps: the same 3-step graph replayed, then a 1-step tail
        b.run(3)
        n_new = min(3, 7 - done)
        for r in refs:
            r.run_steps(n_new)
        done += n_new
        for p, s, r in zip(probs, slots, refs):
            st, t, n = b.poll(s)
            g = b.read(s)
            e, te, ne = r.get_state()
            say(rnd, p.name, st, n, t, te)
            assert n == ne == done
            assert t == te
            assert np.array_equal(g, e), (p.name, rnd, np.abs(g - e).max())
            assert st == (SLOT_DONE if done == 7 else SLOT_RUNNING)
    for s in slots:
        b.release(s)
    b.close()


def test_batch_slot_stops_at_its_end_time():
    from paper_2001_01570_amd.cgks import Batch, Solver, SLOT_DONE
    p = I.vortex_translation_2d(24)
    t_end = 0.05
    b = Batch(GiB // 4, max_slots=2)
    s = b.admit(p, t_end=t_end)
    r = Solver(p)
    r.advance_to(t_end)
    for _ in range(10):
        b.run(4)
        if b.poll(s)[0] == SLOT_DONE:
            break
    st, t, n = b.poll(s)
    e, te, ne = r.get_state()
    assert st == SLOT_DONE and t == t_end == te and n == ne
    assert np.array_equal(b.read(s), e)
    b.close()


def test_batch_slot_matches_the_oracle():
    from paper_2001_01570_amd.cgks import Batch
    p = I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21)
    o = O.Oracle(p, threads=8)
    b = Batch(GiB // 4, max_slots=2)
    s = b.admit(p, max_steps=1)
    b.run(1)
    dt = b.poll(s)[1]
    o.step(dt)
    e = field_errors(b.read(s), o.state)
    say('batch slot vs oracle', e)
    assert e.max() < 1e-12
    b.close()


def test_batch_admission_and_release():
    from paper_2001_01570_amd.cgks import Batch, CgksError, CGKS_EBUSY, CGKS_EINVAL, CGKS_ENONPHYS, SLOT_FREE
    small = I.vortex_translation_2d(24)
    big = I.acoustic_pulse_2d(256, seed=1)
    b = Batch(64 << 20, max_slots=3)          # 64 MiB: one 256^2 problem needs ~42 MB
    s_big = b.admit(big, max_steps=2)
    with pytest.raises(CgksError) as ex:       # no room for a second one
        b.admit(I.acoustic_pulse_2d(256, seed=2), max_steps=2)
    assert ex.value.code == CGKS_EBUSY
    s1 = b.admit(small, max_steps=2)
    s2 = b.admit(small, max_steps=2)
    with pytest.raises(CgksError) as ex:       # no free slot
        b.admit(small, max_steps=2)
    assert ex.value.code == CGKS_EBUSY
    b.release(s_big)
    assert b.poll(s_big)[0] == SLOT_FREE
    s3 = b.admit(I.acoustic_pulse_2d(256, seed=2), max_steps=2)   # memory came back
    assert s3 == s_big
    with pytest.raises(CgksError) as ex:       # 1D is not served by the batch
        b.admit(I.sine_wave_1d(16), max_steps=2)
    assert ex.value.code == CGKS_EINVAL
    b.release(s1)
    bad = small.fields.copy()
    bad[0, 3, 4] = -1.0
    with pytest.raises(CgksError) as ex:
        b.admit(small, fields=bad, max_steps=2)
    assert ex.value.code == CGKS_ENONPHYS
    b.run(2)
    for s in (s2, s3):
        assert b.poll(s)[2] == 2
    b.close()


def test_batch_failing_slot_leaves_the_others_unchanged():
    """A slot whose step turns non-physical (a fixed step far beyond
    stability) fails alone: its state stays at the last good step, the other
    slots advance bitwise as separate contexts."""
    from paper_2001_01570_amd.cgks import Batch, Solver, SLOT_FAILED, SLOT_DONE
    good = [I.vortex_translation_2d(24), I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21)]
    bad = dataclasses.replace(I.acoustic_pulse_2d(32, seed=2, amp=0.05, half_width=0.3), fixed_dt=50.0)
    b = Batch(GiB // 4, max_slots=4)
    sg = [b.admit(p, max_steps=3) for p in good]
    sb = b.admit(bad, max_steps=3)
    b.run(3)
    st, t, n = b.poll(sb)
    assert st == SLOT_FAILED and n == 0 and t == 0.0
    assert np.array_equal(b.read(sb), bad.fields)
    for p, s in zip(good, sg):
        r = Solver(p)
        r.run_steps(3)
        assert b.poll(s)[0] == SLOT_DONE
        assert np.array_equal(b.read(s), r.get_state()[0])
    b.close()


def test_batch_slot_reused_by_another_grid():
    """A released slot index taken by a problem of another size between two
    runs: the launches must follow the new grid (regression: the block table
    was kept when the set of running slot indices looked unchanged)."""
    from paper_2001_01570_amd.cgks import Batch, Solver
    a = I.acoustic_pulse_2d(96, seed=3, amp=1e-3, half_width=0.2)
    c = I.vortex_translation_2d(24)
    d = I.acoustic_pulse_2d(40, seed=6, amp=1e-3, half_width=0.2, ny=28)
    b = Batch(GiB // 4, max_slots=4)
    sa = b.admit(a, max_steps=4)
    sc = b.admit(c, max_steps=4)
    b.run(2)
    b.release(sa)
    sd = b.admit(d, max_steps=4)
    assert sd == sa
    b.run(2)
    rc, rd = Solver(c), Solver(d)
    rc.run_steps(4)
    rd.run_steps(2)
    assert b.poll(sc)[2] == 4 and b.poll(sd)[2] == 2
    assert np.array_equal(b.read(sc), rc.get_state()[0])
    assert np.array_equal(b.read(sd), rd.get_state()[0])
    b.close()


def _kinds():
    """One problem of every slot kind: two and four Gauss points, FP64 and FP32
    gradient storage (walls and inflow among them)."""
    from paper_2001_01570_amd.cgks import CGKS_FP32_STORAGE
    g4 = lambda p: dataclasses.replace(p, gauss_points=4)
    return [(I.acoustic_pulse_2d(48, seed=5, amp=1e-3, half_width=0.2, ny=33), 0),
            (g4(I.shock_vortex_2d(64, 32, Rc=0.12)), 0),
            (g4(I.acoustic_pulse_2d(37, seed=4, amp=0.05, half_width=0.3, ny=21)), 0),
            (I.vortex_translation_2d(24), CGKS_FP32_STORAGE),
            (g4(I.acoustic_pulse_2d(40, seed=2, amp=1e-3, half_width=0.2, ny=24)), CGKS_FP32_STORAGE),
            (I.shock_vortex_2d(64, 32, Rc=0.12), 0)]


def test_batch_of_mixed_kinds_equals_separate_contexts():
    """Slots of all four kinds in one batch (their own face launches in the
    same graph): every replay bitwise equal to separate contexts of the same
    configuration, a slot index reused by another kind included."""
    from paper_2001_01570_amd.cgks import Batch, Solver
    kinds = _kinds()
    say('mixed batch', [(p.name, p.gauss_points, st) for p, st in kinds])
    b = Batch(1 * GiB, max_slots=8)
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
    # slot 0 (two points, FP64) taken by a four-point FP32 problem
    b.release(slots[0])
    p, st = kinds[4]
    s = b.admit_storage(p, st, max_steps=2)
    assert s == slots[0]
    b.run(2)
    r = Solver(p, storage=st)
    r.run_steps(2)
    assert np.array_equal(b.read(s), r.get_state()[0])
    b.close()


def test_batch_four_point_slot_matches_the_oracle():
    from paper_2001_01570_amd.cgks import Batch
    p = dataclasses.replace(I.shock_vortex_2d(64, 32, Rc=0.12), gauss_points=4)
    o = O.Oracle(p, threads=8)
    b = Batch(GiB // 4, max_slots=2)
    s = b.admit(p, max_steps=1)
    b.run(1)
    dt = b.poll(s)[1]
    o.step(dt)
    e = field_errors(b.read(s), o.state)
    say('four-point batch slot vs oracle', e)
    assert e.max() < 1e-12
    b.close()


@pytest.mark.parametrize('tiles', [(0, 0), (1, 2), (2, 1)])
def test_batch_tile_shapes_do_not_change_results(tiles):
    from paper_2001_01570_amd.cgks import Batch, Solver, CgksError, CGKS_ESTATE, batch_tuning
    x, y, n = batch_tuning()
    assert 0 <= x <= 2 and 0 <= y <= 2 and n >= 1
    probs = problems()[:3]
    b = Batch(GiB // 2, max_slots=4)
    b.set_tiles(*tiles)
    slots = [b.admit(p, max_steps=3) for p in probs]
    with pytest.raises(CgksError) as ex:       # not while slots are admitted
        b.set_tiles(0, 0)
    assert ex.value.code == CGKS_ESTATE
    b.run(3)
    for p, s in zip(probs, slots):
        r = Solver(p)
        r.run_steps(3)
        assert np.array_equal(b.read(s), r.get_state()[0]), (p.name, tiles)
    b.close()
