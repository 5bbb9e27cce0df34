"""Per-kernel timing through the C ABI (cgks_set_profiling / cgks_kernel_times):
launch counts per kernel kind, positive device times, the event pool reused
past its capacity, a subset of kinds, results bitwise unchanged by profiling,
and graph replay (a stream of the solver's own) once profiling is off."""
import numpy as np
import pytest

from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_profiling_counts_every_launch_and_changes_no_result():
    import torch
    from paper_2001_01570_amd.cgks import KERNEL_NAMES_2D, Solver
    p = I.acoustic_pulse_2d(48, seed=3, amp=0.05, half_width=0.3, ny=40)
    ref = Solver(p)                                   # torch's current stream: eager launches
    ref.run_steps(200)
    s = Solver(p, stream=torch.cuda.Stream())         # a capturable stream (default priority)
    s.set_profiling(True)
    s.run_steps(200)                                  # 6 kinds x 200 = 1200 event pairs > the pool of 1024
    kt = s.kernel_times()
    assert set(kt) == set(KERNEL_NAMES_2D)
    for name, (ms, calls) in kt.items():
        assert calls == 200 and ms > 0.0, (name, ms, calls)
    assert np.array_equal(s.state, ref.state)
    s.set_profiling(False)                            # the totals stay readable; nothing more is recorded
    s.run_steps(60)                                   # two 25-step graph replays and 10 eager steps
    ref.run_steps(60)
    assert all(calls == 200 for _, calls in s.kernel_times().values())
    g, t, n = s.get_state()
    r, tr, nr = ref.get_state()
    assert n == nr == 260 and t == tr
    assert np.array_equal(g, r)


def test_profiling_a_subset_of_kinds_and_restarting():
    from paper_2001_01570_amd.cgks import Solver
    p = I.acoustic_pulse_2d(32, seed=1, amp=0.05, half_width=0.3)
    s = Solver(p)
    s.set_profiling(True, kinds=['xfaces1', 'update2'])
    s.run_steps(7)
    kt = s.kernel_times()
    assert kt['xfaces1'][1] == 7 and kt['update2'][1] == 7
    assert all(kt[k][1] == 0 and kt[k][0] == 0.0 for k in ('yfaces1', 'update1', 'xfaces2', 'yfaces2'))
    s.set_profiling(True)                             # switching on again starts from zero
    s.step()
    assert all(calls == 1 for _, calls in s.kernel_times().values())


def test_profiling_in_1d():
    from paper_2001_01570_amd.cgks import KERNEL_NAMES_1D, Solver
    p = I.sine_wave_1d(64)
    s = Solver(p)
    s.set_profiling(True)
    s.run_steps(33)                                   # (advance_to also times the no-op launches past t_end)
    kt = s.kernel_times()
    assert set(kt) == set(KERNEL_NAMES_1D) and s.get_state()[2] == 33
    assert all(calls == 33 and ms > 0.0 for ms, calls in kt.values())
