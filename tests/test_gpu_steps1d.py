"""The single-launch 1D step (k_steps1: whole steps in one block for grids of
at most 255 cells) against the separate launches of the same step, which the
library uses while the kernels are timed one by one: equal times and step
counts, and states equal to rounding, through step / run_steps / advance_to,
across the size threshold, at resumed end times, and on a failing step.  Both
run the same device functions, but the compiler may contract a few operations
differently in the two kernels: on shocks, momenta near zero then differ by
1e-20 to 1e-24 of the field's scale after a step, and the gradients at a shock
carry that up to ~1e-14 of their scale within a hundred steps.  The bar is the
parity bar of the scheme against the oracle, 1e-12 of each field's scale."""
import numpy as np
import pytest

from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pair(p):
    from paper_2001_01570_amd.cgks import Solver
    fused, eager = Solver(p), Solver(p)
    eager.set_profiling(True)         # per-kernel events: the separate launches
    return fused, eager


def _same(a, b):
    ga, ta, na = a.get_state()
    gb, tb, nb = b.get_state()
    assert na == nb and ta == tb
    for f in range(ga.shape[0]):
        scale = max(np.abs(gb[f]).max(), 1e-300)
        assert np.abs(ga[f] - gb[f]).max() <= 1e-12 * scale, f


@pytest.mark.parametrize('n', [1, 5, 100, 254, 255, 256, 257])
def test_fused_steps_equal_separate_launches(n):
    fused, eager = _pair(I.sine_wave_1d(n))
    for s in (fused, eager):
        s.step()
        s.step(1e-3)                  # a given step size
        s.run_steps(37)
    _same(fused, eager)


@pytest.mark.parametrize('mk', [lambda: I.shock_entropy_1d(240), lambda: I.shock_tube_1d(100)])
def test_fused_advance_to_and_resume(mk):
    fused, eager = _pair(mk())
    for t_end in (0.05, 0.05, 0.11, 0.2):      # no-op launches past each end must not disturb the next call
        n1, n2 = fused.advance_to(t_end), eager.advance_to(t_end)
        assert n1 == n2
        _same(fused, eager)


def test_fused_failing_step_not_committed():
    from paper_2001_01570_amd.cgks import CgksError, CGKS_ENONPHYS, Solver
    p = I.shock_tube_1d(100)
    s = Solver(p)
    s.run_steps(3)
    before = s.get_state()
    with pytest.raises(CgksError) as ei:
        s.step(50.0)                  # far beyond any stable step
    assert ei.value.code == CGKS_ENONPHYS
    after = s.get_state()
    assert np.array_equal(after[0], before[0]) and after[1:] == before[1:]
