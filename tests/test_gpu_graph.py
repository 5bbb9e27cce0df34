"""run_steps on a capturable stream replays a captured HIP graph of 25 steps:
every replay, with eager work and synchronisation between replays, must give
exactly the state of the same steps launched one by one."""
import numpy as np
import pytest

from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('mk', [lambda: I.acoustic_pulse_2d(48, seed=5, amp=1e-3, half_width=0.2, ny=33),
                                lambda: I.shock_vortex_2d(64, 32, Rc=0.12)], ids=['pulse', 'shock_vortex'])
def test_graph_replays_equal_eager_steps(mk):
    import torch
    from paper_2001_01570_amd.cgks import Solver
    p = mk()
    side = torch.cuda.Stream()
    g = Solver(p, stream=side)          # capturable stream: graph replays
    e = Solver(p)                       # legacy default stream: step-by-step launches
    for rnd in range(3):
        g.run_steps(25)
        e.run_steps(25)
        sg, tg, ng = g.get_state()
        se, te, ne = e.get_state()
        assert ng == ne == 25 * (rnd + 1) and tg == te
        assert np.array_equal(sg, se), (rnd, np.abs(sg - se).max())
    # a remainder shorter than the graph runs step by step on the same context
    g.run_steps(7)
    e.run_steps(7)
    assert np.array_equal(g.get_state()[0], e.get_state()[0])
