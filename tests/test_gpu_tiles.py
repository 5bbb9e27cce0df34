"""Every face tile shape gives bitwise the same steps (the shape only changes
how faces are grouped into blocks), on periodic and on wall/inflow/free
boundaries, with grids that leave ragged tiles for each shape."""
import numpy as np
import pytest

from paper_2001_01570_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize('mk', [lambda: I.acoustic_pulse_2d(70, seed=2, amp=1e-3, half_width=0.2, ny=45),
                                lambda: I.shock_vortex_2d(66, 34, Rc=0.12)], ids=['pulse', 'shock_vortex'])
def test_tile_shapes_agree(mk):
    from paper_2001_01570_amd.cgks import Solver
    p = mk()
    states = []
    for shape in range(3):
        s = Solver(p)
        s.set_tiles(shape, (shape + 1) % 3)
        s.run_steps(3)
        states.append(s.state)
    for st in states[1:]:
        assert np.array_equal(st, states[0])
