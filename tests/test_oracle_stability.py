"""The 2D step on a fluid at rest at CFL 0.15: inputs 1e-10 apart (relative,
on the gradients) stay apart by no more than a small multiple of that after
300 steps (no growing mode in this regime; at CFL 0.3 the step as read grows
an odd-even mode of the gradient fields, documented with its measurements)."""
import numpy as np

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I


def test_rest_state_pulse_is_stable_at_cfl_0_15():
    p = I.acoustic_pulse_2d(32, seed=0, amp=1e-3, half_width=0.2, cfl=0.15)
    rng = np.random.default_rng(1)
    f2 = p.fields.copy()
    f2[4:] *= 1 + 1e-10 * rng.standard_normal(f2[4:].shape)
    q = I.Problem(p.name, 2, p.nx, p.ny, p.x0, p.x1, p.y0, p.y1, f2, bc=p.bc, cfl=p.cfl)
    a, b = O.Oracle(p, threads=8), O.Oracle(q, threads=8)
    d0 = np.abs(a.state - b.state).max()
    for _ in range(300):
        dt = a.step()
        b.step(dt)
    d = np.abs(a.state - b.state).max()
    assert d < 20 * d0, (d0, d)
