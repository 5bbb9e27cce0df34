"""Pins of the oracle's tangential-WENO variant of the 2D assembly (an
evaluated variant, oracle option tang_weno = 1): at each Gauss point the
WENO-Z states of the five nearest face segments are combined by a WENO-Z of
the three average-interpolating quadratics, instead of the quintic of the
three nearest segments with the cells' tangential gradients (two points)
or the sextic of the seven (four points).
Pinned against what the definition fixes: with the linear weights the value
is the quartic through the five averages at the node (solved here with
numpy), quadratics are reproduced at any weights, reversing the segments
gives the other node, a jump leaves the smooth candidate alone; the 2D
y-invariant run equals the 1D run, the transposed problem the transposed
result; and the variant removes the WENO-state fallbacks of a Mach 2
shock-vortex run."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I
from tests.test_oracle_scheme import transpose_fields

ETA = -0.5 / math.sqrt(3.0)
# the four-point nodes (inner and outer pair)
ETA4 = [0.5 * math.sqrt(3.0 / 7.0 - 2.0 / 7.0 * math.sqrt(6.0 / 5.0)),
        0.5 * math.sqrt(3.0 / 7.0 + 2.0 / 7.0 * math.sqrt(6.0 / 5.0))]


def quartic_at(s, eta):
    """Point value at eta of the quartic whose averages over the unit segments
    centred at -2..2 are s (numpy solve of the moment equations)."""
    A = np.array([[((m + 0.5) ** (p + 1) - (m - 0.5) ** (p + 1)) / (p + 1) for p in range(5)] for m in range(-2, 3)])
    c = np.linalg.solve(A, np.asarray(s, dtype=float))
    return sum(c[p] * eta ** p for p in range(5))


def test_linear_weights_give_the_quartic_at_the_node():
    rng = np.random.default_rng(11)
    for _ in range(50):
        s = rng.standard_normal(5)
        v = O.tang_weno(s, eps=1e30)                    # tau / (beta + eps) = 0: the linear weights
        assert v == pytest.approx(quartic_at(s, ETA), abs=1e-14)
        assert O.tang_weno(s[::-1], eps=1e30) == pytest.approx(quartic_at(s, -ETA), abs=1e-14)


@pytest.mark.parametrize('eta', [-ETA4[1], -ETA4[0], ETA4[0], ETA4[1], ETA])
def test_any_node_linear_weights_give_the_quartic(eta):
    """The general-node form (four points): the quartic at the node with the
    linear weights, quadratics exact at any weights, and at the two-point
    node the same value as the fixed-node form."""
    rng = np.random.default_rng(13)
    for _ in range(30):
        s = rng.standard_normal(5)
        assert O.tang_weno_eta(s, eta, eps=1e30) == pytest.approx(quartic_at(s, eta), abs=1e-13)
        a, b, c = rng.standard_normal(3)
        avg = [a + b * m + c * (m * m + 1.0 / 12.0) for m in range(-2, 3)]
        assert O.tang_weno_eta(avg, eta, eps=1e-6) == pytest.approx(a + b * eta + c * eta * eta, abs=1e-13)
        if eta == ETA:
            assert O.tang_weno_eta(s, eta) == pytest.approx(O.tang_weno(s), abs=1e-14)
    _, _, _, w = O.tang_weno_eta(rng.standard_normal(5), eta, eps=1e30, details=True)
    assert (w > 0).all()                              # the linear weights are positive at every node


def test_quadratics_are_exact_at_any_weights():
    rng = np.random.default_rng(12)
    for _ in range(50):
        a, b, c = rng.standard_normal(3)
        avg = [a + b * m + c * (m * m + 1.0 / 12.0) for m in range(-2, 3)]
        v, cand, beta, w = O.tang_weno(avg, eps=1e-6, details=True)
        exact = a + b * ETA + c * ETA * ETA
        assert np.abs(cand - exact).max() < 1e-14
        assert v == pytest.approx(exact, abs=1e-14)
        assert w.sum() == pytest.approx(1.0, abs=1e-15)


def test_a_jump_leaves_the_smooth_candidate():
    """A jump between segments 0 and 1: the quadratic on segments -2..0 is
    smooth and takes almost all the weight at the first node, so the value
    stays at the left state (the linear combination overshoots into the
    jump)."""
    s = np.array([0.0, 0.0, 0.0, 1.0, 1.0])
    v, cand, beta, w = O.tang_weno(s, eps=1e-6, details=True)
    assert beta[0] == 0.0 and beta[1] > 0.1 and beta[2] > 0.1
    assert w[0] > 0.999
    assert abs(v) < 1e-3
    assert abs(O.tang_weno(s, eps=1e30)) > 1e-2


@pytest.mark.parametrize('bad', [dict(recon_vars=1), dict(side_slopes=1)])
def test_refused_configurations(bad):
    with pytest.raises(O.OracleError):
        O.Oracle(dataclasses.replace(I.uniform_2d(6, 6), tang_weno=1, **bad))
    with pytest.raises(O.OracleError):
        O.Oracle(dataclasses.replace(I.shock_tube_1d(20), tang_weno=1))


@pytest.mark.parametrize('gp', [2, 4])
def test_2d_y_invariant_equals_1d(gp):
    """Constant along y: the five segments carry the same states, every
    candidate is that state and the variant changes nothing against the 1D
    run (to the rounding of the normalised weights)."""
    p1 = I.shock_tube_1d(40)
    f = np.zeros((12, 5, 40))
    for a, b in ((0, 0), (1, 1), (3, 2), (4, 3), (5, 4), (7, 5)):
        f[a] = p1.fields[b][None]
    p2 = I.Problem('yinv', 2, 40, 5, 0.0, 1.0, 0.0, 1.0, f, bc=(I.FREE, I.FREE, I.PERIODIC, I.PERIODIC), cfl=0.4,
                   tang_weno=1, gauss_points=gp)
    a, b = O.Oracle(p1), O.Oracle(p2, threads=2)
    for _ in range(8):
        dt = a.cfl_dt()
        a.step(dt)
        b.step(dt)
    for a2, a1 in ((0, 0), (1, 1), (3, 2), (4, 3), (5, 4), (7, 5)):
        np.testing.assert_allclose(b.state[a2], np.broadcast_to(a.state[a1], b.state[a2].shape), rtol=1e-13,
                                   atol=5e-13)
    assert np.abs(b.state[[2, 6, 8, 9, 10, 11]]).max() < 1e-15


@pytest.mark.parametrize('gp', [2, 4])
def test_transpose_symmetry(gp):
    p = dataclasses.replace(I.shock_vortex_2d(24, 16, Rc=0.12), bc=(I.FREE, I.FREE, I.FREE, I.FREE), tang_weno=1,
                            gauss_points=gp)
    pt = dataclasses.replace(p, nx=p.ny, ny=p.nx, x0=p.y0, x1=p.y1, y0=p.x0, y1=p.x1,
                             fields=transpose_fields(p.fields))
    a, b = O.Oracle(p, threads=4), O.Oracle(pt, threads=4)
    for _ in range(3):
        dt = a.cfl_dt()
        assert dt == pytest.approx(b.cfl_dt(), rel=1e-15)
        a.step(dt)
        b.step(dt)
    np.testing.assert_allclose(transpose_fields(a.state), b.state, rtol=0, atol=1e-12)


def test_mach2_shock_vortex_without_weno_fallbacks():
    """Shock-vortex, M_s = 2, M_v = 0.5, 64 x 32, CFL 0.3, to t = 0.3: the
    scheme as read takes 5 WENO-state fallbacks, the variant none; both
    runs reach the end time."""
    counts = {}
    for tw in (0, 1):
        p = dataclasses.replace(I.shock_vortex_2d(64, 32, Ms=2.0, Mv=0.5, cfl=0.3), tang_weno=tw)
        o = O.Oracle(p, threads=8)
        o.advance_to(0.3)
        counts[tw] = o.counters()['guard_weno']
    assert counts[0] >= 1 and counts[1] == 0, counts
