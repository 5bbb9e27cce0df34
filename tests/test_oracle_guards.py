"""Pins of the oracle's two positivity guards (not in the paper; both keep a
step defined where a reconstructed point state is not a gas state):

* equilibrium guard: an inadmissible linearly reconstructed equilibrium state
  W0 (rho <= 0 or p <= 0) is replaced by the state the two initial
  half-Maxwellians carry to the interface, rho_l <psi>_{l,u>0} +
  rho_r <psi>_{r,u<0} (the collision state of Sec. 2.1's distribution at
  t = 0);
* WENO guard: an inadmissible nonlinear (WENO) point state falls back to the
  average of the cell on its side of the face.

The collision state is checked against brute-force velocity-space quadrature
(tests/kinetic_bruteforce.py); the face-level substitution against the
oracle's pinned building blocks on constructed line data; whole runs in which
both guards fire against conservation, symmetry and exact Riemann solutions.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I
from tests import kinetic_bruteforce as KB
from tests import riemann_exact

G = I.GAMMA


def cons1(rho, u, p):
    return np.array([rho, rho * u, p / (G - 1.0) + 0.5 * rho * u * u])


def cons2(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (G - 1.0) + 0.5 * rho * (u * u + v * v)])


def collision_state_bruteforce(Wl, Wr, dim):
    gl, gr = KB.Maxw(Wl, G, dim), KB.Maxw(Wr, G, dim)
    P = lambda u, v, s: KB.psi(u, v, s, dim)
    return gl.rho * gl.integrate(P, +1) + gr.rho * gr.integrate(P, -1)


@pytest.mark.parametrize('dim', [1, 2])
def test_equilibrium_guard_takes_the_collision_state(dim):
    """An inadmissible W0 (negative pressure, then negative density) is
    replaced by the collision state of the two sides: W0used equals its
    brute-force quadrature, and every output equals the evaluation with that
    state given as an admissible W0."""
    rng = np.random.default_rng(5)
    if dim == 1:
        Wl, Wr = cons1(0.9, 0.4, 0.8), cons1(0.3, -0.2, 0.25)
        bad = [cons1(0.5, 0.1, 1.0) - np.array([0.0, 0.0, 2.6]), np.array([-0.1, 0.02, 0.5])]
    else:
        Wl, Wr = cons2(0.9, 0.4, -0.3, 0.8), cons2(0.3, -0.2, 0.5, 0.25)
        bad = [cons2(0.5, 0.1, 0.2, 1.0) - np.array([0.0, 0.0, 0.0, 2.6]), np.array([-0.1, 0.02, 0.01, 0.5])]
    nc = dim + 2
    Wn, Wnn = 0.3 * rng.standard_normal(nc), 0.2 * rng.standard_normal(nc)
    extra = {}
    if dim == 2:
        extra = dict(W0t=0.3 * rng.standard_normal(nc), W0nt=0.1 * rng.standard_normal(nc),
                     W0tt=0.1 * rng.standard_normal(nc))
    S = collision_state_bruteforce(Wl, Wr, dim)
    dt = 2e-3
    for W0 in bad:
        r = O.gks_point_guarded(dim, G, dt, W0, Wn, Wnn, Wl, Wr, **extra)
        assert r['fired'] == 1
        np.testing.assert_allclose(r['W0used'], S, rtol=1e-11, atol=1e-13)
        ref = O.gks_point_guarded(dim, G, dt, S, Wn, Wnn, Wl, Wr, **extra)
        assert ref['fired'] == 0
        for k in ('F', 'Ft', 'Wt', 'Wtt', 'Nh', 'Nf'):
            np.testing.assert_allclose(r[k], ref[k], rtol=1e-9, atol=1e-11 * np.abs(ref[k]).max(), err_msg=k)
        assert r['tau'] == pytest.approx(ref['tau'], rel=1e-9)
    # an admissible W0 is used as given
    W0 = 0.5 * (Wl + Wr)
    r = O.gks_point_guarded(dim, G, dt, W0, Wn, Wnn, Wl, Wr, **extra)
    assert r['fired'] == 0 and np.array_equal(r['W0used'], W0)


def test_collision_state_of_equal_sides_is_that_state():
    """Closed form: with W_l = W_r the two half-space moments add up to the
    full moments of one Maxwellian, so the collision state is W_l itself."""
    W = cons1(0.7, 0.3, 0.6)
    r = O.gks_point_guarded(1, G, 1e-3, np.array([0.7, 0.2, -0.1]), np.zeros(3), np.zeros(3), W, W)
    assert r['fired'] == 1
    np.testing.assert_allclose(r['W0used'], W, rtol=1e-14)
    # a uniform state with zero slopes: the flux is the Euler flux
    u, p = 0.3, 0.6
    np.testing.assert_allclose(r['F'], [0.7 * u, 0.7 * u * u + p, u * (W[2] + p)], rtol=1e-12)


def _line_problem():
    return I.shock_tube_1d(100)


def _compose_face(prob, cells, dt):
    """The face from the oracle's pinned building blocks, with the guards
    applied as stated in the module docstring (stage 1)."""
    h = prob.dx
    ref = cells[:3, 1]
    P = np.empty((3, 3))
    Wl, Wr = np.empty(3), np.empty(3)
    for k in range(3):
        Q = cells[k] - ref[k]
        D = h * cells[3 + k]
        P[k] = O.p7(Q, D)
        Wl[k] = ref[k] + O.weno_left(Q, D, prob.weno_eps)
        Wr[k] = ref[k] + O.weno_right(Q, D, prob.weno_eps)
    nweno = 0
    if not (Wl[0] > 0 and I_pressure(Wl) > 0):
        Wl, nweno = cells[:3, 1].copy(), nweno + 1
    if not (Wr[0] > 0 and I_pressure(Wr) > 0):
        Wr, nweno = cells[:3, 2].copy(), nweno + 1
    W0 = ref + P[:, 0]
    r = O.gks_point_guarded(1, G, dt, W0, P[:, 1] / h, P[:, 2] / h ** 2, Wl, Wr,
                            tau_eps=prob.tau_eps, tau_C=prob.tau_C, mu=prob.mu)
    d0 = r['W0used'] - ref
    A = d0 + 0.5 * dt * r['Wt'] + dt * dt / 8.0 * r['Wtt'] + r['Nh']
    B = d0 + dt * r['Wt'] + dt * dt / 6.0 * r['Wtt'] + r['Nf']
    return np.array([r['F'], r['Ft'], A, B]), (r['fired'], nweno), Wl, Wr


def I_pressure(W):
    return (G - 1.0) * (W[2] - 0.5 * W[1] * W[1] / W[0])


def _quadratic_dip_cells(prob, depth):
    """rho and p follow a(x/h)^2 - depth around the face (x = 0), U = 0:
    every cell average is positive, the point values at the face are -depth.
    The reconstructions are exact on quadratics, so W0 and both WENO values
    are inadmissible."""
    h = prob.dx
    c = np.array([-1.5, -0.5, 0.5, 1.5])
    avg = c * c + 1.0 / 12.0 - depth
    grad = 2.0 * c / h
    rho, p = avg.copy(), 0.8 * avg
    E = p / (G - 1.0)
    return np.concatenate([np.stack([rho, 0.0 * rho, E]), np.stack([grad, 0.0 * grad, 0.8 * grad / (G - 1.0)])])


def test_face_guards_on_constructed_line_data():
    """Both guards at one face.  (a) A quadratic dip below zero at the face:
    W0 and both WENO values are inadmissible; the WENO states fall back to
    the two cell averages and W0 to their collision state (brute force).
    (b) A steep gradient in the left cell: only W0 is inadmissible and takes
    the collision state of the two WENO states.  The face results equal the
    composition from the pinned building blocks."""
    prob = _line_problem()
    dt = 1e-3
    cells = _quadratic_dip_cells(prob, 0.05)
    out, g = O.face_1d(prob, cells, dt)
    ref, g_ref, Wl, Wr = _compose_face(prob, cells, dt)
    assert g == (1, 2) == g_ref
    assert np.array_equal(Wl, cells[:3, 1]) and np.array_equal(Wr, cells[:3, 2])
    S = collision_state_bruteforce(Wl, Wr, 1)
    r = O.gks_point_guarded(1, G, dt, np.array([-1.0, 0.0, 1.0]), np.zeros(3), np.zeros(3), Wl, Wr)
    np.testing.assert_allclose(r["W0used"], S, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-15)

    W = np.array([cons1(1.0, 0.0, 1.0), cons1(0.2, 0.0, 0.2), cons1(0.05, 0.0, 0.05), cons1(0.05, 0.0, 0.05)]).T
    D = np.zeros((3, 4))
    D[:, 1] = 4.0 * (W[:, 2] - W[:, 0]) / (2.0 * prob.dx)
    cells = np.concatenate([W, D])
    out, g = O.face_1d(prob, cells, dt)
    ref, g_ref, Wl, Wr = _compose_face(prob, cells, dt)
    assert g == (1, 0) == g_ref
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(O.gks_point_guarded(1, G, dt, np.array([-1.0, 0.0, 1.0]), np.zeros(3), np.zeros(3),
                                                   Wl, Wr)['W0used'],
                               collision_state_bruteforce(Wl, Wr, 1), rtol=1e-11, atol=1e-15)
    # no guard on the smooth positive version of the dip
    out, g = O.face_1d(prob, _quadratic_dip_cells(prob, -0.5), dt)
    assert g == (0, 0)


def _expansion_exact(n, U, t):
    """Density cell averages of expansion_1d: the double rarefaction at
    x = 1/2 and the collision at x = 0 (= 1), before their waves meet."""
    L, R = (1.0, -U, 0.4), (1.0, U, 0.4)
    x = (np.arange(n) + 0.5) / n
    ex1 = riemann_exact.density_cell_averages(L, R, 0.0, 1.0, n, 0.5, t)
    ex2 = np.roll(riemann_exact.density_cell_averages(R, L, 0.5, 1.5, n, 1.0, t), -(n // 2))
    return np.where((x > 0.25) & (x < 0.75), ex1, ex2)


def test_strong_expansion_with_both_guards():
    """expansion_1d (U = 1.5 against a sound speed of 0.75) to t = 0.05: both
    guards fire (the near-vacuum and the collision), the run stays admissible,
    conserves mass, momentum and energy to rounding, stays mirror-symmetric
    about x = 1/2 to rounding, and converges to the exact solution (L1
    distance halves as the grid is refined)."""
    errs = []
    for n in (100, 200):
        p = I.expansion_1d(n, 1.5)
        o = O.Oracle(p)
        o.advance_to(0.05)
        st, t, _ = o.get_state()
        c = o.counters()
        assert c['guard_w0'] >= 30 and c['guard_weno'] >= 4, c
        assert st[0].min() > 0.0
        for k in range(3):
            assert abs(st[k].sum() - p.fields[k].sum()) / n < 1e-14 * max(1.0, np.abs(p.fields[k]).max())
        assert np.abs(st[0] - st[0][::-1]).max() < 1e-10
        assert np.abs(st[1] + st[1][::-1]).max() < 1e-10
        errs.append(np.abs(st[0] - _expansion_exact(n, 1.5, t)).mean())
    assert errs[0] < 0.016 and errs[1] < 0.55 * errs[0], errs


def test_pressure_ratio_300_tube_with_the_equilibrium_guard():
    """Riemann problem (1, 0, 30) | (0.125, 0, 0.1): the linear equilibrium
    state turns inadmissible at the shock front on most steps; with the
    guard the run reaches t = 0.1/sqrt(30) and converges to the exact
    solution."""
    L, R = (1.0, 0.0, 30.0), (0.125, 0.0, 0.1)
    t_end = 0.1 / np.sqrt(30.0)
    errs = []
    for n in (100, 200):
        p = I.riemann_1d(L, R, n, t_end=t_end)
        o = O.Oracle(p)
        o.advance_to(t_end)
        st, t, steps = o.get_state()
        assert t == t_end
        assert o.counters()['guard_w0'] >= steps // 2
        assert st[0].min() > 0.12 and st[0].max() < 1.01
        errs.append(np.abs(st[0] - riemann_exact.density_cell_averages(L, R, 0.0, 1.0, n, 0.5, t)).mean())
    assert errs[0] < 0.006 and errs[1] < 0.7 * errs[0], errs
