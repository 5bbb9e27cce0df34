"""Pins of the oracle's compact reconstructions (Sec. 3.2, 3.3) against what the
mathematics fixes: polynomial exactness, the linear-weight identity, smoothness
indicators integrated independently, and ENO behaviour at a jump."""
import math

import numpy as np
import pytest

from oracle import oracle as O

# scaled cells: I_{i-1}, I_i, I_{i+1}, I_{i+2} = [-3/2,-1/2], [-1/2,1/2], [1/2,3/2], [3/2,5/2]
CELLS = [(-1.5, -0.5), (-0.5, 0.5), (0.5, 1.5), (1.5, 2.5)]


def poly_data(coef):
    """cell averages and h*slope averages of sum coef[k] x^k on the 4 cells (exact)."""
    P = np.polynomial.Polynomial(coef)
    I = P.integ()
    Q = np.array([I(b) - I(a) for a, b in CELLS])
    D = np.array([P(b) - P(a) for a, b in CELLS])
    return P, Q, D


@pytest.mark.parametrize('seed', range(5))
def test_p7_exact_for_degree7(seed):
    rng = np.random.default_rng(seed)
    P, Q, D = poly_data(rng.normal(size=8))
    v, vx, vxx = O.p7(Q, D)
    assert v == pytest.approx(P(0.5), rel=1e-12, abs=1e-12)
    assert vx == pytest.approx(P.deriv()(0.5), rel=1e-12, abs=1e-11)
    assert vxx == pytest.approx(P.deriv(2)(0.5), rel=1e-12, abs=1e-10)


def test_p7_not_exact_for_degree8():
    # the value error of P7 on x^8 is a fixed nonzero constant (h^8 term)
    P, Q, D = poly_data([0] * 8 + [1.0])
    v, _, _ = O.p7(Q, D)
    assert abs(v - P(0.5)) > 1e-6


CAND_DEG = [2, 2, 3, 2, 2, 4, 4]


@pytest.mark.parametrize('k', range(7))
def test_candidates_exact_for_their_degree(k):
    rng = np.random.default_rng(10 + k)
    P, Q, D = poly_data(rng.normal(size=CAND_DEG[k] + 1))
    _, cand, _, _ = O.weno_left(Q, D, details=True)
    assert cand[k] == pytest.approx(P(0.5), rel=1e-13, abs=1e-13)
    # and not exact one degree higher (each stencil is used to its full degree)
    P2, Q2, D2 = poly_data(list(rng.normal(size=CAND_DEG[k] + 1)) + [1.0])
    _, cand2, _, _ = O.weno_left(Q2, D2, details=True)
    assert abs(cand2[k] - P2(0.5)) > 1e-6


def test_linear_weights_recover_p7():
    rng = np.random.default_rng(3)
    d = np.array([3, 5, 8, 7, 7, 34, 34]) / 98.0
    assert d.sum() == pytest.approx(1.0, abs=1e-15)
    for _ in range(10):
        Q, D = rng.normal(size=4), rng.normal(size=4)
        _, cand, _, _ = O.weno_left(Q, D, details=True)
        assert np.dot(d, cand) == pytest.approx(O.p7(Q, D)[0], abs=1e-13)
        # with a huge epsilon the nonlinear weights collapse to the linear ones
        assert O.weno_left(Q, D, eps=1e30) == pytest.approx(O.p7(Q, D)[0], abs=1e-13)
        assert O.weno_right(Q, D, eps=1e30) == pytest.approx(O.p7(Q, D)[0], abs=1e-13)


# sub-stencils as (kind, cell) conditions; beta_1 uses the cubic on
# {Q_{i-1}, Q_i, Q_{i+1}, Q'_{i-1}} (the symmetric replacement of Sec. 3.3)
STENCILS = [
    (2, [('a', 0), ('a', 1), ('s', 0)]),
    (3, [('a', 0), ('a', 1), ('a', 2), ('s', 0)]),
    (3, [('a', 1), ('a', 2), ('a', 3), ('s', 3)]),
    (2, [('a', 0), ('a', 1), ('a', 2)]),
    (2, [('a', 1), ('a', 2), ('a', 3)]),
    (4, [('a', 0), ('a', 1), ('a', 2), ('s', 0), ('s', 1)]),
    (4, [('a', 1), ('a', 2), ('a', 3), ('s', 2), ('s', 3)]),
]


def beta_bruteforce(k, Q, D):
    """Build the stencil polynomial by a direct solve and integrate
    sum_r int_{-1/2}^{1/2} (q^(r))^2 by Gauss-Legendre quadrature."""
    deg, conds = STENCILS[k]
    A = np.zeros((deg + 1, deg + 1))
    rhs = np.zeros(deg + 1)
    for r, (kind, m) in enumerate(conds):
        a, b = CELLS[m]
        for p in range(deg + 1):
            A[r, p] = (b ** (p + 1) - a ** (p + 1)) / (p + 1) if kind == 'a' else b ** p - a ** p
        rhs[r] = Q[m] if kind == 'a' else D[m]
    P = np.polynomial.Polynomial(np.linalg.solve(A, rhs))
    x, w = np.polynomial.legendre.leggauss(12)
    x, w = x / 2, w / 2
    return sum(float(np.dot(w, P.deriv(r)(x) ** 2)) for r in range(1, deg + 1))


@pytest.mark.parametrize('seed', range(4))
def test_smoothness_indicators_from_definition(seed):
    rng = np.random.default_rng(20 + seed)
    Q, D = rng.normal(size=4), rng.normal(size=4)
    _, _, beta, _ = O.weno_left(Q, D, details=True)
    for k in range(7):
        assert beta[k] == pytest.approx(beta_bruteforce(k, Q, D), rel=1e-11)


def test_indicators_shift_invariant_and_accurate_for_small_perturbations():
    # tiny perturbation on a large background: the indicators must see only the perturbation
    rng = np.random.default_rng(5)
    q, d = 1e-6 * rng.normal(size=4), 1e-6 * rng.normal(size=4)
    _, _, b1, _ = O.weno_left(q, d, details=True)
    _, _, b2, _ = O.weno_left(q + 1.0, d, details=True)
    np.testing.assert_allclose(b2, b1, rtol=1e-8)


def test_zref_is_fifth_order_for_smooth_data():
    def zref(h):
        f = lambda x: np.sin(1.0 + x)
        F = lambda x: -np.cos(1.0 + x)
        Q = np.array([(F(h * b) - F(h * a)) / h for a, b in CELLS])
        D = np.array([f(h * b) - f(h * a) for a, b in CELLS])
        _, _, beta, _ = O.weno_left(Q, D, details=True)
        return abs(3 * (beta[0] - beta[4]) + (beta[4] - beta[3])), beta
    z1, b1 = zref(0.02)
    z2, b2 = zref(0.01)
    assert math.log2(z1 / z2) == pytest.approx(5.0, abs=0.15)
    assert math.log2(b1[0] / b2[0]) == pytest.approx(2.0, abs=0.05)


def test_eno_at_a_jump():
    # jump between I_i and I_{i+1}: the left value comes from the left cells,
    # the right value from the right cells
    Q = np.array([0.0, 0.0, 1.0, 1.0])
    D = np.zeros(4)
    v, cand, beta, w = O.weno_left(Q, D, details=True)
    assert w[0] > 0.999 and abs(v) < 1e-3
    assert O.weno_right(Q, D) == pytest.approx(1.0, abs=1e-3)


def test_right_value_is_the_mirror_image():
    # smooth data reconstructed from the right must match a mirrored polynomial
    rng = np.random.default_rng(9)
    P, Q, D = poly_data(rng.normal(size=4))       # cubic: candidates 2,5,6 exact
    Pm = np.polynomial.Polynomial(P.coef * (-1.0) ** np.arange(4))   # p(-x)
    # mirrored about x = 1/2: cell k -> 3-k; value at 1/2 unchanged
    Pr = Pm(np.polynomial.Polynomial([-1.0, 1.0]))      # p(1 - x)
    Pr, Qr, Dr = poly_data(Pr.coef)
    assert O.weno_left(Qr, Dr) == pytest.approx(O.weno_right(Q, D), abs=1e-12)


@pytest.mark.parametrize('seed', range(3))
def test_tangential_sextic_exact(seed):
    """The 7-segment tangential polynomial (four Gauss points per face)
    reproduces any sextic from its unit-cell averages at offsets -3..3:
    value, first and second derivative at the 4-point Gauss-Legendre nodes."""
    rng = np.random.default_rng(40 + seed)
    P = np.polynomial.Polynomial(rng.normal(size=7))
    I = P.integ()
    s = np.array([I(m - 3 + 0.5) - I(m - 3 - 0.5) for m in range(7)])
    nodes = np.polynomial.legendre.leggauss(4)[0] / 2.0
    for eta in list(nodes) + [0.0]:
        v, d1, d2 = O.sextic(s, eta)
        assert v == pytest.approx(P(eta), abs=1e-11)
        assert d1 == pytest.approx(P.deriv()(eta), abs=1e-10)
        assert d2 == pytest.approx(P.deriv(2)(eta), abs=1e-9)


@pytest.mark.parametrize('seed', range(3))
def test_tangential_hermite_quintic_exact(seed):
    """The two-point tangential fit: the quintic fixed by the averages of a
    function and of its derivative over the three nearest unit segments
    (offsets -1..1) reproduces any quintic -- value, first and second
    derivative at the Gauss-Legendre nodes and elsewhere in the segment."""
    rng = np.random.default_rng(30 + seed)
    P = np.polynomial.Polynomial(rng.normal(size=6))
    I = P.integ()
    s = np.array([I(m + 0.5) - I(m - 0.5) for m in (-1, 0, 1)])
    d = np.array([P(m + 0.5) - P(m - 0.5) for m in (-1, 0, 1)])   # unit width: average of P'
    for eta in (-0.5 / math.sqrt(3), 0.5 / math.sqrt(3), 0.3, -0.5, 0.5):
        v, d1, d2 = O.hermite3(s, d, eta)
        assert v == pytest.approx(P(eta), abs=1e-12)
        assert d1 == pytest.approx(P.deriv()(eta), abs=1e-11)
        assert d2 == pytest.approx(P.deriv(2)(eta), abs=1e-10)
    # a sextic term is not reproduced (the fit has six conditions)
    Q = np.polynomial.Polynomial([0, 0, 0, 0, 0, 0, 1.0])
    J = Q.integ()
    s6 = np.array([J(m + 0.5) - J(m - 0.5) for m in (-1, 0, 1)])
    d6 = np.array([Q(m + 0.5) - Q(m - 0.5) for m in (-1, 0, 1)])
    assert abs(O.hermite3(s6, d6, 0.3)[0] - Q(0.3)) > 1e-4


@pytest.mark.parametrize('seed', range(3))
def test_tangential_quadratic_exact(seed):
    rng = np.random.default_rng(50 + seed)
    P = np.polynomial.Polynomial(rng.normal(size=3))
    I = P.integ()
    s = np.array([I(m + 0.5) - I(m - 0.5) for m in (-1, 0, 1)])
    for eta in (-0.5 / math.sqrt(3), 0.5 / math.sqrt(3), 0.3):
        v, d1, d2 = O.quadratic3(s, eta)
        assert v == pytest.approx(P(eta), abs=1e-13)
        assert d1 == pytest.approx(P.deriv()(eta), abs=1e-12)
        assert d2 == pytest.approx(P.deriv(2)(eta), abs=1e-12)


@pytest.mark.parametrize('seed', range(3))
def test_cross_face_cubic_exact(seed):
    """The cells' tangential gradients are carried to a face by the cubic
    through the averages of the 4 cells of the normal stencil: value and
    normal derivative at the face are exact for cubics; the value is the
    classic fourth-order (-1, 7, 7, -1)/12 and the derivative (1, -15, 15, -1)/12."""
    rng = np.random.default_rng(60 + seed)
    P = np.polynomial.Polynomial(rng.normal(size=4))
    I = P.integ()
    a = np.array([I(m - 0.5) - I(m - 1.5) for m in range(4)])   # cell m spans [m-3/2, m-1/2]
    v, d1 = O.cubic_face(a)
    assert v == pytest.approx(P(0.5), abs=1e-13)
    assert d1 == pytest.approx(P.deriv()(0.5), abs=1e-12)
    e = np.eye(4)
    assert np.allclose([O.cubic_face(e[m])[0] for m in range(4)], np.array([-1, 7, 7, -1]) / 12, atol=1e-15)
    assert np.allclose([O.cubic_face(e[m])[1] for m in range(4)], np.array([1, -15, 15, -1]) / 12, atol=1e-14)


def test_weno_weighted_slopes_exact_on_quadratics():
    """The evaluated side-slope variant: every candidate reproduces quadratics,
    and the nonlinear weights sum to one, so the WENO-weighted slopes of both
    sides equal the exact derivative of a quadratic at the interface (and the
    values its exact value), whatever the weights; on a jump the left slope
    comes from the smooth side."""
    rng = np.random.default_rng(11)
    xc = np.array([-1.0, 0.0, 1.0, 2.0])     # centres of cells i-1 .. i+2 (width 1, interface at 1/2)
    for _ in range(20):
        a, b, c = rng.standard_normal(3)
        q = lambda x: a + b * x + c * x * x
        Q = a + b * xc + c * (xc * xc + 1.0 / 12.0)       # cell averages
        D = q(xc + 0.5) - q(xc - 0.5)
        vl, dl, vr, dr = O.weno_slopes(Q, D)
        exact_d = b + 2.0 * c * 0.5
        scale = abs(a) + abs(b) + abs(c)
        assert abs(vl - q(0.5)) < 1e-13 * scale and abs(vr - q(0.5)) < 1e-13 * scale
        assert abs(dl - exact_d) < 1e-12 * scale and abs(dr - exact_d) < 1e-12 * scale
    # a jump between cells 2 and 3 (right of the interface's right cell): the
    # left side's slope is the smooth part's (here linear: slope 0.3)
    Q = np.array([1.0 - 0.3, 1.0, 1.0 + 0.3, 5.0])
    D = np.array([0.3, 0.3, 0.3, 0.0])
    vl, dl, _, _ = O.weno_slopes(Q, D)
    lin = O.p7(Q - Q[1], D)[1]                   # the linear derivative sees the jump
    assert abs(dl - 0.3) < 0.05 * abs(lin - 0.3) and abs(vl - 1.15) < 0.05 * abs(O.p7(Q - Q[1], D)[0] + Q[1] - 1.15)
