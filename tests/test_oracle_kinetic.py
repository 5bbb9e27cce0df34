"""Pins of the oracle's gas-kinetic evolution (Sec. 2) against brute-force
velocity-space quadrature, Euler-equation identities and a symbolic
Cauchy-Kowalewski expansion."""
import math

import numpy as np
import pytest
import sympy as sp

from oracle import oracle as O
from tests import kinetic_bruteforce as B

G = 1.4


def cons(dim, rho, U, V, p):
    if dim == 1:
        return np.array([rho, rho * U, p / (G - 1) + 0.5 * rho * U * U])
    return np.array([rho, rho * U, rho * V, p / (G - 1) + 0.5 * rho * (U * U + V * V)])


def euler_flux(W, dim):
    rho = W[0]
    U = W[1] / rho
    if dim == 1:
        p = (G - 1) * (W[2] - 0.5 * rho * U * U)
        return np.array([rho * U, rho * U * U + p, (W[2] + p) * U])
    V = W[2] / rho
    p = (G - 1) * (W[3] - 0.5 * rho * (U * U + V * V))
    return np.array([rho * U, rho * U * U + p, rho * U * V, (W[3] + p) * U])


def euler_flux_y(W):
    Wr = W[[0, 2, 1, 3]]
    return euler_flux(Wr, 2)[[0, 2, 1, 3]]


def jvp(fn, W, v, h=1e-30):
    """Jacobian-vector product by the complex step (exact to rounding)."""
    return np.imag(fn(W.astype(complex) + 1j * h * v)) / h


@pytest.mark.parametrize('half', [0, 1, -1])
def test_moments_against_quadrature(half):
    U, V, lam = 0.37, -0.21, 0.83
    for dim in (1, 2):
        W = cons(dim, 1.0, U, V, 1.0 / (2 * lam))
        g = B.Maxw(W, G, dim)
        for n in range(7):
            for m in (range(6) if dim == 2 else [0]):
                for k in range(3):
                    ref = g.integrate(lambda u, v, s: np.array([u ** n * v ** m * s ** k]), half)[0]
                    got = O.moment(dim, G, U, V, lam, half, n, m, k)
                    assert got == pytest.approx(ref, rel=1e-10, abs=1e-13), (dim, n, m, k)


def test_slope_solution_reproduces_rhs():
    rng = np.random.default_rng(1)
    for dim in (1, 2):
        W = cons(dim, 1.3, 0.4, -0.7, 0.9)
        b = rng.normal(size=dim + 2)
        a = O.slope(dim, G, W, b)
        g = B.Maxw(W, G, dim)
        back = g.integrate(lambda u, v, s: B.psi(u, v, s, dim) * B.a_of(a, u, v, s, dim))
        np.testing.assert_allclose(back, b, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize('dim', [1, 2])
def test_kfvs_split_and_equilibrium_flux(dim):
    # no slopes, W_l = W_r = W0: the two half-space fluxes sum to the full one
    # and the flux is the Euler flux at every tau
    W0 = cons(dim, 1.2, 0.5, -0.3, 0.8)
    z = np.zeros(dim + 2)
    for tau in (1e-4, 0.3, 5.0):
        Fh = O.flux_integral(dim, G, tau, 0.1, W0, z, W0, W0, W0t=z)
        np.testing.assert_allclose(Fh, 0.1 * euler_flux(W0, dim), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize('dim', [1, 2])
def test_flux_time_integral_against_bruteforce(dim):
    # shock-like data: distinct left/right states, nonzero slopes
    W0 = cons(dim, 1.0, 0.3, 0.1, 1.0)
    Wl = cons(dim, 1.3, 0.5, 0.15, 1.4)
    Wr = cons(dim, 0.8, 0.1, -0.05, 0.7)
    rng = np.random.default_rng(7)
    W0n = 0.3 * rng.normal(size=dim + 2)
    W0t = 0.2 * rng.normal(size=dim + 2) if dim == 2 else None
    for tau, tau_ce, delta in ((0.02, 0.0, 0.05), (0.04, 0.0, 0.025), (0.03, 0.02, 0.05)):
        got = O.flux_integral(dim, G, tau, delta, W0, W0n, Wl, Wr, W0t=W0t, tau_ce=tau_ce)
        ref = B.flux_time_integral(dim, G, tau, delta, W0, W0n, W0t, Wl, Wr, tau_ce=tau_ce)
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize('dim', [1, 2])
def test_interface_state_against_bruteforce(dim):
    W0 = cons(dim, 1.0, 0.3, 0.1, 1.0)
    Wl = cons(dim, 1.3, 0.5, 0.15, 1.4)
    Wr = cons(dim, 0.8, 0.1, -0.05, 0.7)
    rng = np.random.default_rng(8)
    W0n = 0.3 * rng.normal(size=dim + 2)
    W0t = 0.2 * rng.normal(size=dim + 2) if dim == 2 else None
    z = np.zeros(dim + 2)
    dt = 0.05
    r = O.gks_point(dim, G, dt, W0, W0n, z, Wl, Wr, W0t=W0t)
    # the collision time of Sec. 4 from the nonlinear states
    pl, pr = B.Maxw(Wl, G, dim).p, B.Maxw(Wr, G, dim).p
    tau_ce = abs((pl - pr) / (pl + pr)) * dt
    assert r['tau'] == pytest.approx(0.01 * dt + tau_ce, rel=1e-14)
    for t, N in ((0.5 * dt, r['Nh']), (dt, r['Nf'])):
        ref = B.state_at(dim, G, r['tau'], t, W0, W0n, W0t, Wl, Wr, tau_ce=tau_ce)
        np.testing.assert_allclose(W0 + t * r['Wt'] + N, ref, rtol=1e-9, atol=1e-12)
    # the extracted F, Ft reproduce both time integrals of a linear-in-time flux
    # fit; the pressure-jump part of tau is the Chapman-Enskog collision time
    Fh = B.flux_time_integral(dim, G, r['tau'], 0.5 * dt, W0, W0n, W0t, Wl, Wr, tau_ce=tau_ce)
    Ff = B.flux_time_integral(dim, G, r['tau'], dt, W0, W0n, W0t, Wl, Wr, tau_ce=tau_ce)
    np.testing.assert_allclose(r['F'] * 0.5 * dt + r['Ft'] * dt * dt / 8, Fh, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r['F'] * dt + r['Ft'] * dt * dt / 2, Ff, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize('dim', [1, 2])
def test_viscous_collision_time_and_flux_against_bruteforce(dim):
    """Navier-Stokes (Sec. 4, viscous form): tau = mu/p0 + C|dp/sum p| dt with
    p0 the pressure of the interface equilibrium, used in both roles; the
    whole distribution integrated by brute force with tau_ce = tau."""
    W0 = cons(dim, 1.0, 0.3, 0.1, 1.0)
    Wl = cons(dim, 1.3, 0.5, 0.15, 1.4)
    Wr = cons(dim, 0.8, 0.1, -0.05, 0.7)
    rng = np.random.default_rng(9)
    W0n = 0.3 * rng.normal(size=dim + 2)
    W0t = 0.2 * rng.normal(size=dim + 2) if dim == 2 else None
    z = np.zeros(dim + 2)
    dt, mu = 0.05, 0.004
    r = O.gks_point(dim, G, dt, W0, W0n, z, Wl, Wr, W0t=W0t, mu=mu)
    pl, pr, p0 = B.Maxw(Wl, G, dim).p, B.Maxw(Wr, G, dim).p, B.Maxw(W0, G, dim).p
    tau = mu / p0 + abs((pl - pr) / (pl + pr)) * dt
    assert r['tau'] == pytest.approx(tau, rel=1e-14)
    Fh = B.flux_time_integral(dim, G, tau, 0.5 * dt, W0, W0n, W0t, Wl, Wr, tau_ce=tau)
    Ff = B.flux_time_integral(dim, G, tau, dt, W0, W0n, W0t, Wl, Wr, tau_ce=tau)
    np.testing.assert_allclose(r['F'] * 0.5 * dt + r['Ft'] * dt * dt / 8, Fh, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r['F'] * dt + r['Ft'] * dt * dt / 2, Ff, rtol=1e-9, atol=1e-12)
    for t, N in ((0.5 * dt, r['Nh']), (dt, r['Nf'])):
        ref = B.state_at(dim, G, tau, t, W0, W0n, W0t, Wl, Wr, tau_ce=tau)
        np.testing.assert_allclose(W0 + t * r['Wt'] + N, ref, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize('dim', [1, 2])
def test_smooth_limit_is_the_euler_flux_and_its_ck_derivative(dim):
    """W_l = W_r = W0 with shared slopes: the flux is F(W0) + t F_t exactly with
    F_t = dF/dW . W_t and W_t = -(dF/dW W_n + dG/dW W_t); no remainder."""
    W0 = cons(dim, 1.1, 0.4, -0.25, 0.9)
    rng = np.random.default_rng(11)
    W0n = 0.2 * rng.normal(size=dim + 2)
    W0t = 0.15 * rng.normal(size=dim + 2) if dim == 2 else None
    z = np.zeros(dim + 2)
    dt = 0.01
    r = O.gks_point(dim, G, dt, W0, W0n, z, W0, W0, W0t=W0t)
    f = lambda W: euler_flux(W, dim)
    Wt = -jvp(f, W0, W0n)
    if dim == 2:
        Wt = Wt - jvp(euler_flux_y, W0, W0t)
    np.testing.assert_allclose(r['Wt'], Wt, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r['F'], euler_flux(W0, dim), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r['Ft'], jvp(f, W0, Wt), rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(r['Nh'], 0.0, atol=1e-30)
    np.testing.assert_allclose(r['Nf'], 0.0, atol=1e-30)
    # the time integral is exactly F delta + Ft delta^2 / 2
    for delta in (dt, 0.5 * dt, 0.37 * dt):
        Fh = O.flux_integral(dim, G, r['tau'], delta, W0, W0n, W0, W0, W0t=W0t)
        np.testing.assert_allclose(Fh, r['F'] * delta + r['Ft'] * delta ** 2 / 2, rtol=1e-12, atol=1e-16)


def _ce_flux(dim, W0, W0n, W0t=None, tau_ce=0.01, delta=0.05):
    """Chapman-Enskog part of the flux time integral over [0, delta] per unit
    time: the difference the tau_ce term makes, everything else equal."""
    z = np.zeros(dim + 2)
    f1 = O.flux_integral(dim, G, 0.02, delta, W0, W0n, W0, W0, W0t=W0t, tau_ce=tau_ce)
    f0 = O.flux_integral(dim, G, 0.02, delta, W0, W0n, W0, W0, W0t=W0t)
    return (f1 - f0) / delta


def test_chapman_enskog_term_is_the_navier_stokes_flux():
    """The BGK Chapman-Enskog flux with mu = tau p (Prandtl number 1): viscous
    stress -tau p [2 U_x - 2/(K + dim) div U] on the normal momentum, shear
    -tau p (U_y + V_x), viscous work U times the stress, heat flux
    -tau p (K + dim + 2)/2 d(p/rho)/dx, nothing on the mass; K the internal
    degrees of freedom (4 in 1D, 3 in 2D at gamma = 1.4)."""
    t = 0.013
    # 1D normal stress and its work: rho, p uniform, U = 0.4 with U_x = 0.7
    rho, U, p, Ux = 1.1, 0.4, 0.9, 0.7
    K1 = (3 - G) / (G - 1)
    W0 = cons(1, rho, U, 0, p)
    W0n = np.array([0.0, rho * Ux, rho * U * Ux])
    s = -t * p * (2 * Ux - 2 / (K1 + 1) * Ux)
    np.testing.assert_allclose(_ce_flux(1, W0, W0n, tau_ce=t), [0.0, s, U * s], rtol=1e-11, atol=1e-15)
    # 1D heat flux: U = 0, p uniform, rho_x = -0.6
    rx = -0.6
    W0 = cons(1, rho, 0.0, 0, p)
    W0n = np.array([rx, 0.0, 0.0])
    q = -t * p * (K1 + 3) / 2 * (-p * rx / rho ** 2)
    np.testing.assert_allclose(_ce_flux(1, W0, W0n, tau_ce=t), [0.0, 0.0, q], rtol=1e-11, atol=1e-15)
    # 2D at rest, rho and p uniform: U_x, V_y (normal stress), V_x, U_y (shear)
    K2 = (4 - 2 * G) / (G - 1)
    Ux, Vy, Vx, Uy = 0.5, -0.3, 0.25, 0.45
    W0 = cons(2, rho, 0.0, 0.0, p)
    W0n = np.array([0.0, rho * Ux, rho * Vx, 0.0])
    W0t = np.array([0.0, rho * Uy, rho * Vy, 0.0])
    sxx = -t * p * (2 * Ux - 2 / (K2 + 2) * (Ux + Vy))
    sxy = -t * p * (Uy + Vx)
    np.testing.assert_allclose(_ce_flux(2, W0, W0n, W0t, tau_ce=t), [0.0, sxx, sxy, 0.0], rtol=1e-11, atol=1e-15)


def _symbolic_wtt(W0, Wx, Wy, Wxx, Wxy, Wyy):
    x, y = sp.symbols('x y')
    W = [W0[c] + Wx[c] * x + Wy[c] * y + sp.Rational(1, 2) * Wxx[c] * x * x + Wxy[c] * x * y
         + sp.Rational(1, 2) * Wyy[c] * y * y for c in range(4)]
    g = sp.Rational(7, 5)

    def FG(w):
        r, m, n, E = w
        p = (g - 1) * (E - (m * m + n * n) / (2 * r))
        return [m, m * m / r + p, m * n / r, (E + p) * m / r], [n, m * n / r, n * n / r + p, (E + p) * n / r]

    F, Gy = FG(W)
    Wt = [-(sp.diff(F[c], x) + sp.diff(Gy[c], y)) for c in range(4)]
    e = sp.symbols('e')
    Fe, Ge = FG([W[c] + e * Wt[c] for c in range(4)])
    Ft = [sp.diff(Fe[c], e).subs(e, 0) for c in range(4)]
    Gt = [sp.diff(Ge[c], e).subs(e, 0) for c in range(4)]
    Wtt = [-(sp.diff(Ft[c], x) + sp.diff(Gt[c], y)) for c in range(4)]
    return np.array([float(sp.N(w.subs({x: 0, y: 0}), 30)) for w in Wtt])


def test_euler_second_time_derivative_symbolic():
    rng = np.random.default_rng(4)
    W0 = cons(2, 1.2, 0.3, -0.4, 0.9)
    d = [0.3 * rng.normal(size=4) for _ in range(5)]
    got = O.euler_wtt(G, W0, *d)
    ref = _symbolic_wtt(W0, *d)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-13)


def test_entropy_wave_wtt():
    # rho = rho(x - U t), U, p uniform: W_tt = U^2 W_xx
    U = 0.7
    W0 = cons(2, 1.1, U, 0.0, 1.0)
    rx, rxx = 0.3, -0.8
    Wx = np.array([rx, rx * U, 0.0, 0.5 * rx * U * U])
    Wxx = np.array([rxx, rxx * U, 0.0, 0.5 * rxx * U * U])
    z = np.zeros(4)
    np.testing.assert_allclose(O.euler_wtt(G, W0, Wx, z, Wxx, z, z), U * U * Wxx, rtol=1e-13, atol=1e-15)


def test_1d_is_2d_without_y_dependence():
    W1 = cons(1, 1.05, 0.6, 0.0, 0.95)
    W2 = cons(2, 1.05, 0.6, 0.0, 0.95)
    rng = np.random.default_rng(12)
    g1 = 0.2 * rng.normal(size=3)
    gg1 = 0.1 * rng.normal(size=3)
    to2 = lambda v: np.array([v[0], v[1], 0.0, v[2]])
    Wl1, Wr1 = cons(1, 1.2, 0.7, 0, 1.1), cons(1, 0.9, 0.5, 0, 0.8)
    r1 = O.gks_point(1, G, 0.02, W1, g1, gg1, Wl1, Wr1)
    r2 = O.gks_point(2, G, 0.02, W2, to2(g1), to2(gg1), to2(Wl1), to2(Wr1), W0t=np.zeros(4))
    for k in ('F', 'Ft', 'Wt', 'Wtt', 'Nh', 'Nf'):
        np.testing.assert_allclose(to2(r1[k]), r2[k], rtol=1e-12, atol=1e-14)
