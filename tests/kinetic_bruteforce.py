"""Brute-force velocity-space quadrature of the gas-kinetic quantities, written
independently of the oracle for its pins.  Integrals over u use Gauss-Hermite
nodes on the full line and composite Gauss-Legendre on a truncated half line;
v uses Gauss-Hermite; the K internal degrees of freedom enter through
s = xi^2, whose density under a Maxwellian is a Gamma(K/2, 1/lambda) law,
integrated with generalized Gauss-Laguerre nodes.  Time integrals use
adaptive quadrature.  No moment recursion or closed form is used."""
import math

import numpy as np
from scipy import integrate, special


def K_of(dim, gamma):
    # total translational + internal DOF: gamma = (K + dim + 2)/(K + dim)
    return 2.0 / (gamma - 1.0) - dim


class Maxw:
    def __init__(self, W, gamma, dim):
        self.dim = dim
        self.rho = W[0]
        self.U = W[1] / W[0]
        self.V = W[2] / W[0] if dim == 2 else 0.0
        E = W[dim + 1]
        ke = 0.5 * self.rho * (self.U ** 2 + self.V ** 2)
        self.p = (gamma - 1.0) * (E - ke)
        self.lam = self.rho / (2.0 * self.p)
        self.K = K_of(dim, gamma)
        a = self.K / 2.0 - 1.0
        x, w = special.roots_genlaguerre(8, a)
        self.s = x / self.lam
        self.ws = w / special.gamma(a + 1.0)

    def _u_nodes(self, half):
        lam, U = self.lam, self.U
        if half == 0:
            x, w = np.polynomial.hermite.hermgauss(80)
            return U + x / math.sqrt(lam), w / math.sqrt(math.pi)
        L = abs(U) + 14.0 / math.sqrt(lam)
        lo, hi = (0.0, L) if half > 0 else (-L, 0.0)
        x, w = np.polynomial.legendre.leggauss(64)
        edges = np.linspace(lo, hi, 9)
        us, ws = [], []
        for a, b in zip(edges[:-1], edges[1:]):
            us.append(0.5 * (b - a) * x + 0.5 * (a + b))
            ws.append(0.5 * (b - a) * w)
        u = np.concatenate(us)
        wt = np.concatenate(ws) * math.sqrt(lam / math.pi) * np.exp(-lam * (u - U) ** 2)
        return u, wt

    def integrate(self, h, half=0):
        """(1/rho) int h(u, v, s) g du dv dxi; h maps node arrays to (ncomp, ...)."""
        u, wu = self._u_nodes(half)
        if self.dim == 2:
            x, w = np.polynomial.hermite.hermgauss(40)
            v, wv = self.V + x / math.sqrt(self.lam), w / math.sqrt(math.pi)
        else:
            v, wv = np.zeros(1), np.ones(1)
        U_, V_, S_ = np.meshgrid(u, v, self.s, indexing='ij')
        W_ = wu[:, None, None] * wv[None, :, None] * self.ws[None, None, :]
        vals = np.asarray(h(U_, V_, S_))
        return np.tensordot(vals, W_, axes=([-3, -2, -1], [0, 1, 2]))


def psi(u, v, s, dim):
    one = np.ones_like(u)
    if dim == 1:
        return np.array([one, u, 0.5 * (u * u + s)])
    return np.array([one, u, v, 0.5 * (u * u + v * v + s)])


def a_of(a, u, v, s, dim):
    return np.tensordot(a, psi(u, v, s, dim), axes=(0, 0))


def slope(g, b):
    """solve <psi a> = b with the moment matrix integrated numerically"""
    dim = g.dim
    M = g.integrate(lambda u, v, s: psi(u, v, s, dim)[:, None] * psi(u, v, s, dim)[None, :])
    return np.linalg.solve(M, b)


def _setup(dim, gamma, W0, W0n, W0t, Wl, Wr):
    W0, W0n, Wl, Wr = map(np.asarray, (W0, W0n, Wl, Wr))
    W0t = np.zeros_like(W0) if W0t is None else np.asarray(W0t)
    g0, gl, gr = Maxw(W0, gamma, dim), Maxw(Wl, gamma, dim), Maxw(Wr, gamma, dim)
    z = np.zeros(dim + 2)
    an0 = slope(g0, W0n / W0[0])
    at0 = slope(g0, W0t / W0[0]) if dim == 2 else z
    anl = slope(gl, W0n / Wl[0])
    atl = slope(gl, W0t / Wl[0]) if dim == 2 else z
    anr = slope(gr, W0n / Wr[0])
    atr = slope(gr, W0t / Wr[0]) if dim == 2 else z
    # compatibility: <psi (a_n u + a_t v + A)>_0 = 0
    bA = -g0.integrate(lambda u, v, s: psi(u, v, s, dim) * (a_of(an0, u, v, s, dim) * u + a_of(at0, u, v, s, dim) * v))
    A0 = slope(g0, bA)
    return g0, gl, gr, an0, at0, anl, atl, anr, atr, A0


def flux_time_integral(dim, gamma, tau, delta, W0, W0n, W0t, Wl, Wr, tau_ce=0.0):
    """int_0^delta int u psi f dXi dt for the second-order interface distribution
    (the third-order simplified distribution without a_tt, a_xt, a_yt), with
    tau in exp(-t/tau) and tau_ce in the Chapman-Enskog term
    -tau_ce (a_n u + a_t v + A) g0."""
    g0, gl, gr, an0, at0, anl, atl, anr, atr, A0 = _setup(dim, gamma, W0, W0n, W0t, Wl, Wr)
    T = lambda fn: integrate.quad(fn, 0.0, delta, epsabs=1e-300, epsrel=1e-13, limit=200)[0]
    t_g0 = T(lambda t: 1.0 - math.exp(-t / tau))
    t_A = T(lambda t: t - tau_ce)
    t_s0 = T(lambda t: math.exp(-t / tau) * t - tau_ce)
    t_lr = T(lambda t: math.exp(-t / tau))
    t_slr = T(lambda t: -math.exp(-t / tau) * t)
    up = lambda u, v, s: u * psi(u, v, s, dim)
    sl = lambda a_n, a_t: (lambda u, v, s: up(u, v, s) * (a_of(a_n, u, v, s, dim) * u + a_of(a_t, u, v, s, dim) * v))
    F = g0.rho * (t_g0 * g0.integrate(up)
                  + t_A * g0.integrate(lambda u, v, s: up(u, v, s) * a_of(A0, u, v, s, dim))
                  + t_s0 * g0.integrate(sl(an0, at0)))
    F = F + t_lr * (gl.rho * gl.integrate(up, +1) + gr.rho * gr.integrate(up, -1))
    F = F + t_slr * (gl.rho * gl.integrate(sl(anl, atl), +1) + gr.rho * gr.integrate(sl(anr, atr), -1))
    return F


def state_at(dim, gamma, tau, t, W0, W0n, W0t, Wl, Wr, tau_ce=0.0):
    """int psi f(t) dXi of the second-order interface distribution (no a_tt
    term); the Chapman-Enskog term integrates to zero by compatibility but is
    kept here as it stands."""
    g0, gl, gr, an0, at0, anl, atl, anr, atr, A0 = _setup(dim, gamma, W0, W0n, W0t, Wl, Wr)
    E = math.exp(-t / tau)
    P = lambda u, v, s: psi(u, v, s, dim)
    sl = lambda a_n, a_t: (lambda u, v, s: P(u, v, s) * (a_of(a_n, u, v, s, dim) * u + a_of(a_t, u, v, s, dim) * v))
    W = g0.rho * (g0.integrate(P) + t * g0.integrate(lambda u, v, s: P(u, v, s) * a_of(A0, u, v, s, dim)))
    W = W - tau_ce * g0.rho * (g0.integrate(sl(an0, at0)) + g0.integrate(lambda u, v, s: P(u, v, s) * a_of(A0, u, v, s, dim)))
    W = W - E * g0.rho * (g0.integrate(P) - t * g0.integrate(sl(an0, at0)))
    W = W + E * gl.rho * (gl.integrate(P, +1) - t * gl.integrate(sl(anl, atl), +1))
    W = W + E * gr.rho * (gr.integrate(P, -1) - t * gr.integrate(sl(anr, atr), -1))
    return W
