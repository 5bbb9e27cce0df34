"""Seeded synthetic workloads: initial conditions and exact solutions.

This module holds no part of the scheme's arithmetic.  It turns analytic
initial conditions into the two kinds of data the compact scheme evolves --
cell averages and cell-averaged gradients of the conservative variables -- and
evaluates exact solutions for error norms.  Both the oracle and the GPU path
take their inputs from here.

Conventions (shared with the C interfaces):
  * 1D fields: [rho, rhoU, rhoE, (rho)_x, (rhoU)_x, (rhoE)_x], each (nx,)
  * 2D fields: [W(4), W_x(4), W_y(4)], W = (rho, rhoU, rhoV, rhoE), each (ny, nx)
  * boundary codes: 0 periodic, 1 free, 2 wall, 3 inflow (xlo, xhi, ylo, yhi)

Cell averages use Gauss-Legendre quadrature (closed forms where they exist);
the cell-averaged gradient of cell i is, by the Gauss theorem, the difference
of the interface values (1D) or interface line averages (2D) divided by the
cell width.  A discontinuity lying on a cell face is evaluated as the limit
from inside each cell.
"""
from __future__ import annotations

import dataclasses
import math

from scipy.special import erf as _erf
from typing import Callable, List, Optional, Sequence

import numpy as np

GAMMA = 1.4
PERIODIC, FREE, WALL, INFLOW, NOSLIP = 0, 1, 2, 3, 4


@dataclasses.dataclass
class Problem:
    """A complete initial-value problem for the solver."""
    name: str
    dim: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    fields: np.ndarray            # (6, nx) or (12, ny, nx), float64
    bc: Sequence[int] = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    inflow_prim: Optional[np.ndarray] = None   # (4, 4): (rho, U, V, p) per side
    gamma: float = GAMMA
    cfl: float = 0.3
    t_end: float = 0.0
    steps: int = 0                # fixed step count (0: run to t_end)
    fixed_dt: float = 0.0
    weno_eps: float = 1e-6
    tau_eps: float = 0.01
    tau_C: float = 1.0
    mu: float = 0.0               # dynamic viscosity (0: Euler equations)
    gauss_points: int = 2         # 2D: Gauss points per face segment (2: quartic on 5 segments, 4: sextic on 7)
    recon_vars: int = 0           # variables of the WENO-Z states: 0 conservative, 1 characteristic
    side_slopes: int = 0          # 1 = WENO-weighted slopes of the non-equilibrium sides (evaluated variant)
    tang_weno: int = 0            # 1 = tangential WENO-Z of the WENO-Z states (evaluated variant, 2D two points)
    exact: Optional[Callable[[float], np.ndarray]] = None   # t -> exact fields (cell averages)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny if self.dim == 2 else 1.0

    @property
    def ncells(self) -> int:
        return self.nx * self.ny

    def config_dict(self) -> dict:
        inflow = self.inflow_prim if self.inflow_prim is not None else np.zeros((4, 4))
        return dict(dim=self.dim, nx=self.nx, ny=self.ny, x0=self.x0, x1=self.x1, y0=self.y0,
                    y1=self.y1, gamma=self.gamma, cfl=self.cfl, bc=list(self.bc),
                    inflow_prim=np.asarray(inflow, dtype=np.float64).tolist(),
                    weno_eps=self.weno_eps, tau_eps=self.tau_eps, tau_C=self.tau_C,
                    fixed_dt=self.fixed_dt, mu=self.mu, gauss_points=self.gauss_points,
                    recon_vars=self.recon_vars, side_slopes=self.side_slopes, tang_weno=self.tang_weno)


# ---------------------------------------------------------------- helpers

_GL_X, _GL_W = np.polynomial.legendre.leggauss(8)
_GL_W = _GL_W / 2.0          # weights for an average over [-1/2, 1/2]
_GL_X = _GL_X / 2.0


def prim_to_cons(rho, U, V, p, gamma=GAMMA, dim=2):
    if dim == 1:
        return np.stack([rho, rho * U, p / (gamma - 1.0) + 0.5 * rho * U * U])
    return np.stack([rho, rho * U, rho * V, p / (gamma - 1.0) + 0.5 * rho * (U * U + V * V)])


def _cell_fields_1d(cons_fn, x0, x1, nx, closed_avg=None, closed_face=None):
    """cons_fn(x, side) -> (3, ...) conservative state; side = -1/+1 at faces."""
    dx = (x1 - x0) / nx
    xc = x0 + (np.arange(nx) + 0.5) * dx
    if closed_avg is not None:
        W = closed_avg(xc, dx)
    else:
        pts = xc[None, :] + _GL_X[:, None] * dx
        vals = cons_fn(pts, 0)                          # (3, 8, nx)
        W = np.einsum('q,cqn->cn', _GL_W, vals)
    if closed_face is not None:
        right = closed_face(xc + 0.5 * dx, -1)
        left = closed_face(xc - 0.5 * dx, +1)
    else:
        right = cons_fn(xc + 0.5 * dx, -1)
        left = cons_fn(xc - 0.5 * dx, +1)
    G = (right - left) / dx
    return np.concatenate([W, G]).astype(np.float64)


def _cell_fields_2d(prim_fn, x0, x1, y0, y1, nx, ny, gamma=GAMMA, row_block=64):
    """prim_fn(x, y, sx, sy) -> (rho, U, V, p); sx/sy = -1/+1 select one-sided
    limits at faces, 0 otherwise."""
    dx = (x1 - x0) / nx
    dy = (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    out = np.empty((12, ny, nx), dtype=np.float64)

    def cons(x, y, sx, sy):
        r, U, V, p = prim_fn(x, y, sx, sy)
        return prim_to_cons(r, U, V, p, gamma, 2)

    for j0 in range(0, ny, row_block):
        j1 = min(ny, j0 + row_block)
        yc = y0 + (np.arange(j0, j1) + 0.5) * dy
        # cell averages: 8x8 Gauss-Legendre
        acc = np.zeros((4, j1 - j0, nx))
        for qy, wy in zip(_GL_X, _GL_W):
            Y = (yc + qy * dy)[:, None]
            for qx, wx in zip(_GL_X, _GL_W):
                X = (xc + qx * dx)[None, :]
                acc += wy * wx * cons(X + 0 * Y, Y + 0 * X, 0, 0)
        out[0:4, j0:j1] = acc
        # x gradients: line averages over the x faces of each cell
        gx = np.zeros((4, j1 - j0, nx))
        for qy, wy in zip(_GL_X, _GL_W):
            Y = (yc + qy * dy)[:, None]
            Xr = (xc + 0.5 * dx)[None, :]
            Xl = (xc - 0.5 * dx)[None, :]
            gx += wy * (cons(Xr + 0 * Y, Y + 0 * Xr, -1, 0) - cons(Xl + 0 * Y, Y + 0 * Xl, +1, 0))
        out[4:8, j0:j1] = gx / dx
        # y gradients
        gy = np.zeros((4, j1 - j0, nx))
        for qx, wx in zip(_GL_X, _GL_W):
            X = (xc + qx * dx)[None, :]
            Yt = (yc + 0.5 * dy)[:, None]
            Yb = (yc - 0.5 * dy)[:, None]
            gy += wx * (cons(X + 0 * Yt, Yt + 0 * X, 0, -1) - cons(X + 0 * Yb, Yb + 0 * X, 0, +1))
        out[8:12, j0:j1] = gy / dy
    return out


def _min_image(d, L):
    return d - L * np.round(d / L)


def vortex_prim(x, y, xv, yv, Mv, Rc, rho_inf, U_inf, V_inf, p_inf, gamma=GAMMA, Lx=None, Ly=None):
    """Isentropic vortex scaled to a background state (u_theta = Mv c r e^{(1-r^2)/2},
    r = distance / Rc, T/T_inf = 1 - (gamma-1)/2 Mv^2 e^{1-r^2})."""
    dxv = x - xv
    dyv = y - yv
    if Lx is not None:
        dxv = _min_image(dxv, Lx)
    if Ly is not None:
        dyv = _min_image(dyv, Ly)
    c_inf = math.sqrt(gamma * p_inf / rho_inf)
    r2 = (dxv * dxv + dyv * dyv) / (Rc * Rc)
    e = np.exp(1.0 - r2)
    T = 1.0 - 0.5 * (gamma - 1.0) * Mv * Mv * e
    rho = rho_inf * T ** (1.0 / (gamma - 1.0))
    p = p_inf * T ** (gamma / (gamma - 1.0))
    # u_theta / dist = Mv c e^{(1-r^2)/2} / Rc
    f = Mv * c_inf * np.exp(0.5 * (1.0 - r2)) / Rc
    U = U_inf - f * dyv
    V = V_inf + f * dxv
    return rho, U, V, p


# ---------------------------------------------------------------- 1D workloads

def sine_wave_1d(n: int, eps: float = 0.2, cfl: float = 0.3, t_end: float = 2.0,
                 fixed_dt: float = 0.0, gamma: float = GAMMA) -> Problem:
    """rho = 1 + eps sin(pi x), U = 1, p = 1 on periodic [0, 2] (advection of a
    density perturbation, Sec. 4.1); the exact solution is the translated wave.
    Cell averages and gradients use closed forms."""
    x0, x1 = 0.0, 2.0

    def avg(xc, dx, shift=0.0):
        s = 2.0 * math.sin(math.pi * dx / 2.0) / (math.pi * dx)
        rho = 1.0 + eps * s * np.sin(math.pi * (xc - shift))
        return np.stack([rho, rho, 1.0 / (gamma - 1.0) + 0.5 * rho])

    def grad(xc, dx, shift=0.0):
        g = eps * 2.0 * np.cos(math.pi * (xc - shift)) * math.sin(math.pi * dx / 2.0) / dx
        return np.stack([g, g, 0.5 * g])

    dx = (x1 - x0) / n
    xc = x0 + (np.arange(n) + 0.5) * dx
    fields = np.concatenate([avg(xc, dx), grad(xc, dx)]).astype(np.float64)

    def exact(t):
        return np.concatenate([avg(xc, dx, t), grad(xc, dx, t)])

    return Problem('sine_wave_1d', 1, n, 1, x0, x1, 0.0, 1.0, fields, cfl=cfl, t_end=t_end,
                   fixed_dt=fixed_dt, gamma=gamma, exact=exact, meta=dict(eps=eps))


def shock_entropy_1d(n: int = 400, t_end: float = 1.8, cfl: float = 0.3) -> Problem:
    """Shock-entropy interaction on [-5, 5]: (3.857143, 2.629369, 10.33333) for
    x < -4, rho = 1 + 0.2 sin(5x), U = 0, p = 1 otherwise.  Left side: fixed
    post-shock inflow; right side: free flow."""
    x0, x1 = -5.0, 5.0
    left = (3.857143, 2.629369, 10.33333)

    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        is_left = (x < -4.0) | ((x == -4.0) & (np.asarray(side) < 0))
        rho = np.where(is_left, left[0], 1.0 + 0.2 * np.sin(5.0 * x))
        U = np.where(is_left, left[1], 0.0)
        p = np.where(is_left, left[2], 1.0)
        return prim_to_cons(rho, U, 0.0 * U, p, GAMMA, 1)

    fields = _cell_fields_1d(cons, x0, x1, n)
    inflow = np.zeros((4, 4))
    inflow[0] = (left[0], left[1], 0.0, left[2])
    return Problem('shock_entropy_1d', 1, n, 1, x0, x1, 0.0, 1.0, fields,
                   bc=(INFLOW, FREE, PERIODIC, PERIODIC), inflow_prim=inflow, cfl=cfl, t_end=t_end)


def shock_tube_1d(n: int = 100, t_end: float = 0.16, cfl: float = 0.3) -> Problem:
    """Riemann problem (0.445, 0.698, 3.528) | (0.5, 0, 0.571) at x = 0.5 on [0, 1]
    with free-flow boundaries (Sec. 4.4)."""
    left, right = (0.445, 0.698, 3.528), (0.5, 0.0, 0.571)

    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        is_left = (x < 0.5) | ((x == 0.5) & (np.asarray(side) < 0))
        st = [np.where(is_left, a, b) for a, b in zip(left, right)]
        return prim_to_cons(st[0], st[1], 0.0 * st[1], st[2], GAMMA, 1)

    fields = _cell_fields_1d(cons, 0.0, 1.0, n)
    return Problem('shock_tube_1d', 1, n, 1, 0.0, 1.0, 0.0, 1.0, fields, bc=(FREE, FREE, PERIODIC, PERIODIC),
                   cfl=cfl, t_end=t_end, meta=dict(left=left, right=right, x_diaphragm=0.5))


def riemann_1d(left, right, n: int, x0: float = 0.0, x1: float = 1.0, x_d: float = 0.5, t_end: float = 0.1,
               cfl: float = 0.3) -> Problem:
    """Riemann problem with primitive states left = (rho, U, p) for x < x_d and
    right for x > x_d, free-flow boundaries."""
    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        is_left = (x < x_d) | ((x == x_d) & (np.asarray(side) < 0))
        st = [np.where(is_left, a, b) for a, b in zip(left, right)]
        return prim_to_cons(st[0], st[1], 0.0 * st[1], st[2], GAMMA, 1)

    fields = _cell_fields_1d(cons, x0, x1, n)
    return Problem('riemann_1d', 1, n, 1, x0, x1, 0.0, 1.0, fields, bc=(FREE, FREE, PERIODIC, PERIODIC),
                   cfl=cfl, t_end=t_end, meta=dict(left=tuple(left), right=tuple(right), x_diaphragm=x_d))


def expansion_1d(n: int, U: float = 1.5, rho: float = 1.0, p: float = 0.4, cfl: float = 0.3) -> Problem:
    """Periodic [0, 1] with (rho, -U, p) for x < 1/2 and (rho, U, p) for
    x > 1/2: two rarefactions leave a near-vacuum behind them at x = 1/2 (the
    double-rarefaction Riemann problem of the test suites for positivity) and
    the two streams collide at x = 0 (two shocks)."""
    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        right = (x > 0.5) | ((x == 0.5) & (np.asarray(side) > 0))
        return prim_to_cons(rho + 0.0 * x, np.where(right, U, -U), 0.0 * x, p + 0.0 * x, GAMMA, 1)

    fields = _cell_fields_1d(cons, 0.0, 1.0, n)
    return Problem('expansion_1d', 1, n, 1, 0.0, 1.0, 0.0, 1.0, fields, bc=(PERIODIC,) * 4, cfl=cfl,
                   meta=dict(U=U, rho=rho, p=p))


def expansion_2d(nx: int, ny: int = 0, U: float = 1.25, amp: float = 0.1, rho: float = 1.0, p: float = 0.4,
                 cfl: float = 0.3, gauss_points: int = 2) -> Problem:
    """The 1D expansion made two-dimensional: periodic [0, 1]^2, U = -U left of
    the curve x = 1/2 + amp sin(2 pi y) and +U right of it, V = 0."""
    ny = ny or nx

    def prim(x, y, sx, sy):
        right = x > 0.5 + amp * np.sin(2.0 * np.pi * y)
        return rho + 0.0 * x, np.where(right, U, -U), 0.0 * x, p + 0.0 * x

    fields = _cell_fields_2d(prim, 0.0, 1.0, 0.0, 1.0, nx, ny)
    return Problem('expansion_2d', 2, nx, ny, 0.0, 1.0, 0.0, 1.0, fields, bc=(PERIODIC,) * 4, cfl=cfl,
                   gauss_points=gauss_points, meta=dict(U=U, amp=amp, rho=rho, p=p))


def stationary_shock_1d(n: int = 128, Ms: float = 1.1, t_end: float = 0.5, cfl: float = 0.3) -> Problem:
    """Normal shock of Mach Ms at rest at x = 0.5 on [0, 1]: upstream rho = p = 1,
    U = Ms sqrt(gamma), downstream from the Rankine-Hugoniot relations (the
    1D cut through the shock of the shock-vortex case); fixed inflow at x = 0,
    free flow at x = 1."""
    g = GAMMA
    U1 = Ms * math.sqrt(g)
    r2 = (g + 1.0) * Ms * Ms / ((g - 1.0) * Ms * Ms + 2.0)
    p2 = 1.0 + 2.0 * g / (g + 1.0) * (Ms * Ms - 1.0)
    U2 = U1 / r2

    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        up = (x < 0.5) | ((x == 0.5) & (np.asarray(side) < 0))
        return prim_to_cons(np.where(up, 1.0, r2), np.where(up, U1, U2), 0.0 * x, np.where(up, 1.0, p2), g, 1)

    fields = _cell_fields_1d(cons, 0.0, 1.0, n)
    inflow = np.zeros((4, 4))
    inflow[0] = (1.0, U1, 0.0, 1.0)
    return Problem('stationary_shock_1d', 1, n, 1, 0.0, 1.0, 0.0, 1.0, fields,
                   bc=(INFLOW, FREE, PERIODIC, PERIODIC), inflow_prim=inflow, cfl=cfl, t_end=t_end,
                   meta=dict(Ms=Ms, upstream=(1.0, U1, 1.0), downstream=(r2, U2, p2)))


def acoustic_wave_1d(n: int, eps: float = 1e-5, cfl: float = 0.2) -> Problem:
    """1D acoustic wave of Sec. 4.3 on periodic [0, 1/3]: U = eps a cos(w x),
    rho = rho_inf (1 + eps cos(2 w x)), p = p_inf (rho/rho_inf)^gamma with
    rho_inf = 1.1771, p_inf = 101325, w = 6 pi; averages and gradients from
    16-point Gauss-Legendre and face values.  exact(t) is the linear solution
    (the two Riemann invariants u +- p'/(rho a) carried at +-a), valid to
    O(eps) relative: nonlinear steepening reaches ~1e-3 of the amplitude after
    10 domain lengths."""
    g = GAMMA
    rho0, p0, w, L = 1.1771, 101325.0, 6.0 * math.pi, 1.0 / 3.0
    a = math.sqrt(g * p0 / rho0)
    dx = L / n
    xl = np.arange(n) * dx
    xr = xl + dx
    gx, gw = np.polynomial.legendre.leggauss(16)

    def prim(x, t):
        wp = eps * a * (np.cos(w * (x - a * t)) + np.cos(2 * w * (x - a * t)))
        wm = eps * a * (np.cos(w * (x + a * t)) - np.cos(2 * w * (x + a * t)))
        u = 0.5 * (wp + wm)
        rho = rho0 * (1.0 + 0.5 * (wp - wm) / a)
        return rho, u, p0 * (rho / rho0) ** g

    def cons(x, t):
        rho, u, p = prim(x, t)
        return np.array([rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u])

    def fields_at(t):
        pts = 0.5 * (xl + xr)[:, None] + 0.5 * dx * gx[None, :]
        avg = (cons(pts, t) * gw[None, None, :]).sum(axis=2) * 0.5
        return np.concatenate([avg, (cons(xr, t) - cons(xl, t)) / dx])

    return Problem('acoustic_wave_1d', 1, n, 1, 0.0, L, 0.0, 1.0, fields_at(0.0), cfl=cfl, exact=fields_at,
                   meta=dict(eps=eps, rho_inf=rho0, a=a))


def square_wave_1d(n: int, x0: float, x1: float, t_end: float, cfl: float = 0.3) -> Problem:
    """rho = 1 + 0.5 (H(x+50) - H(x-50)), U = 1, p = 1 with free-flow boundaries
    (Sec. 4.4); the exact solution is the translated square."""
    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        s = np.asarray(side)
        inside = ((x > -50.0) | ((x == -50.0) & (s > 0))) & ((x < 50.0) | ((x == 50.0) & (s < 0)))
        rho = np.where(inside, 1.5, 1.0)
        return prim_to_cons(rho, 1.0 + 0 * rho, 0 * rho, 1.0 + 0 * rho, GAMMA, 1)

    fields = _cell_fields_1d(cons, x0, x1, n)
    return Problem('square_wave_1d', 1, n, 1, x0, x1, 0.0, 1.0, fields, bc=(FREE, FREE, PERIODIC, PERIODIC),
                   cfl=cfl, t_end=t_end)


def gaussian_advection_1d(n: int, x0: float, x1: float, b: float, t_end: float, cfl: float = 0.3) -> Problem:
    """rho = 1 + 0.5 exp(-ln2 x^2/b^2), U = 1, p = 1 (Sec. 4.2), free-flow boundaries."""
    def cons(x, side):
        x = np.asarray(x, dtype=np.float64)
        rho = 1.0 + 0.5 * np.exp(-math.log(2.0) * x * x / (b * b))
        return prim_to_cons(rho, 1.0 + 0 * rho, 0 * rho, 1.0 + 0 * rho, GAMMA, 1)

    fields = _cell_fields_1d(cons, x0, x1, n)

    def exact(t):
        return _cell_fields_1d(lambda x, s: cons(np.asarray(x) - t, s), x0, x1, n)

    return Problem('gaussian_advection_1d', 1, n, 1, x0, x1, 0.0, 1.0, fields,
                   bc=(FREE, FREE, PERIODIC, PERIODIC), cfl=cfl, t_end=t_end, exact=exact)


# ---------------------------------------------------------------- 2D workloads

def acoustic_pulse_2d(n: int = 1024, seed: int = 0, amp: float = 1e-3, half_width: float = 0.05,
                      steps: int = 500, cfl: float = 0.3, ny: Optional[int] = None) -> Problem:
    """Periodic [-1,1]^2, background (rho,U,V,p) = (1,0,0,1/gamma), a Gaussian
    pulse amp*exp(-ln2 r^2/b^2) added to both density and pressure (the
    acoustic-pulse form of Sec. 4.6), centred at a point drawn uniformly from
    [-1,1]^2 by numpy's default_rng(seed); minimum-image distances."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    xc, yc = rng.uniform(-1.0, 1.0, size=2)
    L = 2.0
    a = math.log(2.0) / (half_width * half_width)

    def prim(x, y, sx, sy):
        dxp = _min_image(x - xc, L)
        dyp = _min_image(y - yc, L)
        g = amp * np.exp(-a * (dxp * dxp + dyp * dyp))
        return 1.0 + g, 0.0 * g, 0.0 * g, 1.0 / GAMMA + g

    fields = _cell_fields_2d(prim, -1.0, 1.0, -1.0, 1.0, n, ny)
    return Problem('acoustic_pulse_2d', 2, n, ny, -1.0, 1.0, -1.0, 1.0, fields, cfl=cfl, steps=steps,
                   meta=dict(seed=seed, centre=(float(xc), float(yc)), amp=amp, half_width=half_width))


def shock_vortex_2d(nx: int = 2048, ny: int = 1024, Ms: float = 1.1, Mv: float = 0.3, Rc: float = 0.05,
                    xv: float = 0.25, yv: float = 0.5, t_end: float = 0.8, cfl: float = 0.5) -> Problem:
    """[0,2]x[0,1]: stationary normal shock of Mach Ms at x = 0.5 (upstream
    rho = p = 1, U = Ms sqrt(gamma); downstream from the Rankine-Hugoniot
    relations), isentropic vortex upstream; reflecting walls at y = 0, 1,
    fixed inflow at x = 0, free flow at x = 2.  CFL 0.5, the number Sec. 3
    gives for inviscid flow."""
    g = GAMMA
    U1 = Ms * math.sqrt(g)
    r2 = (g + 1.0) * Ms * Ms / ((g - 1.0) * Ms * Ms + 2.0)
    p2 = 1.0 + 2.0 * g / (g + 1.0) * (Ms * Ms - 1.0)
    U2 = U1 / r2

    def prim(x, y, sx, sy):
        up = (x < 0.5) | ((x == 0.5) & (np.asarray(sx) < 0))
        rv, Uv, Vv, pv = vortex_prim(x, y, xv, yv, Mv, Rc, 1.0, U1, 0.0, 1.0)
        rho = np.where(up, rv, r2)
        U = np.where(up, Uv, U2)
        V = np.where(up, Vv, 0.0)
        p = np.where(up, pv, p2)
        return rho, U, V, p

    fields = _cell_fields_2d(prim, 0.0, 2.0, 0.0, 1.0, nx, ny)
    inflow = np.zeros((4, 4))
    inflow[0] = (1.0, U1, 0.0, 1.0)
    return Problem('shock_vortex_2d', 2, nx, ny, 0.0, 2.0, 0.0, 1.0, fields, bc=(INFLOW, FREE, WALL, WALL),
                   inflow_prim=inflow, cfl=cfl, t_end=t_end,
                   meta=dict(Ms=Ms, Mv=Mv, Rc=Rc, downstream=(r2, U2, 0.0, p2)))


def viscous_shock_vortex_2d(nx: int = 700, ny: int = 600, Ms: float = 1.2, Mv: float = 0.5, Re: float = 800.0,
                            t_end: float = 6.0, cfl: float = 0.3) -> Problem:
    """The viscous shock-vortex interaction of Sec. 4.8 on [-20,8]x[-12,12]:
    a stationary normal shock of Mach Ms at x = 0, the supersonic stream
    (rho = 1, p = 1/gamma, sound speed 1, U = -Ms) entering at x = 8 and
    carrying a counter-clockwise isentropic vortex of strength Mv (core radius
    1) from (2, 0); mu = rho a / Re of that stream; periodic in y, free flow
    at x = -20 (standing in for the paper's non-reflecting boundary)."""
    g = GAMMA
    p1 = 1.0 / g
    U1 = -Ms
    r2 = (g + 1.0) * Ms * Ms / ((g - 1.0) * Ms * Ms + 2.0)
    p2 = p1 * (1.0 + 2.0 * g / (g + 1.0) * (Ms * Ms - 1.0))
    U2 = U1 / r2

    def prim(x, y, sx, sy):
        up = (x > 0.0) | ((x == 0.0) & (np.asarray(sx) > 0))
        rv, Uv, Vv, pv = vortex_prim(x, y, 2.0, 0.0, Mv, 1.0, 1.0, U1, 0.0, p1)
        return np.where(up, rv, r2), np.where(up, Uv, U2), np.where(up, Vv, 0.0), np.where(up, pv, p2)

    fields = _cell_fields_2d(prim, -20.0, 8.0, -12.0, 12.0, nx, ny)
    inflow = np.zeros((4, 4))
    inflow[1] = (1.0, U1, 0.0, p1)
    return Problem('viscous_shock_vortex_2d', 2, nx, ny, -20.0, 8.0, -12.0, 12.0, fields,
                   bc=(FREE, INFLOW, PERIODIC, PERIODIC), inflow_prim=inflow, cfl=cfl, t_end=t_end, mu=1.0 / Re,
                   meta=dict(Ms=Ms, Mv=Mv, Re=Re, downstream=(r2, U2, 0.0, p2), upstream=(1.0, U1, 0.0, p1)))


def shock_reflection_2d(nx: int = 200, ny: int = 50, t_end: float = 50.0, cfl: float = 0.3) -> Problem:
    """Regular shock reflection of Sec. 4.4 on [0,4]x[0,1]: a Mach 2.9 stream
    (rho, U, V, p) = (1, 2.9, 0, 1/gamma) enters on the left, the state behind
    an oblique shock that meets the bottom wall at 29 degrees enters on the top
    (1.69997, 2.61934, -0.50632, 1.52819; Rankine-Hugoniot), slip wall at the
    bottom, free flow on the right; the domain starts at the left state."""
    left = (1.0, 2.9, 0.0, 1.0 / GAMMA)
    top = (1.69997, 2.61934, -0.50632, 1.52819)

    def prim(x, y, sx, sy):
        one = np.ones_like(np.asarray(x, dtype=np.float64) + 0.0 * np.asarray(y))
        return left[0] * one, left[1] * one, left[2] * one, left[3] * one

    fields = _cell_fields_2d(prim, 0.0, 4.0, 0.0, 1.0, nx, ny)
    inflow = np.zeros((4, 4))
    inflow[0] = left
    inflow[3] = top
    return Problem('shock_reflection_2d', 2, nx, ny, 0.0, 4.0, 0.0, 1.0, fields, bc=(INFLOW, FREE, WALL, INFLOW),
                   inflow_prim=inflow, cfl=cfl, t_end=t_end)


def plane_pulse(n: int = 300, ny: int = 0, eps: float = 1e-4, b: float = 0.08, mu: float = 0.0,
                cfl: float = 0.3) -> Problem:
    """Plane pressure pulse of Sec. 4.5 on [-5,5] (x [0,1] in 2D, ny > 0):
    rho = 1, U = V = 0, p = 1/gamma + eps exp(-ln2 (x/b)^2); free flow at
    x = +-5 (the waves stay inside for t < 4), periodic in y.  exact(t) is the
    linear inviscid solution: two acoustic halves moving at +-1 (the sound
    speed) and an entropy wave at rest, -eps f(x) in density."""
    g = GAMMA
    a = math.sqrt(math.log(2.0)) / b
    x0, x1 = -5.0, 5.0
    dx = (x1 - x0) / n
    xl = x0 + np.arange(n) * dx
    xr = xl + dx

    def favg(s):          # cell averages of f(x - s)
        return math.sqrt(math.pi) / (2 * a) * (_erf(a * (xr - s)) - _erf(a * (xl - s))) / dx

    def fpt(x):
        return np.exp(-(a * x) ** 2)

    def fields_at(t):
        pa = 0.5 * eps * (favg(t) + favg(-t))                    # pressure (acoustic)
        ra = pa - eps * favg(0.0)                                 # density: acoustic + entropy
        dpa = 0.5 * eps * (fpt(xr - t) - fpt(xl - t) + fpt(xr + t) - fpt(xl + t)) / dx
        dra = dpa - eps * (fpt(xr) - fpt(xl)) / dx
        # momentum of the two acoustic halves: rho U = (p_right-moving - p_left-moving) / c
        mu_ = 0.5 * eps * (favg(t) - favg(-t))
        dmu = 0.5 * eps * (fpt(xr - t) - fpt(xl - t) - fpt(xr + t) + fpt(xl + t)) / dx
        rows = [1.0 + ra, mu_, (1.0 / g + pa) / (g - 1.0), dra, dmu, dpa / (g - 1.0)]
        if ny <= 0:
            return np.array(rows)
        out = np.zeros((12, ny, n))
        for k, src in zip((0, 1, 3, 4, 5, 7), rows):
            out[k] = src
        return out

    if ny <= 0:
        return Problem('plane_pulse_1d', 1, n, 1, x0, x1, 0.0, 1.0, fields_at(0.0), bc=(FREE, FREE, PERIODIC, PERIODIC),
                       cfl=cfl, mu=mu, exact=fields_at, meta=dict(eps=eps))
    return Problem('plane_pulse_2d', 2, n, ny, x0, x1, 0.0, 1.0, fields_at(0.0), bc=(FREE, FREE, PERIODIC, PERIODIC),
                   cfl=cfl, mu=mu, exact=fields_at, meta=dict(eps=eps))


def serving_request(k: int) -> Problem:
    """Request k of the serving workload: periodic [-1,1]^2, background
    (1,0,0,1/gamma), a Gaussian acoustic pulse (amplitude log-uniform in
    [1e-4, 1e-2], half-width 0.1) plus an isentropic vortex (strength uniform
    in [0.1, 0.5], core radius 0.1); side drawn from {64,128,256,512}; 200 steps.
    All draws from numpy's default_rng(1000 + k)."""
    rng = np.random.default_rng(1000 + k)
    n = int(rng.choice([64, 128, 256, 512]))
    amp = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-2))))
    Mv = float(rng.uniform(0.1, 0.5))
    pc = rng.uniform(-1.0, 1.0, size=2)
    vc = rng.uniform(-1.0, 1.0, size=2)
    a = math.log(2.0) / (0.1 * 0.1)
    L = 2.0

    def prim(x, y, sx, sy):
        rv, Uv, Vv, pv = vortex_prim(x, y, vc[0], vc[1], Mv, 0.1, 1.0, 0.0, 0.0, 1.0 / GAMMA, Lx=L, Ly=L)
        dxp = _min_image(x - pc[0], L)
        dyp = _min_image(y - pc[1], L)
        gp = amp * np.exp(-a * (dxp * dxp + dyp * dyp))
        return rv + gp, Uv, Vv, pv + gp

    fields = _cell_fields_2d(prim, -1.0, 1.0, -1.0, 1.0, n, n)
    return Problem('serving_request_%d' % k, 2, n, n, -1.0, 1.0, -1.0, 1.0, fields, steps=200,
                   meta=dict(k=k, amp=amp, Mv=Mv))


def tam_webb_2d(n: int = 200, t_end: float = 28.45, L: float = 100.0, cfl: float = 0.3) -> Problem:
    """Sound, entropy and vorticity pulses on a uniform flow (Sec. 4.6):
    [-L,L]^2 (the paper's L = 100), rho_inf = 1, U_inf = 0.5, Mach 0.5
    (c_inf = 1, p_inf = 1/gamma), CFL 0.3; periodic boundaries: at L = 100 no
    wave reaches them before t = 56.9, at L = 250 none reaches them, nor
    any periodic image the window [-100,100]^2, before t = 100."""
    e1, e2, e3 = 1e-2, 1e-3, 4e-4
    a1 = math.log(2.0) / 9.0
    a2 = a3 = math.log(2.0) / 25.0
    x1c, x2c = -100.0 / 3.0, 100.0 / 3.0

    def prim(x, y, sx, sy):
        r1 = (x - x1c) ** 2 + y * y
        r2 = (x - x2c) ** 2 + y * y
        rho = 1.0 + e1 * np.exp(-a1 * r1) + e2 * np.exp(-a2 * r2)
        p = 1.0 / GAMMA + e1 * np.exp(-a1 * r1)
        U = 0.5 + e3 * np.exp(-a3 * r2) * y
        V = -e3 * np.exp(-a3 * r2) * (x - x2c)
        return rho, U, V, p

    fields = _cell_fields_2d(prim, -L, L, -L, L, n, n)
    return Problem('tam_webb_2d', 2, n, n, -L, L, -L, L, fields, cfl=cfl, t_end=t_end)


def diagonal_wave_2d(n: int, eps: float = 0.2, t_end: float = 0.5, cfl: float = 0.3,
                     fixed_dt: float = 0.0, U: float = 1.0, V: float = 1.0) -> Problem:
    """rho = 1 + eps sin(pi (x + y)), (U, V) uniform, p = 1 on periodic [0,2]^2;
    the exact solution is the translated wave (closed-form averages)."""
    x0, x1 = 0.0, 2.0

    def avg_fields(t):
        h = (x1 - x0) / n
        xc = x0 + (np.arange(n) + 0.5) * h
        X, Y = np.meshgrid(xc - U * t, xc - V * t)
        s = (2.0 * math.sin(math.pi * h / 2.0) / (math.pi * h)) ** 2
        rho = 1.0 + eps * s * np.sin(math.pi * (X + Y))
        # gradient averages: (1/h^2) int int d/dx ... = eps * pi * cos(...) * s
        grad = eps * math.pi * s * np.cos(math.pi * (X + Y))
        f = np.empty((12, n, n))
        f[0] = rho
        f[1] = rho * U
        f[2] = rho * V
        f[3] = 1.0 / (GAMMA - 1.0) + 0.5 * rho * (U * U + V * V)
        for off in (4, 8):
            f[off] = grad
            f[off + 1] = grad * U
            f[off + 2] = grad * V
            f[off + 3] = 0.5 * grad * (U * U + V * V)
        return f

    return Problem('diagonal_wave_2d', 2, n, n, x0, x1, x0, x1, avg_fields(0.0), cfl=cfl, t_end=t_end,
                   fixed_dt=fixed_dt, exact=avg_fields, meta=dict(eps=eps))


def vortex_translation_2d(n: int, Mv: float = 0.3, Rc: float = 0.5, t_end: float = 0.5,
                          U: float = 1.0, V: float = 0.5, cfl: float = 0.3) -> Problem:
    """Isentropic vortex carried by a uniform flow on periodic [-5,5]^2: an
    exact Euler solution (the vortex profile is negligible at the boundary)."""
    L = 10.0

    def prim_at(t):
        def prim(x, y, sx, sy):
            return vortex_prim(x, y, U * t, V * t, Mv, Rc, 1.0, U, V, 1.0 / GAMMA, Lx=L, Ly=L)
        return prim

    fields = _cell_fields_2d(prim_at(0.0), -5.0, 5.0, -5.0, 5.0, n, n)

    def exact(t):
        return _cell_fields_2d(prim_at(t), -5.0, 5.0, -5.0, 5.0, n, n)

    return Problem('vortex_translation_2d', 2, n, n, -5.0, 5.0, -5.0, 5.0, fields, cfl=cfl, t_end=t_end,
                   exact=exact, meta=dict(Mv=Mv, Rc=Rc))


def shear_wave_2d(n: int, mu: float, A: float = 1e-3, ny: int = 3, U: float = 0.0, rho: float = 1.0,
                  p: float = 1.0, t_end: float = 1.0, cfl: float = 0.3, fixed_dt: float = 0.0) -> Problem:
    """Viscous shear wave on periodic [0,1]^2: uniform rho, p, velocity
    (U, A sin 2 pi (x - U t)) decaying as exp(-mu k^2 t / rho), k = 2 pi (the
    Navier-Stokes solution up to the O(A^2) viscous heating); y-invariant."""
    k = 2.0 * math.pi

    def prim_at(t):
        amp = A * math.exp(-mu * k * k * t / rho)

        def prim(x, y, sx, sy):
            x = np.asarray(x, dtype=np.float64)
            one = np.ones_like(x + 0.0 * np.asarray(y))
            return rho * one, U * one, amp * np.sin(k * (x - U * t)) * one, p * one
        return prim

    fields = _cell_fields_2d(prim_at(0.0), 0.0, 1.0, 0.0, 1.0, n, ny)
    return Problem('shear_wave_2d', 2, n, ny, 0.0, 1.0, 0.0, 1.0, fields, cfl=cfl, t_end=t_end, mu=mu,
                   fixed_dt=fixed_dt,
                   exact=lambda t: _cell_fields_2d(prim_at(t), 0.0, 1.0, 0.0, 1.0, n, ny),
                   meta=dict(A=A, k=k))


def channel_shear_2d(n: int, mu: float, A: float = 1e-3, ny: int = 3, rho: float = 1.0, p: float = 1.0,
                     t_end: float = 1.0, cfl: float = 0.3, fixed_dt: float = 0.0) -> Problem:
    """Viscous shear flow between no-slip walls at x = 0 and 1 (periodic in y):
    uniform rho, p, velocity (0, A sin pi x) decaying as exp(-mu pi^2 t / rho)
    (the Navier-Stokes solution up to the O(A^2) heating); y-invariant."""
    k = math.pi

    def prim_at(t):
        amp = A * math.exp(-mu * k * k * t / rho)

        def prim(x, y, sx, sy):
            x = np.asarray(x, dtype=np.float64)
            one = np.ones_like(x + 0.0 * np.asarray(y))
            return rho * one, 0.0 * one, amp * np.sin(k * x) * one, p * one
        return prim

    fields = _cell_fields_2d(prim_at(0.0), 0.0, 1.0, 0.0, 1.0, n, ny)
    return Problem('channel_shear_2d', 2, n, ny, 0.0, 1.0, 0.0, 1.0, fields, bc=(NOSLIP, NOSLIP, PERIODIC, PERIODIC),
                   cfl=cfl, t_end=t_end, mu=mu, fixed_dt=fixed_dt,
                   exact=lambda t: _cell_fields_2d(prim_at(t), 0.0, 1.0, 0.0, 1.0, n, ny), meta=dict(A=A, k=k))


def uniform_2d(nx: int, ny: int, prim=(1.0, 0.3, -0.2, 0.8), bc=(PERIODIC,) * 4) -> Problem:
    """Free stream: a uniform state with zero gradients."""
    W = prim_to_cons(np.float64(prim[0]), np.float64(prim[1]), np.float64(prim[2]), np.float64(prim[3]))
    f = np.zeros((12, ny, nx))
    for k in range(4):
        f[k] = W[k]
    inflow = np.zeros((4, 4))
    for s in range(4):
        inflow[s] = prim
    return Problem('uniform_2d', 2, nx, ny, 0.0, 1.0, 0.0, 1.0, f, bc=bc, inflow_prim=inflow, steps=5)


def density_errors(num: np.ndarray, ref: np.ndarray) -> tuple:
    """L1 (mean |e|), L2 (rms) and Linf of the density cell averages."""
    e = np.abs(np.asarray(num[0]) - np.asarray(ref[0])).ravel()
    return float(e.mean()), float(np.sqrt((e * e).mean())), float(e.max())
