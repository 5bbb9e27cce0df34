"""Von Neumann model of the 2D step linearised about a uniform state.

TEST INFRASTRUCTURE: an independent derivation of what the oracle's 2D step
does to one Fourier mode, used to pin the oracle's 2D assembly and to study
its stability.  It imports nothing from oracle/ or from the package.

About a uniform state and with linear reconstruction weights, every
non-equilibrium term of the interface evolution cancels (the left and right
states equal the equilibrium one, the two slope terms cancel, the pressure
jump of the collision time is of second order), so each Gauss point carries
the Euler flux of the reconstructed state and its Cauchy-Kowalewski time
derivatives (Sec. 2.1, the smooth limit of eq. 3rd-simplify-flux):
    F = A W0,  W_t = -(A W_n + B W_t'),  F_t = A W_t,
    W_tt = A^2 W_nn + (AB + BA) W_nt + B^2 W_t't'      (A normal, B tangential
Jacobian).  The cell averages follow eq. step-hyper-1; the gradients follow
the Gauss theorem (eq. compact-deriv-1) applied to the interface states of
the same two-stage method (Sec. 2.2).  A mode is exp(i (kx i + ky j)) over
cells (i, j); cell widths 1 (gradients per cell width), time step in units of
the cell width.

Normal reconstruction: eq. (recons-8th-val).  Along a face (the 2D algorithm
figure of Sec. 3 is missing; this is the reading the oracle uses): the cells'
tangential gradients reach the face by the cubic through the 4 stencil cells
(value and normal derivative); two Gauss points take every point quantity
from the three nearest segments (the quintic matching 3 segment averages and
3 segment-averaged tangential derivatives; W_nn by the quadratic); four
points take values and first derivatives from the sextic through 7 segment
averages and W_nt, W_tt from the three-segment quintics.
"""
import numpy as np

# eq. (recons-8th-val): value, h d/dx, h^2 d2/dx2 of P7 at x_{i+1/2} from
# (Q_{i-1}, Q_i, Q_{i+1}, Q_{i+2}, hQ'_{i-1}, hQ'_i, hQ'_{i+1}, hQ'_{i+2})
P7 = np.array([
    np.array([25, 185, 185, 25, 6, 102, -102, -6]) / 420.0,
    np.array([-14, -270, 270, 14, -3, -99, -99, -3]) / 108.0,
    np.array([-4, 4, 4, -4, -1, -9, 9, 1]) / 4.0,
])


def _avg_row(lo, hi, n):
    return np.array([(hi ** (p + 1) - lo ** (p + 1)) / (p + 1) for p in range(n)])


def _point_rows(eta, n):
    p = np.arange(n, dtype=float)
    v = eta ** p
    d1 = np.where(p >= 1, p * eta ** np.maximum(p - 1, 0), 0.0)
    d2 = np.where(p >= 2, p * (p - 1) * eta ** np.maximum(p - 2, 0), 0.0)
    return v, d1, d2


def fit_weights(nseg, eta, with_derivatives):
    """Weights (value, d1, d2 at eta) over the data of nseg unit segments at
    offsets -nseg//2..nseg//2: their averages, then (with_derivatives) the
    averages of the derivative over the same segments (end-value differences)."""
    offs = np.arange(nseg) - nseg // 2
    rows = [_avg_row(o - 0.5, o + 0.5, 2 * nseg if with_derivatives else nseg) for o in offs]
    if with_derivatives:
        n = 2 * nseg
        for o in offs:
            rows.append(np.array([(o + 0.5) ** p - (o - 0.5) ** p for p in range(n)]))
    M = np.array(rows)
    Minv = np.linalg.inv(M)
    return tuple(r @ Minv for r in _point_rows(eta, M.shape[0]))


# the cubic through 4 unit cells (offsets -1..2 about the face at +1/2)
_CUB = np.linalg.inv(np.array([_avg_row(m - 1.5, m - 0.5, 4) for m in range(4)]))
CUBIC_FACE = (_point_rows(0.5, 4)[0] @ _CUB, _point_rows(0.5, 4)[1] @ _CUB)


def gauss(npts):
    x, w = np.polynomial.legendre.leggauss(npts)
    return x / 2.0, w / 2.0


def euler_jacobians(gamma, rho, U, V, p):
    """Flux Jacobians dF/dW, dG/dW of the 2D Euler equations in (rho, rhoU, rhoV, rhoE)."""
    E = p / (gamma - 1.0) + 0.5 * rho * (U * U + V * V)
    H = (E + p) / rho
    q2 = U * U + V * V
    g1 = gamma - 1.0
    A = np.array([[0, 1, 0, 0],
                  [0.5 * g1 * q2 - U * U, (3 - gamma) * U, -g1 * V, g1],
                  [-U * V, V, U, 0],
                  [U * (0.5 * g1 * q2 - H), H - g1 * U * U, -g1 * U * V, gamma * U]])
    B = np.array([[0, 0, 1, 0],
                  [-U * V, V, U, 0],
                  [0.5 * g1 * q2 - V * V, -g1 * U, (3 - gamma) * V, g1],
                  [V * (0.5 * g1 * q2 - H), -g1 * U * V, H - g1 * V * V, gamma * V]])
    return A, B


class LinearStep:
    """The linearised step for a uniform state (rho, U, V, p), time step dt (in
    cell widths over speed units), npts = 2 or 4 Gauss points."""

    def __init__(self, gamma, prim, dt, npts=2):
        self.A, self.B = euler_jacobians(gamma, *prim)
        self.dt = dt
        self.npts = npts
        self.eta, self.wg = gauss(npts)
        self.h3 = [fit_weights(3, e, True) for e in self.eta]
        self.q3 = [fit_weights(3, e, False) for e in self.eta]
        self.s7 = [fit_weights(7, e, False) for e in self.eta]

    def _face(self, W, Gn, Gt, kn, kt, An, At):
        dt = self.dt
        ph_n = np.exp(1j * kn * (np.arange(4) - 1))
        L = P7 @ np.concatenate([np.outer(ph_n, W), np.outer(ph_n, Gn)])   # value, n-derivative, nn lines
        T = CUBIC_FACE[0] @ np.outer(ph_n, Gt)
        TN = CUBIC_FACE[1] @ np.outer(ph_n, Gt)
        p3 = np.exp(1j * kt * np.arange(-1, 2))
        p7 = np.exp(1j * kt * np.arange(-3, 4))
        out = {k: np.zeros(4, complex) for k in ('F', 'Ft', 'A', 'B', 'Wtt')}
        for g in range(self.npts):
            hv, h1, h2 = self.h3[g]
            herm = lambda w, s, d: (w[:3] @ p3) * s + (w[3:] @ p3) * d
            W0t = herm(h1, L[0], T)
            W0tt = herm(h2, L[0], T)
            Wnt = herm(h1, L[1], TN)
            if self.npts == 2:
                W0 = herm(hv, L[0], T)
                Wn = herm(hv, L[1], TN)
                Wnn = (self.q3[g][0] @ p3) * L[2]
            else:
                sv, s1, _ = self.s7[g]
                W0 = (sv @ p7) * L[0]
                W0t = (s1 @ p7) * L[0]
                Wn = (sv @ p7) * L[1]
                Wnn = (sv @ p7) * L[2]
            Wt = -(An @ Wn + At @ W0t)
            Wtt = An @ An @ Wnn + (An @ At + At @ An) @ Wnt + At @ At @ W0tt
            w = self.wg[g]
            out['F'] += w * (An @ W0)
            out['Ft'] += w * (An @ Wt)
            out['A'] += w * (W0 + 0.5 * dt * Wt + dt * dt / 8.0 * Wtt)
            out['B'] += w * (W0 + dt * Wt + dt * dt / 6.0 * Wtt)
            out['Wtt'] += w * Wtt
        return out

    def _stage(self, W, Gx, Gy, kx, ky):
        fx = self._face(W, Gx, Gy, kx, ky, self.A, self.B)
        fy = self._face(W, Gy, Gx, ky, kx, self.B, self.A)
        dxm, dym = 1 - np.exp(-1j * kx), 1 - np.exp(-1j * ky)   # face +1/2 minus face -1/2
        L = -(fx['F'] * dxm + fy['F'] * dym)
        Lt = -(fx['Ft'] * dxm + fy['Ft'] * dym)
        return fx, fy, L, Lt, dxm, dym

    def apply(self, state, kx, ky):
        """state: 12 complex amplitudes (W, W_x, W_y); returns the amplitudes after one step."""
        dt = self.dt
        W, Gx, Gy = state[:4], state[4:8], state[8:]
        fx, fy, L, Lt, dxm, dym = self._stage(W, Gx, Gy, kx, ky)
        Ws = W + 0.5 * dt * L + dt * dt / 8.0 * Lt
        PW = W + dt * L + dt * dt / 6.0 * Lt
        fx2, fy2, _, Lt2, _, _ = self._stage(Ws, fx['A'] * dxm, fy['A'] * dym, kx, ky)
        return np.concatenate([PW + dt * dt / 3.0 * Lt2,
                               fx['B'] * dxm + dt * dt / 3.0 * fx2['Wtt'] * dxm,
                               fy['B'] * dym + dt * dt / 3.0 * fy2['Wtt'] * dym])

    def matrix(self, kx, ky):
        G = np.zeros((12, 12), complex)
        for c in range(12):
            e = np.zeros(12, complex)
            e[c] = 1.0
            G[:, c] = self.apply(e, kx, ky)
        return G

    def spectral_radius(self, n):
        """max |eigenvalue| over the wave numbers 2 pi m / n in both directions"""
        ks = 2 * np.pi * np.arange(n) / n
        return max(np.abs(np.linalg.eigvals(self.matrix(kx, ky))).max() for kx in ks for ky in ks)
