"""Linear stability of the 2D step at the CFL numbers of Sec. 4.

Sec. 4 runs every test at CFL >= 0.3 (0.5 for inviscid flow in Sec. 3), so a
small perturbation of a uniform state must not grow over a run of a few
hundred steps at those CFL numbers.  These pins fix the 2D assembly against
that requirement: with the x faces blind to the cells' y-gradients (the
reading this oracle used before), the linearised step about rest has spectral
radius 1.067 at CFL 0.3 -- a checkerboard of d(rhoU)/dx + d(rhoV)/dy fed by
the cell averages through both directions -- and 500 steps amplify rounding
by ~1e14.  With the cells' tangential gradients entering the faces the
radius is 1 + O(dt^2) (9.3e-5 at CFL 0.3 on the 8 x 8 grid below).  The
last test pins the linearised 2D step itself, mode by mode, against an
independent von Neumann derivation.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I

GAMMA = 1.4


def _uniform(n, U, cfl, gp):
    base = I.uniform_2d(n, n, prim=(1.0, U, 0.0, 1.0 / GAMMA))
    return dataclasses.replace(base, cfl=cfl, gauss_points=gp)


def _perturbed(p, amp, seed):
    """uniform state plus noise: amp on the averages, amp/dx on the gradients
    (the scale of a gradient of noise of size amp), so that the difference of
    two runs measures growth and not the first step's re-scaling"""
    rng = np.random.default_rng(seed)
    dx = (p.x1 - p.x0) / p.nx
    f = p.fields.copy()
    f[:4] += amp * rng.standard_normal(f[:4].shape)
    f[4:] += amp / dx * rng.standard_normal(f[4:].shape)
    return dataclasses.replace(p, fields=f)


def _growth(p, steps, amp=1e-8, seed=1):
    a = O.Oracle(p, threads=8)
    b = O.Oracle(_perturbed(p, amp, seed), threads=8)
    d = []
    for _ in range(steps):
        dt = a.step()
        b.step(dt)
        d.append(np.abs(a.state - b.state).max())
    return np.array(d)


@pytest.mark.parametrize('gp,U', [(2, 0.0), (4, 0.0), (2, 0.5)])
def test_perturbation_of_a_uniform_state_stays_bounded_over_500_steps_at_cfl_0_3(gp, U):
    """16 x 16 periodic, fluid at rest (and moving at Mach 0.5), noise of
    1e-8: after the first steps have mapped the noise onto the scheme's own
    modes, the difference of the two runs grows by at most 3x over the next
    400 steps (measured: at most 1.29x, 1.31x and 1.38x, ending at 1.15x,
    1.19x and 0.83x)."""
    d = _growth(_uniform(16, U, 0.3, gp), 500)
    ref = d[99]
    assert np.isfinite(d).all()
    assert d[100:].max() < 3.0 * ref, (ref, d[100:].max(), d[-1])


def _jacobian_radius(p, eps=1e-7):
    o = O.Oracle(p, threads=1)
    dt = o.cfl_dt()
    f0 = p.fields.copy()
    o.step(dt)
    s0 = o.state.reshape(-1)
    J = np.empty((f0.size, f0.size))
    flat = f0.reshape(-1)
    for c in range(f0.size):
        f = flat.copy()
        f[c] += eps
        o.set_state(f.reshape(f0.shape))
        o.step(dt)
        J[:, c] = (o.state.reshape(-1) - s0) / eps
    return np.abs(np.linalg.eigvals(J)).max()


@pytest.mark.parametrize('cfl,bound', [(0.15, 1.0 + 4e-4), (0.3, 1.0 + 2e-4), (0.5, 1.0 + 1e-6)])
def test_linearised_step_about_rest_has_no_growing_mode_of_order_dt(cfl, bound):
    """Spectral radius of the step's Jacobian (central differences about the
    fluid at rest, 8 x 8 periodic, every wave number pi m/4): measured
    1 + 2.3e-4, 1 + 9.3e-5 and 1 + 5e-9 at CFL 0.15, 0.3 and 0.5 -- growth
    of order dt^2 per step, from the second time derivative of the interface
    state, which a run of a few thousand steps does not see."""
    r = _jacobian_radius(_uniform(8, 0.0, cfl, 2))
    assert r < bound, r


def _mode_response(gp, prim, cfl, k, v, n=8, delta=1e-7):
    """The oracle's step applied to a uniform state plus delta Re(v exp(i k.(i, j)))
    (12 amplitudes: averages, then gradients per cell width), by central
    differences; returns (oracle response, model response) as fields / delta."""
    from tests.linear_model import LinearStep
    rho, U, V, p = prim
    c = np.sqrt(GAMMA * p / rho)
    dt = cfl / max(abs(U) + c, abs(V) + c)
    base = I.uniform_2d(n, n, prim=prim)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
    phase = np.exp(1j * (k[0] * ii + k[1] * jj))
    pert = np.real(v[:, None, None] * phase[None])
    out = []
    for s in (+1.0, -1.0):
        prob = dataclasses.replace(base, x0=0.0, x1=float(n), y0=0.0, y1=float(n), fields=base.fields + s * delta * pert,
                                   gauss_points=gp, weno_eps=1e6, tau_C=0.0)
        o = O.Oracle(prob, threads=1)
        o.step(dt)
        out.append(o.state)
    got = (out[0] - out[1]) / (2 * delta)
    G = LinearStep(GAMMA, prim, dt, gp).matrix(*k)
    want = np.real((G @ v)[:, None, None] * phase[None])
    return got, want


@pytest.mark.parametrize('gp', [2, 4])
@pytest.mark.parametrize('prim', [(1.0, 0.0, 0.0, 1.0 / GAMMA), (1.2, 0.5, -0.3, 0.9)], ids=['rest', 'moving'])
def test_oracle_step_on_a_fourier_mode_equals_the_independent_linear_model(gp, prim):
    """The 2D assembly pinned mode by mode: about a uniform state, with linear
    reconstruction weights and no pressure-jump collision time, the oracle's
    step acts on each Fourier mode as the 12 x 12 amplification matrix of an
    independent von Neumann derivation (tests/linear_model.py: Euler flux and
    Cauchy-Kowalewski derivatives at the Gauss points, the same tangential
    fits written from their definitions, eq. step-hyper-1 and the Gauss
    theorem).  Checks the tangential fits, the Gauss quadrature, the cross
    derivatives, the two-stage combination of averages and gradients and the
    rotation of the y faces together; an error in any term of the assembly
    shows in some mode.  Central differences of amplitude 1e-7: agreement to
    1e-7 of the response (measured 1e-10 to 1.3e-9, the rounding of the
    differences)."""
    rng = np.random.default_rng(7 + gp)
    for k in [(2 * np.pi / 8, 0.0), (np.pi, np.pi), (2 * np.pi * 3 / 8, 2 * np.pi * 5 / 8), (2 * np.pi * 7 / 8, np.pi / 4)]:
        v = rng.standard_normal(12) + 1j * rng.standard_normal(12)
        got, want = _mode_response(gp, prim, 0.3, k, v)
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err < 1e-7, (k, err)
