"""Oracle steps on a window of a large grid, for sampled parity at full size.

A step reads cells within 4 of a cell (2 per stage; 6, 3 per stage, with four
Gauss points and their 7-segment tangential stencil), so a window with a
4k-cell (6k-cell) margin on every artificial side reproduces k full-grid steps
exactly on its core.  Sides where the window meets the real domain boundary keep the real
boundary condition; artificial sides use free-flow ghosts (never compared)."""
import numpy as np

from oracle import oracle as O
from paper_2001_01570_amd import inputs as I

H = 4


def _axis(i0, size, n, periodic, bclo, bchi, h=H):
    if periodic:
        idx = np.arange(i0 - h, i0 + size + h) % n
        return idx, I.FREE, I.FREE, h, h + size
    a, b = max(0, i0 - h), min(n, i0 + size + h)
    lo = bclo if a == 0 else I.FREE
    hi = bchi if b == n else I.FREE
    c0 = max(i0, a + (0 if a == 0 else h)) - a
    c1 = min(i0 + size, b - (0 if b == n else h)) - a
    return np.arange(a, b), lo, hi, c0, c1


def window_step(prob, fields, i0, j0, size, dt, ulp_seed=None):
    """Returns (oracle core after one step of size dt, or after one step per
    entry of a sequence dt, (slice_y, slice_x) of the core in full-grid
    indices).  With ulp_seed, every input value is first moved
    by -1, 0 or +1 ulp (seeded): the spread of the result measures the
    conditioning of the FP64 step on that window."""
    bc = list(prob.bc)
    dts = list(dt) if np.ndim(dt) else [dt]
    h = (6 if prob.gauss_points == 4 else H) * len(dts)
    ix, xlo, xhi, cx0, cx1 = _axis(i0, size, prob.nx, bc[0] == I.PERIODIC, bc[0], bc[1], h)
    iy, ylo, yhi, cy0, cy1 = _axis(j0, size, prob.ny, bc[2] == I.PERIODIC, bc[2], bc[3], h)
    patch = np.ascontiguousarray(fields[:, iy][:, :, ix])
    if ulp_seed is not None:
        steps = np.random.default_rng(ulp_seed).integers(-1, 2, size=patch.shape)
        patch = np.where(steps > 0, np.nextafter(patch, np.inf), np.where(steps < 0, np.nextafter(patch, -np.inf), patch))
    dx, dy = prob.dx, prob.dy
    p = I.Problem('window', 2, len(ix), len(iy), 0.0, dx * len(ix), 0.0, dy * len(iy), patch,
                  bc=(xlo, xhi, ylo, yhi), inflow_prim=prob.inflow_prim, gamma=prob.gamma, cfl=prob.cfl,
                  weno_eps=prob.weno_eps, tau_eps=prob.tau_eps, tau_C=prob.tau_C, mu=prob.mu,
                  gauss_points=prob.gauss_points, recon_vars=prob.recon_vars, side_slopes=prob.side_slopes,
                  tang_weno=prob.tang_weno)
    o = O.Oracle(p, threads=4)
    for d in dts:
        o.step(d)
    st = o.state
    core = st[:, cy0:cy1, cx0:cx1]
    return core, (iy[cy0:cy1], ix[cx0:cx1])
