"""Parity metrics between the HIP path and the oracle.

single-step: per field, max|g - o| / max|o| (the tolerance 1e-12 of a GPU
step against the FP64 oracle).  The momentum averages of a fluid near rest
are produced by differences of O(p) momentum fluxes, so their rounding floor
is eps * rho c whatever |rho U| is: they are measured against
max(|rho U|, rho (|u| + c)).
multi-step: per conservative component c, the largest difference over
(W_c, dx W_x,c, dy W_y,c) relative to max|W_c|.  Rounding of the O(1) cell
averages reaches a gradient amplified by 1/dx, so after several steps the
gradients are compared in the units the reconstruction consumes them."""
import numpy as np


def momentum_scale(o, gamma=1.4):
    o = np.asarray(o)
    nc = 3 if o.shape[0] == 6 else 4
    rho = o[0]
    mom = o[1:nc - 1]
    ke = 0.5 * (mom * mom).sum(axis=0) / rho
    p = (gamma - 1.0) * (o[nc - 1] - ke)
    speed = np.sqrt((mom * mom).sum(axis=0)) / rho + np.sqrt(gamma * np.abs(p) / rho)
    return float((rho * speed).max())


def field_scales(o):
    """norm of each field over the whole grid (momentum averages floored by rho c)"""
    o = np.asarray(o)
    nf = o.shape[0]
    nc = 3 if nf == 6 else 4
    ms = momentum_scale(o)
    out = []
    for f in range(nf):
        den = np.abs(o[f]).max()
        if 1 <= f < nc - 1:
            den = max(den, ms)
        if den == 0.0:    # identically zero field: measure against its component's scale
            den = np.abs(o[f % nc]).max()
            if 1 <= f % nc < nc - 1:
                den = max(den, ms)
        out.append(den if den > 0.0 else 1.0)
    return np.array(out)


def field_errors(g, o, scales=None):
    """per field max|g - o| / ||field||; pass scales (field_scales of the full
    grid) when g, o are windows of a larger grid"""
    g = np.asarray(g)
    o = np.asarray(o)
    if scales is None:
        scales = field_scales(o)
    return np.array([np.abs(g[f] - o[f]).max() / scales[f] for f in range(g.shape[0])])


def scaled_errors(g, o, dx, dy=1.0):
    g = np.asarray(g)
    o = np.asarray(o)
    nf = g.shape[0]
    nc = 3 if nf == 6 else 4
    ms = momentum_scale(o)
    out = []
    for c in range(nc):
        scale = np.abs(o[c]).max()
        if 1 <= c < nc - 1:
            scale = max(scale, ms)
        d = np.abs(g[c] - o[c]).max()
        d = max(d, dx * np.abs(g[nc + c] - o[nc + c]).max())
        if nf == 12:
            d = max(d, dy * np.abs(g[8 + c] - o[8 + c]).max())
        out.append(d / scale)
    return np.array(out)
