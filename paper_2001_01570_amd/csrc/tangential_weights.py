"""Exact weights of the tangential fits used by the face kernels (cgks_device.h).

Prints the constants of kHerm2 / kHerm4 (sympy, exact rationals and radicals,
evaluated to 25 digits).  Unit segment width, segments at offsets -1, 0, 1:

* the quintic p fixed by the three segment averages s_l and by the averages of
  its derivative over the same segments, d_l = p(l + 1/2) - p(l - 1/2);
* the quadratic through the three segment averages.

For a Gauss-Legendre node eta the weights give p(eta) = sum v_l s_l + vd_l d_l,
p'(eta) = sum d1_l s_l + d1d_l d_l, p''(eta) = sum d2_l s_l + d2d_l d_l and the
quadratic's value sum q_l s_l.  Nodes: -1/(2 sqrt 3) (two points per segment);
-a, -b with a, b the inner and outer nodes of the 4-point rule on [-1/2, 1/2].
The mirrored nodes are taken by reading the segments in reverse order (the
derivative data then change sign).
"""
import sympy as sp

eta = sp.Symbol('eta')


def fit(nconds_deriv):
    n = 3 + nconds_deriv
    c = sp.symbols('c0:%d' % n)
    p = sum(c[i] * eta ** i for i in range(n))
    eqs = []
    for l in (-1, 0, 1):
        a, b = sp.Rational(2 * l - 1, 2), sp.Rational(2 * l + 1, 2)
        eqs.append(sp.integrate(p, (eta, a, b)))
    if nconds_deriv:
        for l in (-1, 0, 1):
            a, b = sp.Rational(2 * l - 1, 2), sp.Rational(2 * l + 1, 2)
            eqs.append(p.subs(eta, b) - p.subs(eta, a))
    M = sp.Matrix([[sp.diff(e, ci) for ci in c] for e in eqs])
    Minv = M.inv()
    basis = sp.Matrix([eta ** i for i in range(n)])
    # weights of datum r: row of basis^T Minv
    return [sp.simplify((basis.T * Minv)[0, r]) for r in range(n)]


def weights(node):
    h = fit(3)
    q = fit(0)
    out = {}
    out['v'] = [h[r].subs(eta, node) for r in range(3)]
    out['vd'] = [h[3 + r].subs(eta, node) for r in range(3)]
    out['d1'] = [sp.diff(h[r], eta).subs(eta, node) for r in range(3)]
    out['d1d'] = [sp.diff(h[3 + r], eta).subs(eta, node) for r in range(3)]
    out['d2'] = [sp.diff(h[r], eta, 2).subs(eta, node) for r in range(3)]
    out['d2d'] = [sp.diff(h[3 + r], eta, 2).subs(eta, node) for r in range(3)]
    out['q'] = [q[r].subs(eta, node) for r in range(3)]
    return out


def fmt(ws):
    keys = ('v', 'vd', 'd1', 'd1d', 'd2', 'd2d', 'q')
    rows = []
    for k in keys:
        rows.append('{' + ', '.join(sp.N(x, 25).__str__() for x in ws[k]) + '}')
    return '{' + ', '.join(rows) + '}'


if __name__ == '__main__':
    g2 = -1 / (2 * sp.sqrt(3))
    a = sp.sqrt(sp.Rational(3, 7) - sp.Rational(2, 7) * sp.sqrt(sp.Rational(6, 5))) / 2
    b = sp.sqrt(sp.Rational(3, 7) + sp.Rational(2, 7) * sp.sqrt(sp.Rational(6, 5))) / 2
    print('kHerm2 (node -1/(2 sqrt 3)):', fmt(weights(g2)))
    print('kHerm2 (node +1/(2 sqrt 3), host check):', fmt(weights(-g2)))
    print('kHerm4 inner:', fmt(weights(-a)))
    print('kHerm4 outer:', fmt(weights(-b)))
