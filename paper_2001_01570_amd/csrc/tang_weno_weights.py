"""Linear weights of the tangential WENO-Z at the Gauss nodes (the
tangential-WENO variant of the 2D assembly).

The three quadratics have the averages of the unit segments (-2..0), (-1..1)
and (0..2); at a node eta the weights d_k are the ones for which
sum_k d_k q_k(eta) equals the quartic through the five averages at eta, for
any averages.  Printed for the first node of each mirror pair: two points
-1/(2 sqrt 3); four points -a (inner) and -b (outer) with
a, b = sqrt(3/7 -+ 2/7 sqrt(6/5)) / 2.  Run: python tang_weno_weights.py"""
import sympy as sp


def weights(eta):
    y = sp.symbols('y')
    s = sp.symbols('s0:5')
    c = sp.symbols('c0:5')
    p = sum(c[i] * y ** i for i in range(5))
    half = sp.Rational(1, 2)
    sol = sp.solve([sp.integrate(p, (y, m - half, m + half)) - s[m + 2] for m in range(-2, 3)], c)
    quartic = p.subs(sol)

    def quad(cc, A, B, C):
        return B - (A - 2 * B + C) / 24 + (C - A) / 2 * (y - cc) + (A - 2 * B + C) / 2 * (y - cc) ** 2

    q = [quad(-1, s[0], s[1], s[2]), quad(0, s[1], s[2], s[3]), quad(1, s[2], s[3], s[4])]
    d = sp.symbols('d0:3')
    resid = sp.expand((sum(d[k] * q[k] for k in range(3)) - quartic).subs(y, eta))
    eqs = [resid.coeff(s[i]) for i in range(5)]
    sd = sp.solve(eqs[:3], d)
    assert all(sp.simplify(e.subs(sd)) == 0 for e in eqs)
    return [sp.nsimplify(sp.simplify(sd[d[k]])) for k in range(3)]


if __name__ == '__main__':
    a = sp.sqrt(sp.Rational(3, 7) - sp.Rational(2, 7) * sp.sqrt(sp.Rational(6, 5))) / 2
    b = sp.sqrt(sp.Rational(3, 7) + sp.Rational(2, 7) * sp.sqrt(sp.Rational(6, 5))) / 2
    for name, eta in (('two points', -1 / (2 * sp.sqrt(3))), ('inner', -a), ('outer', -b)):
        w = weights(eta)
        print(name, 'eta = %s' % sp.N(eta, 21), ', '.join('%s' % sp.N(x, 21) for x in w))
