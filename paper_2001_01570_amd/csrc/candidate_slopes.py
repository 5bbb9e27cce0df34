"""Exact coefficients of the candidate polynomials of the WENO-Z left state
at the interface x_{i+1/2} (Sec. 3.3): value and first derivative of each
candidate in terms of the cell data of its stencil, printed for
cgks_device.h.

Unit cells centred at m = -1, 0, 1, 2 (cells i-1 .. i+2), the interface at
x = 1/2.  A candidate of degree r matches the cell averages of its stencil
cells and, where listed, the cells' averaged derivative (for a unit cell the
difference of the end values).  Inputs are shifted by Q_i:
a = Q_{i-1} - Q_i, c = Q_{i+1} - Q_i, d = Q_{i+2} - Q_i and A..D = h Q' of
cells i-1 .. i+2.  Candidate 1 takes its value from the quadratic on
{Q_{i-1}, Q_i, Q_{i+1}} (its smoothness indicator alone comes from the
cubic), as the value formulas of the left state do.

    python candidate_slopes.py
"""
import sympy as sp

x = sp.symbols('x')
a, c, d, A, B, C, D = sp.symbols('a c d A B C D')
Q = {-1: a, 0: sp.Integer(0), 1: c, 2: d}
DQ = {-1: A, 0: B, 1: C, 2: D}
STENCILS = {  # k: (average cells, derivative cells)
    0: ((-1, 0), (-1,)),
    1: ((-1, 0, 1), ()),
    2: ((0, 1, 2), (2,)),
    3: ((-1, 0, 1), ()),
    4: ((0, 1, 2), ()),
    5: ((-1, 0, 1), (-1, 0)),
    6: ((0, 1, 2), (1, 2)),
}


def candidate(k):
    avg, der = STENCILS[k]
    n = len(avg) + len(der)
    cs = sp.symbols('k0:%d' % n)
    p = sum(cs[j] * x ** j for j in range(n))
    eqs = [sp.integrate(p, (x, m - sp.Rational(1, 2), m + sp.Rational(1, 2))) - Q[m] for m in avg]
    eqs += [p.subs(x, m + sp.Rational(1, 2)) - p.subs(x, m - sp.Rational(1, 2)) - DQ[m] for m in der]
    sol = sp.solve(eqs, cs, dict=True)[0]
    p = p.subs(sol)
    return sp.expand(p.subs(x, sp.Rational(1, 2))), sp.expand(sp.diff(p, x).subs(x, sp.Rational(1, 2)))


if __name__ == '__main__':
    for k in range(7):
        v, s = candidate(k)
        print('q%d = %s    s%d = %s' % (k, v, k, s))
