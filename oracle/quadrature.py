"""Oracle quadrature rules, solved from their moment equations.

TEST INFRASTRUCTURE: only tests, the smoke check and the CPU-baseline leg of
the benchmark use this package.  The GPU library never imports it.

The paper integrates the local matrices with quadrature (section 3.2.2,
equations for the quadrature mass and stiffness): a rule (xi_i, w_i) on the
reference element with weights summing to the reference measure
(1 segment, 1/2 triangle, 1/6 tetrahedron).  The rules used by the
workloads are fixed here by *symmetry + moment equations*: the unknown orbit
parameters are the roots of "the rule integrates every symmetric polynomial
of degree <= p exactly", solved by Newton's method in 40-digit arithmetic and
rounded to float64 at the end.

Exact reference integrals used as right-hand sides (barycentric monomials):
  triangle (area 1/2):  int l0^a l1^b l2^c = a! b! c! / (a+b+c+2)!
  tetrahedron (vol 1/6): int l0^a l1^b l2^c l3^d = a! b! c! d! / (a+b+c+d+3)!
"""

from __future__ import annotations

from functools import lru_cache

import mpmath as mp
import numpy as np

mp.mp.dps = 40

# rule id = (simplex dimension, number of points) -> polynomial degree
DEGREE = {(1, 1): 1, (1, 2): 3, (1, 3): 5, (1, 4): 7, (1, 5): 9, (1, 6): 11,
          (2, 1): 1, (2, 3): 2, (2, 6): 4, (2, 16): 8,
          (3, 1): 1, (3, 4): 2, (3, 11): 4, (3, 35): 7}


def _bary_to_ref(lam):
    """Barycentric (l0, ..., ld) -> reference coordinates (l1, ..., ld)."""
    return [lam[i] for i in range(1, len(lam))]


def _orbit(sym, params):
    """All distinct permutations of a barycentric pattern."""
    if sym == "S3":
        return [[mp.mpf(1) / 3] * 3]
    if sym == "S21":
        a = params[0]
        b = 1 - 2 * a
        return [[a, a, b], [a, b, a], [b, a, a]]
    if sym == "S111":
        a, b = params
        c = 1 - a - b
        return [[a, b, c], [a, c, b], [b, a, c], [b, c, a], [c, a, b], [c, b, a]]
    if sym == "S4":
        return [[mp.mpf(1) / 4] * 4]
    if sym == "S31":
        a = params[0]
        b = 1 - 3 * a
        return [[b, a, a, a], [a, b, a, a], [a, a, b, a], [a, a, a, b]]
    if sym == "S22":
        a = params[0]
        b = mp.mpf(1) / 2 - a
        pts = []
        for i in range(4):
            for j in range(i + 1, 4):
                lam = [b] * 4
                lam[i] = a
                lam[j] = a
                pts.append(lam)
        return pts
    if sym == "S211":
        a, b = params
        c = 1 - 2 * a - b
        pts = []
        for i in range(4):
            for j in range(i + 1, 4):
                rest = [m for m in range(4) if m not in (i, j)]
                for u, v in ((rest[0], rest[1]), (rest[1], rest[0])):
                    lam = [None] * 4
                    lam[i] = a
                    lam[j] = a
                    lam[u] = b
                    lam[v] = c
                    pts.append(lam)
        return pts
    raise ValueError(sym)


def _sym_moments_tri(lam):
    l0, l1, l2 = lam
    return [mp.mpf(1), l0 ** 2 + l1 ** 2 + l2 ** 2, l0 * l1 * l2, l0 ** 4 + l1 ** 4 + l2 ** 4]


_TRI_EXACT = [mp.mpf(1) / 2, mp.mpf(1) / 4, mp.mpf(1) / 120, mp.mpf(1) / 10]


# degree <= 8 invariants of the triangle's symmetry group: with sum l = 1 every
# symmetric polynomial is a polynomial in e2 = l0 l1 + l0 l2 + l1 l2 and
# e3 = l0 l1 l2; the monomials e2^a e3^b, 2a + 3b <= 8, span degree <= 8
_TRI8 = [(a, b) for b in range(3) for a in range(5) if 2 * a + 3 * b <= 8]


def _sym_moments_tri8(lam):
    l0, l1, l2 = lam
    e2 = l0 * l1 + l0 * l2 + l1 * l2
    e3 = l0 * l1 * l2
    return [e2 ** a * e3 ** b for a, b in _TRI8]


def _tri_exact(a, b):
    """int over the triangle (area 1/2) of e2^a e3^b, expanded into barycentric
    monomials, each integrated exactly (Dirichlet integral)."""
    from fractions import Fraction
    from math import factorial
    poly = {(0, 0, 0): Fraction(1)}
    def mul(p, q):
        out = {}
        for ka, ca in p.items():
            for kb, cb in q.items():
                k = tuple(x + y for x, y in zip(ka, kb))
                out[k] = out.get(k, 0) + ca * cb
        return out
    e2 = {(1, 1, 0): Fraction(1), (1, 0, 1): Fraction(1), (0, 1, 1): Fraction(1)}
    e3 = {(1, 1, 1): Fraction(1)}
    for _ in range(a):
        poly = mul(poly, e2)
    for _ in range(b):
        poly = mul(poly, e3)
    tot = Fraction(0)
    for k, c in poly.items():
        tot += c * Fraction(factorial(k[0]) * factorial(k[1]) * factorial(k[2]), factorial(sum(k) + 2))
    return mp.mpf(tot.numerator) / tot.denominator


def _sym_moments_tet(lam):
    s2 = sum(x ** 2 for x in lam)
    s3 = sum(x ** 3 for x in lam)
    s4 = sum(x ** 4 for x in lam)
    s22 = sum(lam[i] ** 2 * lam[j] ** 2 for i in range(4) for j in range(i + 1, 4))
    return [mp.mpf(1), s2, s3, s4, s22]


_TET_EXACT = [mp.mpf(1) / 6, mp.mpf(1) / 15, mp.mpf(1) / 30, mp.mpf(2) / 105, mp.mpf(1) / 210]


# degree <= 7 invariants of the tetrahedron's symmetry group: with sum l = 1
# every symmetric polynomial is a polynomial in e2, e3, e4 (elementary
# symmetric polynomials of l0..l3); the monomials e2^a e3^b e4^c with
# 2a + 3b + 4c <= 7 span degree <= 7
_TET7 = [(a, b, c) for c in range(2) for b in range(3) for a in range(4) if 2 * a + 3 * b + 4 * c <= 7]


def _elementary(lam, r):
    from itertools import combinations
    tot = mp.mpf(0)
    for idx in combinations(range(len(lam)), r):
        t = mp.mpf(1)
        for i in idx:
            t *= lam[i]
        tot += t
    return tot


def _sym_moments_tet7(lam):
    e2, e3, e4 = (_elementary(lam, r) for r in (2, 3, 4))
    return [e2 ** a * e3 ** b * e4 ** c for a, b, c in _TET7]


def _simplex_exact(factors, dim):
    """int over the reference dim-simplex (measure 1/dim!) of the product of
    polynomials in barycentric coordinates, each given as {exponents: coef}:
    expanded into monomials, each integrated by the Dirichlet formula
    prod a_i! / (sum a_i + dim)!."""
    from fractions import Fraction
    from math import factorial
    poly = {(0,) * (dim + 1): Fraction(1)}
    for f in factors:
        out = {}
        for ka, ca in poly.items():
            for kb, cb in f.items():
                k = tuple(x + y for x, y in zip(ka, kb))
                out[k] = out.get(k, 0) + ca * cb
        poly = out
    tot = Fraction(0)
    for k, c in poly.items():
        num = 1
        for x in k:
            num *= factorial(x)
        tot += c * Fraction(num, factorial(sum(k) + dim))
    return mp.mpf(tot.numerator) / tot.denominator


def _elementary_poly(r):
    from fractions import Fraction
    from itertools import combinations
    return {tuple(1 if i in idx else 0 for i in range(4)): Fraction(1) for idx in combinations(range(4), r)}


def _tet7_exact(a, b, c):
    return _simplex_exact([_elementary_poly(2)] * a + [_elementary_poly(3)] * b + [_elementary_poly(4)] * c, 3)


def _solve(orbits, moments, exact, x0):
    """orbits: list of (sym, n_params); unknowns per orbit: weight, params."""
    def residual(*x):
        x = list(x)
        total = [mp.mpf(0)] * len(exact)
        for sym, npar in orbits:
            w = x.pop(0)
            params = [x.pop(0) for _ in range(npar)]
            for lam in _orbit(sym, params):
                m = moments(lam)
                for i in range(len(exact)):
                    total[i] += w * m[i]
        return [total[i] - exact[i] for i in range(len(exact))]
    sol = mp.findroot(residual, [mp.mpf(v) for v in x0], tol=mp.mpf(10) ** -36)
    sol = [sol[i] for i in range(len(x0))] if hasattr(sol, "__len__") else [sol]
    pts, wts = [], []
    sol = list(sol)
    for sym, npar in orbits:
        w = sol.pop(0)
        params = [sol.pop(0) for _ in range(npar)]
        for lam in _orbit(sym, params):
            pts.append(_bary_to_ref(lam))
            wts.append(w)
    return pts, wts


def _legendre(n, t):
    """P_n(t) and P_n'(t) by the three-term recurrence."""
    p0, p1 = mp.mpf(1), t
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
    dp = n * (t * p1 - p0) / (t ** 2 - 1)
    return p1, dp


def _gauss_legendre(n):
    """n-point Gauss-Legendre on [0, 1]: roots of P_n by Newton's method from
    the usual cosine estimates (one root per estimate)."""
    pts, wts = [], []
    for i in range(1, n + 1):
        x = mp.cos(mp.pi * (i - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
        for _ in range(100):
            p, dp = _legendre(n, x)
            step = p / dp
            x -= step
            if abs(step) < mp.mpf(10) ** -38:
                break
        _, dp = _legendre(n, x)
        w = 2 / ((1 - x ** 2) * dp ** 2)
        pts.append([(1 + x) / 2])
        wts.append(w / 2)
    order = sorted(range(n), key=lambda i: pts[i][0])
    return [pts[i] for i in order], [wts[i] for i in order]


@lru_cache(maxsize=None)
def _rule_mp(dim: int, npts: int):
    if dim == 1:
        return _gauss_legendre(npts)
    if dim == 2:
        if npts == 1:
            return _solve([("S3", 0)], lambda l: [mp.mpf(1)], [mp.mpf(1) / 2], [0.5])
        if npts == 3:
            # interior orbit (a, a, 1-2a) with a near 1/6 (the other root, a = 1/2,
            # is the edge-midpoint rule)
            return _solve([("S21", 1)], lambda l: _sym_moments_tri(l)[:2], _TRI_EXACT[:2],
                          [0.16, 0.15])
        if npts == 6:
            return _solve([("S21", 1), ("S21", 1)], _sym_moments_tri, _TRI_EXACT,
                          [0.11, 0.44, 0.05, 0.09])
        if npts == 16:
            # degree 8: centroid + three S21 orbits + one S111 orbit, the
            # structure of the 16-point rule the paper uses (Dunavant); the
            # published values (weights summing to 1) only seed the iteration
            seed = [0.144315607677787 / 2,
                    0.095091634267285 / 2, 0.459292588292723,
                    0.103217370534718 / 2, 0.170569307751760,
                    0.032458497623198 / 2, 0.050547228317031,
                    0.027230314174435 / 2, 0.008394777409958, 0.263112829634638]
            exact = [_tri_exact(a, b) for a, b in _TRI8]
            return _solve([("S3", 0), ("S21", 1), ("S21", 1), ("S21", 1), ("S111", 2)],
                          _sym_moments_tri8, exact, seed)
    if dim == 3:
        if npts == 1:
            return _solve([("S4", 0)], lambda l: [mp.mpf(1)], [mp.mpf(1) / 6], [0.1])
        if npts == 4:
            return _solve([("S31", 1)], lambda l: _sym_moments_tet(l)[:2], _TET_EXACT[:2],
                          [0.04, 0.14])
        if npts == 11:
            return _solve([("S4", 0), ("S31", 1), ("S22", 1)], _sym_moments_tet, _TET_EXACT,
                          [-0.013, 0.0076, 0.07, 0.025, 0.4])
        if npts == 35:
            # degree 7, the degree of the paper's tetrahedral rule (section
            # 5.2): centroid + (a,a,a,1-3a) + (a,a,1/2-a,1/2-a) + two orbits
            # (a,a,b,1-2a-b); eleven unknowns for the eleven invariants.  The
            # start selects the root with positive weights and interior points
            seed = [0.0159, 0.00705, 0.3157, 0.00532, 0.4495, 0.00135, 0.02127, 0.1466,
                    0.0062, 0.1888, 0.04716]
            exact = [_tet7_exact(a, b, c) for a, b, c in _TET7]
            return _solve([("S4", 0), ("S31", 1), ("S22", 1), ("S211", 2), ("S211", 2)],
                          _sym_moments_tet7, exact, seed)
    raise ValueError(f"no rule with {npts} points on the {dim}-simplex")


def rule(dim: int, npts: int):
    """(points (Q, dim) float64 in reference coordinates, weights (Q,) float64)."""
    pts, wts = _rule_mp(dim, npts)
    P = np.array([[float(c) for c in p] for p in pts], dtype=np.float64).reshape(npts, dim)
    W = np.array([float(w) for w in wts], dtype=np.float64)
    return P, W


def rule_mp(dim: int, npts: int):
    """The same rule in 40-digit arithmetic (for the exactness pins)."""
    return _rule_mp(dim, npts)


def degree(dim: int, npts: int) -> int:
    return DEGREE[(dim, npts)]
