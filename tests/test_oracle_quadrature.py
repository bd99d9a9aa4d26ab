"""Pins of the oracle's quadrature rules (section 3.2.2: the local matrices are
quadrature sums; the rule fixes the matrix).

Each rule must integrate every monomial up to its degree exactly -- checked
against exact rationals -- and must fail for some monomial of degree + 1, so
the stated degree is not an accident of symmetry."""

import itertools
from fractions import Fraction
from math import factorial

import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature as Q

RULES = [(1, 2), (1, 3), (1, 5), (1, 6), (2, 1), (2, 3), (2, 6), (2, 16), (3, 1), (3, 4), (3, 11), (3, 35)]


def exact_monomial(alpha):
    """int over the unit reference simplex of prod xi_m^alpha_m
    (Dirichlet integral): prod alpha_m! / (|alpha| + d)!."""
    num = 1
    for a in alpha:
        num *= factorial(a)
    return Fraction(num, factorial(sum(alpha) + len(alpha)))


def monomials(d, deg):
    return [a for a in itertools.product(range(deg + 1), repeat=d) if sum(a) == deg]


@pytest.mark.parametrize("dim,npts", RULES)
def test_rule_exact_to_degree_mp(dim, npts):
    pts, wts = Q.rule_mp(dim, npts)
    deg = Q.degree(dim, npts)
    for k in range(deg + 1):
        for alpha in monomials(dim, k):
            s = mp.mpf(0)
            for p, w in zip(pts, wts):
                t = w
                for m in range(dim):
                    t *= p[m] ** alpha[m]
                s += t
            ex = exact_monomial(alpha)
            assert abs(s - mp.mpf(ex.numerator) / ex.denominator) < mp.mpf(10) ** -30, (alpha, s)


@pytest.mark.parametrize("dim,npts", RULES)
def test_rule_not_exact_beyond_degree(dim, npts):
    pts, wts = Q.rule_mp(dim, npts)
    deg = Q.degree(dim, npts)
    worst = 0
    for alpha in monomials(dim, deg + 1):
        s = sum(w * np.prod([p[m] ** alpha[m] for m in range(dim)]) for p, w in zip(pts, wts))
        ex = exact_monomial(alpha)
        worst = max(worst, abs(float(s) - float(ex)))
    assert worst > 1e-8


@pytest.mark.parametrize("dim,npts", RULES)
def test_rule_float64(dim, npts):
    P, W = Q.rule(dim, npts)
    assert P.shape == (npts, dim)
    assert abs(W.sum() - 1.0 / factorial(dim)) < 1e-15
    # points inside the reference simplex
    assert np.all(P >= 0) and np.all(P.sum(1) <= 1 + 1e-15)
    deg = Q.degree(dim, npts)
    for k in range(deg + 1):
        for alpha in monomials(dim, k):
            s = float(np.sum(W * np.prod(P ** np.array(alpha), axis=1)))
            assert abs(s - float(exact_monomial(alpha))) < 5e-16


def test_known_rule_values():
    """Independent cross-check against the published closed forms of the
    degree-4 rules (triangle: two S21 orbits; tetrahedron: centroid + S31 + S22
    with a negative centroid weight)."""
    P, W = Q.rule(2, 6)
    s10 = np.sqrt(10.0)
    a = sorted([(8 - s10 + np.sqrt(38 - 44 * np.sqrt(0.4))) / 18,
                (8 - s10 - np.sqrt(38 - 44 * np.sqrt(0.4))) / 18])
    bary = np.concatenate([1 - P.sum(1, keepdims=True), P], 1)
    # the repeated barycentric coordinate of each S21 orbit (a, a, 1 - 2a)
    rep = np.sort(np.unique(np.round(np.median(bary, axis=1), 14)))
    assert np.allclose(rep, a, atol=1e-14)
    P, W = Q.rule(3, 11)
    assert abs(W.min() * 6 + 148 / 1875) < 1e-15
    assert np.sum(W < 0) == 1


def test_degree8_triangle_matches_published_rule():
    """The 16-point degree-8 rule solved from the moment equations equals the
    published 16-point rule (Dunavant, 1985) to the 15 digits printed there
    (weights normalised to sum 1)."""
    P, W = Q.rule(2, 16)
    lam = np.column_stack([1 - P.sum(1), P])
    W1 = 2 * W
    published = [  # (weight, orbit of barycentric coordinates)
        (0.144315607677787, (1 / 3, 1 / 3, 1 / 3)),
        (0.095091634267285, (0.459292588292723, 0.459292588292723, 0.081414823414554)),
        (0.103217370534718, (0.170569307751760, 0.170569307751760, 0.658861384496480)),
        (0.032458497623198, (0.050547228317031, 0.050547228317031, 0.898905543365938)),
        (0.027230314174435, (0.008394777409958, 0.263112829634638, 0.728492392955404)),
    ]
    seen = 0
    for w, orbit in published:
        perms = {tuple(np.round(p, 12)): p for p in itertools.permutations(orbit)}
        for p in perms.values():
            d = np.abs(lam - np.array(p)).max(1)
            i = int(d.argmin())
            assert d[i] < 2e-14 and abs(W1[i] - w) < 2e-14, (p, d[i], W1[i], w)
            seen += 1
    assert seen == 16


def test_degree7_tetrahedron_positive_interior_distinct():
    """The 35-point rule of degree 7 (the degree of the paper's tetrahedral
    rule, section 5.2): positive weights, points strictly inside, no point
    repeated, and invariant under the 24 vertex permutations (the set of
    (barycentric point, weight) pairs maps onto itself)."""
    P, W = Q.rule(3, 35)
    assert np.all(W > 0)
    lam = np.column_stack([1 - P.sum(1), P])
    assert lam.min() > 0.02
    key = {tuple(np.round(l, 12)): w for l, w in zip(lam, W)}
    assert len(key) == 35
    for s in itertools.permutations(range(4)):
        for l, w in zip(lam, W):
            m = tuple(np.round(l[list(s)], 12))
            assert m in key and abs(key[m] - w) <= 1e-17
