"""Pins of the oracle's nodal-coefficient branch: the weighted mass M_c and
the coefficient stiffness A_a (section 3.2 quadrature forms with the factor
c_h(xi_q) = sum_r c_r phi_r(xi_q); the weighted terms of section 6.2).

Three routes that share nothing with the oracle's interpolation of c_h:

* row sums against the load vector: since sum_b phi_b = 1,
  (M_c 1)_a = sum_E sum_q w mu c_h phi_a = b(c)_a, the load vector of the
  same nodal data, which the oracle computes in a separate function (itself
  pinned by exact rational integration); every element type and order;
* exact rational integration on single affine elements of every type with a
  non-symmetric nodal coefficient, under a rule exact for the integrand
  (degree 3p for M_c, 3p - 2 for A_a):
      M_c[a][b] = mu sum_r c_r int phi_r phi_a phi_b,
      A_a[a][b] = mu sum_r c_r sum_ij (G^-1)_ij int phi_r d_i phi_a d_j phi_b;
* the brute-force route of test_oracle_bruteforce (Vandermonde basis, entry
  by entry) with c_h and a_h.

A build of the oracle with a planted mistake (the coefficient of node r paired
with the basis function of node r + 1) must fail each of them.
"""

from fractions import Fraction

import numpy as np
import pytest

import meshgen
import oracle
from meshgen import meshes as mg
from test_oracle_bruteforce import brute
from test_oracle_closed_forms import AFFINE_CASES, basis_poly, pgrad_ref, pint, pmul, single
from test_oracle_high_order import lagrange_polys

PLANTED = "ORACLE_PLANTED_COEF_MISTAKE"

# rules exact for the weighted integrands (points per element dimension and order)
EXACT_RULE = {(1, 1): 2, (1, 2): 5, (1, 3): 5, (2, 1): 6, (2, 2): 16, (3, 1): 11, (3, 2): 35}


# ---------------------------------------------------------------------------
# route 1: M_c 1 = b(c)
# ---------------------------------------------------------------------------
def load_route_error(m, c):
    N = m["coords"].shape[1]
    Mc = oracle.to_scipy(N, oracle.assemble(m, "mass", coef=c))
    b = oracle.load(m, c)
    return float(np.abs(Mc @ np.ones(N) - b).max() / np.abs(b).max())


def high_order_meshes():
    out = []
    for p in (3, 4):
        V, F = mg.circle(9, order=1)
        V, F = mg.p1_to_pp(V, F, p, mg.SEG_EDGES)
        coords, conn = mg.to_soa(V * (1 + 0.03 * np.sin(5 * np.arctan2(V[:, 1], V[:, 0])))[:, None], F)
        out.append(dict(domain="surface", dim=1, order=p, quad=5 if p == 3 else 6, coords=coords,
                        conn=conn))
        V, F = mg.icosphere_red(1, order=1)
        V, F = mg.p1_to_pp(V, F, p, mg.TRI_EDGES)
        V = mg.normalize_rows(V) * (1 + 0.05 * V[:, :1] * V[:, 1:2])
        coords, conn = mg.to_soa(V, F)
        out.append(dict(domain="surface", dim=2, order=p, quad=16, coords=coords, conn=conn))
    return out


def nodal_coefficient(m):
    X = m["coords"]
    return 1.0 + 0.5 * np.sin(3 * X[0]) * np.cos(2 * X[-1]) + 0.2 * X[1]


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_weighted_mass_rows_are_the_load_vector(t):
    m = meshgen.small_mesh(*t, size=3)
    assert load_route_error(m, m["coef_c"]) <= 1e-14


@pytest.mark.parametrize("i", range(4))
def test_weighted_mass_rows_are_the_load_vector_high_order(i):
    m = high_order_meshes()[i]
    assert load_route_error(m, nodal_coefficient(m)) <= 1e-14


# ---------------------------------------------------------------------------
# route 2: exact rational integration on affine elements
# ---------------------------------------------------------------------------
def nodal_basis(dim, order):
    return basis_poly(dim, order) if order <= 2 else lagrange_polys(dim, order)


def exact_weighted(domain, dim, verts, order, c):
    """(M_c, A_a) of one affine element with nodal coefficient c (rationals),
    exactly: barycentric monomials integrate to alpha! / (|alpha| + d)! on the
    reference simplex."""
    import sympy
    X = [[Fraction(x) for x in v] for v in verts]
    n = len(X[0])
    J = [[X[m + 1][cc] - X[0][cc] for m in range(dim)] for cc in range(n)]
    G = [[sum(J[cc][i] * J[cc][j] for cc in range(n)) for j in range(dim)] for i in range(dim)]
    Gi = sympy.Matrix(dim, dim, lambda i, j: sympy.Rational(G[i][j].numerator, G[i][j].denominator)).inv()
    Gi = [[Fraction(int(Gi[i, j].p), int(Gi[i, j].q)) for j in range(dim)] for i in range(dim)]
    mu = float(np.sqrt(np.linalg.det(np.array([[float(x) for x in r] for r in G]))))
    phis = nodal_basis(dim, order)
    k = len(phis)
    ch = {}
    for r in range(k):
        for mono, coef in phis[r].items():
            ch[mono] = ch.get(mono, 0) + c[r] * coef
    grads = [[pgrad_ref(ph, dim, m) for m in range(dim)] for ph in phis]
    Mex = np.zeros((k, k))
    Aex = np.zeros((k, k))
    for a in range(k):
        for b in range(k):
            Mex[a, b] = float(pint(pmul(ch, pmul(phis[a], phis[b])), dim))
            s = Fraction(0)
            for i in range(dim):
                for j in range(dim):
                    s += Gi[i][j] * pint(pmul(ch, pmul(grads[a][i], grads[b][j])), dim)
            Aex[a, b] = float(s)
    return Mex * mu, Aex * mu


def exact_route_error(domain, dim, verts, order):
    k = len(nodal_basis(dim, order))
    # a non-symmetric rational coefficient: no permutation of the local nodes maps it to itself
    c = [Fraction(3 + 2 * r, 4 + r) + Fraction(r * r, 7) for r in range(k)]
    Mex, Aex = exact_weighted(domain, dim, verts, order, c)
    Vf = np.array([[float(x) for x in v] for v in verts])
    m = single(domain, dim, min(order, 2), Vf, [list(range(dim + 1))], quad=EXACT_RULE[(dim, order)])
    if order > 2:
        V, F = mg.p1_to_pp(Vf, np.array([list(range(dim + 1))]), order, mg.SEG_EDGES if dim == 1 else mg.TRI_EDGES)
        coords, conn = mg.to_soa(V, F)
        m = dict(domain=domain, dim=dim, order=order, quad=EXACT_RULE[(dim, order)], coords=coords, conn=conn)
    nodes = m["conn"][:, 0]
    cn = np.zeros(m["coords"].shape[1])
    cn[nodes] = [float(x) for x in c]
    M = oracle.element_matrices(m, "mass", coef=cn)[0]
    A = oracle.element_matrices(m, "stiffness", coef=cn)[0]
    return max(float(np.abs(M - Mex).max() / np.abs(Mex).max()),
               float(np.abs(A - Aex).max() / np.abs(Aex).max()))


EXACT_CASES = [(dom, dim, verts, order) for dom, dim, verts in AFFINE_CASES for order in (1, 2)] + \
              [(dom, dim, verts, 3) for dom, dim, verts in AFFINE_CASES if dim == 1]


@pytest.mark.parametrize("domain,dim,verts,order", EXACT_CASES)
def test_weighted_exact_rational(domain, dim, verts, order):
    assert exact_route_error(domain, dim, verts, order) <= 1e-13


# ---------------------------------------------------------------------------
# route 3: brute force with c_h and a_h
# ---------------------------------------------------------------------------
def brute_route_error(t):
    mesh = meshgen.small_mesh(*t, size=1)
    T = min(mesh["conn"].shape[1], 6)
    mesh = dict(mesh)
    mesh["conn"] = np.ascontiguousarray(mesh["conn"][:, :T])
    c, a = mesh["coef_c"], mesh["coef_a"]
    Mb, Ab = brute(mesh, coef_c=c, coef_a=a)
    N = mesh["coords"].shape[1]
    worst = 0.0
    for kind, ref, coef in (("mass", Mb, c), ("stiffness", Ab, a)):
        rp, ci, va = oracle.assemble(mesh, kind, coef=coef)
        got = {(i, int(ci[s])): va[s] for i in range(N) for s in range(rp[i], rp[i + 1])}
        scale = max(abs(v) for v in ref.values())
        worst = max(worst, max(abs(got[key] - v) for key, v in ref.items()) / scale)
    return worst


# ---------------------------------------------------------------------------
# the planted mistake fails every route
# ---------------------------------------------------------------------------
def test_planted_pairing_mistake_is_caught():
    with oracle.planted(PLANTED):
        for t in meshgen.ALL_TYPES:
            m = meshgen.small_mesh(*t, size=3)
            assert load_route_error(m, m["coef_c"]) > 1e-6, t
            assert brute_route_error(t) > 1e-6, t
        for domain, dim, verts, order in EXACT_CASES:
            assert exact_route_error(domain, dim, verts, order) > 1e-6, (domain, dim, order)
        for m in high_order_meshes():
            assert load_route_error(m, nodal_coefficient(m)) > 1e-6
    # and the oracle proper is back in place afterwards
    m = meshgen.small_mesh("surface", 2, 2, size=3)
    assert load_route_error(m, m["coef_c"]) <= 1e-14
