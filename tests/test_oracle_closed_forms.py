"""Closed-form pins of the oracle's local matrices.

* P1 triangle mass = |det DF|/24 [2 1 1; 1 2 1; 1 1 2] (golden fixture), in R^2
  and on a tilted triangle in R^3.
* P1 triangle stiffness: off-diagonal entries are -cot(opposite angle)/2
  (cotangent formula), rows sum to zero.
* Affine P2 triangle mass = area/180 * integer matrix (golden fixture).
* Every element type on affine elements: local mass and stiffness equal the
  exact integrals of the nodal basis, computed here in exact rational
  arithmetic from the barycentric monomial formula
  int lambda^alpha = alpha! / (|alpha| + d)!, which the default rules must
  reproduce (degree 2p for mass, 2p - 2 for stiffness).
* The paper's worked half-disk mesh: 1^T M 1 = 1 + (4/3)(sqrt2 - 1).
"""

import itertools
import os
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle
from meshgen import meshes as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_int_matrix(name):
    rows, div = [], None
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("divisor"):
                div = int(line.split()[1])
            else:
                rows.append([int(t) for t in line.split()])
    return np.array(rows, dtype=np.float64), div


def single(domain, dim, order, V, F, quad=None):
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    if order == 2:
        edges = {1: mg.SEG_EDGES, 2: mg.TRI_EDGES, 3: mg.TET_EDGES}[dim]
        V, F, _ = mg.p1_to_p2(V, F, edges)
    coords, conn = mg.to_soa(V, F)
    default = {(1, 1): 2, (1, 2): 3, (2, 1): 3, (2, 2): 6, (3, 1): 4, (3, 2): 11}[(dim, order)]
    return dict(domain=domain, dim=dim, order=order, quad=quad or default, coords=coords,
                conn=conn)


def test_p1_triangle_mass_golden():
    G, div = read_int_matrix("p1_triangle_mass.txt")
    # flat triangle in R^2
    V = [[0.1, 0.2], [1.3, 0.4], [0.5, 1.7]]
    m = single("bulk", 2, 1, V, [[0, 1, 2]])
    det = abs(np.linalg.det(np.array([np.subtract(V[1], V[0]), np.subtract(V[2], V[0])])))
    M = oracle.element_matrices(m, "mass")[0]
    assert np.allclose(M, det * G / div, rtol=1e-14, atol=0)
    # the same triangle rotated into R^3 as a surface element
    R = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))[0]
    V3 = (np.concatenate([np.array(V), np.zeros((3, 1))], 1) @ R.T) + [0.3, -0.2, 0.9]
    m3 = single("surface", 2, 1, V3, [[0, 1, 2]])
    M3 = oracle.element_matrices(m3, "mass")[0]
    assert np.allclose(M3, det * G / div, rtol=1e-13, atol=0)


def cot(u, v):
    return np.dot(u, v) / np.linalg.norm(np.cross(np.r_[u, 0][:3], np.r_[v, 0][:3]))


def test_p1_cotangent_formula():
    V = np.array([[0.1, 0.2], [1.3, 0.4], [0.5, 1.7]])
    for domain, X in (("bulk", V),
                      ("surface", np.concatenate([V, np.array([[0.0], [0.5], [-0.3]])], 1))):
        m = single(domain, 2, 1, X, [[0, 1, 2]])
        A = oracle.element_matrices(m, "stiffness")[0]
        for a, b in itertools.permutations(range(3), 2):
            c = 3 - a - b
            u, v = X[a] - X[c], X[b] - X[c]
            cu = np.dot(u, v) / np.linalg.norm(np.cross(np.r_[u, [0] * (3 - len(u))],
                                                        np.r_[v, [0] * (3 - len(v))]))
            assert abs(A[a, b] + 0.5 * cu) < 1e-14 * np.abs(A).max()
        assert np.allclose(A.sum(1), 0, atol=1e-14)


def test_p2_triangle_affine_mass_golden():
    G, div = read_int_matrix("p2_triangle_mass_affine.txt")
    V = [[0.0, 0.0], [2.0, 0.1], [0.5, 1.5]]
    m = single("bulk", 2, 2, V, [[0, 1, 2]])
    area = 0.5 * abs(np.linalg.det(np.array([np.subtract(V[1], V[0]), np.subtract(V[2], V[0])])))
    M = oracle.element_matrices(m, "mass")[0]
    assert np.allclose(M, area * G / div, rtol=0, atol=1e-15 * area * 32 / div * 4)


# ---------------------------------------------------------------------------
# exact rational integration of the nodal basis (barycentric polynomials)
# ---------------------------------------------------------------------------
EDGES = {1: [(0, 1)], 2: [(0, 1), (1, 2), (2, 0)],
         3: [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]}


def pmul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0) + ca * cb
    return out


def padd(p, q, s=1):
    out = dict(p)
    for k, c in q.items():
        out[k] = out.get(k, 0) + s * c
    return out


def pint(p, d):
    tot = Fraction(0)
    for a, c in p.items():
        num = 1
        for e in a:
            num *= factorial(e)
        tot += c * Fraction(num, factorial(sum(a) + d))
    return tot


def lam(i, d):
    e = [0] * (d + 1)
    e[i] = 1
    return {tuple(e): Fraction(1)}


def const(c, d):
    return {tuple([0] * (d + 1)): Fraction(c)}


def basis_poly(d, p):
    if p == 1:
        return [lam(i, d) for i in range(d + 1)]
    out = [pmul(lam(i, d), padd(pmul(const(2, d), lam(i, d)), const(1, d), -1))
           for i in range(d + 1)]
    out += [pmul(const(4, d), pmul(lam(a, d), lam(b, d))) for a, b in EDGES[d]]
    return out


def pdiff_lambda(p, i):
    out = {}
    for a, c in p.items():
        if a[i] > 0:
            b = list(a)
            b[i] -= 1
            out[tuple(b)] = out.get(tuple(b), 0) + c * a[i]
    return out


def pgrad_ref(p, d, m):
    """d/d xi_m with lambda_0 = 1 - sum xi, lambda_{m+1} = xi_m."""
    return padd(pdiff_lambda(p, m + 1), pdiff_lambda(p, 0), -1)


AFFINE_CASES = [
    ("surface", 1, [[Fraction(1, 3), Fraction(1, 5)], [Fraction(7, 4), Fraction(-2, 3)]]),
    ("surface", 2, [[0, 0, 0], [Fraction(3, 2), Fraction(1, 3), Fraction(1, 2)],
                    [Fraction(1, 4), Fraction(5, 4), Fraction(-1, 3)]]),
    ("bulk", 2, [[Fraction(1, 10), Fraction(1, 5)], [Fraction(13, 10), Fraction(2, 5)],
                 [Fraction(1, 2), Fraction(17, 10)]]),
    ("bulk", 3, [[0, 0, 0], [Fraction(6, 5), Fraction(1, 10), Fraction(1, 5)],
                 [Fraction(1, 5), Fraction(11, 10), 0],
                 [Fraction(1, 10), Fraction(1, 5), Fraction(9, 10)]]),
]


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("domain,dim,verts", AFFINE_CASES)
def test_affine_exact_rational(domain, dim, verts, order):
    affine_exact_check(domain, dim, verts, order)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("domain,dim,verts", [c for c in AFFINE_CASES if c[1] == 3])
def test_affine_exact_rational_degree7_tetrahedron(domain, dim, verts, order):
    """The 35-point degree-7 rule gives the exact affine matrices too."""
    affine_exact_check(domain, dim, verts, order, quad=35)


def affine_exact_check(domain, dim, verts, order, quad=None):
    X = [[Fraction(c) for c in v] for v in verts]
    n = len(X[0])
    J = [[X[m + 1][c] - X[0][c] for m in range(dim)] for c in range(n)]  # n x d
    G = [[sum(J[c][i] * J[c][j] for c in range(n)) for j in range(dim)] for i in range(dim)]
    Gm = np.array([[float(x) for x in r] for r in G])
    # exact rational inverse of G
    import sympy
    Gi = sympy.Matrix(dim, dim, lambda i, j: sympy.Rational(G[i][j].numerator, G[i][j].denominator)).inv()
    detG = float(np.linalg.det(Gm))
    mu = np.sqrt(detG)
    phis = basis_poly(dim, order)
    k = len(phis)
    grads = [[pgrad_ref(ph, dim, m) for m in range(dim)] for ph in phis]
    Mex = np.zeros((k, k))
    Aex = np.zeros((k, k))
    for a in range(k):
        for b in range(k):
            Mex[a, b] = float(pint(pmul(phis[a], phis[b]), dim))
            s = Fraction(0)
            for i in range(dim):
                for j in range(dim):
                    gij = Fraction(int(Gi[i, j].p), int(Gi[i, j].q))
                    s += gij * pint(pmul(grads[a][i], grads[b][j]), dim)
            Aex[a, b] = float(s)
    Mex *= mu
    Aex *= mu
    Vf = np.array([[float(c) for c in v] for v in verts])
    m = single(domain, dim, order, Vf, [list(range(dim + 1))], quad=quad)
    M = oracle.element_matrices(m, "mass")[0]
    A = oracle.element_matrices(m, "stiffness")[0]
    assert np.abs(M - Mex).max() <= 1e-14 * np.abs(Mex).max()
    assert np.abs(A - Aex).max() <= 1e-13 * np.abs(Aex).max()


def read_half_disk():
    V, F, formula = [], [], None
    mode = None
    with open(os.path.join(GOLD, "half_disk_p2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("nodes"):
                mode = "n"
                continue
            if line.startswith("elements"):
                mode = "e"
                continue
            if line.startswith("area_formula"):
                formula = line.split(None, 1)[1]
                continue
            if mode == "n":
                V.append([float(t) for t in line.split()])
            else:
                F.append([int(t) for t in line.split()])
    return np.array(V), np.array(F), formula


@pytest.mark.parametrize("quad", [3, 6])
def test_paper_half_disk_area(quad):
    V, F, formula = read_half_disk()
    assert np.allclose(V, mg.half_disk_paper()[0], atol=1e-15)
    coords, conn = mg.to_soa(V, F)
    mesh = dict(domain="bulk", dim=2, order=2, quad=quad, coords=coords, conn=conn)
    rp, ci, va = oracle.assemble(mesh, "mass")
    expected = eval(formula, {"sqrt": np.sqrt})
    assert abs(va.sum() - expected) < 4e-16 * 4
    # A 1 = 0 and the linear-reproduction identity on the curved mesh
    A = oracle.to_scipy(9, oracle.assemble(mesh, "stiffness"))
    assert np.abs(A @ np.ones(9)).max() < 1e-14
    lhs = sum(coords[c] @ (A @ coords[c]) for c in range(2))
    assert abs(lhs - 2 * expected) < 1e-14
