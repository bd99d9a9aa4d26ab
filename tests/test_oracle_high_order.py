"""Pins of the oracle's cubic and quartic elements on segments, triangles and
tetrahedra (degree 3 and up, which the paper notes its assembly extends to,
section 1; its mesh utility builds orders 2 to 4 in one to three dimensions,
section 5.4).

* the nodal basis against an independent construction: the Lagrange basis of
  the node lattice obtained by solving the Vandermonde system of the
  barycentric monomials of degree p in exact rationals (not the product
  formula the oracle uses); values and gradients at random points;
* the delta property at the nodes, partition of unity;
* single affine elements of every type: mass and stiffness matrices against
  exact rational integration of that basis (rules of degree >= 2p; for the
  quartic tetrahedron under the degree-7 rule the stiffness (degree 6) and
  the mass row sums (degree 4) are exact, the full mass (degree 8) is not);
* meshes from the P1 -> Pp converter: node positions are the lattice points of
  each element, 1^T M 1 is the area or volume (flat) and A 1 = 0,
  sum_k x_k^T A x_k = d 1^T M 1 (linear reproduction) on a curved sphere and
  on a tetrahedral cube with curved (jittered) nodes.
"""

import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from meshgen import meshes as mg
from test_oracle_closed_forms import AFFINE_CASES, padd, pgrad_ref, pint, pmul

EDGES = {1: [(0, 1)], 2: [(0, 1), (1, 2), (2, 0)], 3: [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]}
FACES = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]


def node_alphas(d, p):
    """Multi-indices of the local nodes: vertices, edge nodes (from the edge's
    first vertex), interior nodes."""
    out = []
    for i in range(d + 1):
        a = [0] * (d + 1)
        a[i] = p
        out.append(a)
    for u, v in EDGES[d]:
        for i in range(1, p):
            a = [0] * (d + 1)
            a[u], a[v] = p - i, i
            out.append(a)
    if d == 2:
        if p == 3:
            out.append([1, 1, 1])
        elif p == 4:
            out += [[2, 1, 1], [1, 2, 1], [1, 1, 2]]
    if d == 3:
        inner = [(1, 1, 1)] if p == 3 else [(2, 1, 1), (1, 2, 1), (1, 1, 2)] if p == 4 else []
        for f in FACES:
            for w in inner:
                a = [0] * 4
                for j, v in enumerate(f):
                    a[v] = w[j]
                out.append(a)
        if p == 4:
            out.append([1, 1, 1, 1])
    return out


def monomials(d, p):
    return [m for m in itertools.product(range(p + 1), repeat=d + 1) if sum(m) == p]


def solve_rational(A, B):
    """Gauss-Jordan elimination over Fractions: A X = B."""
    n = len(A)
    M = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [x * inv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def lagrange_polys(d, p):
    """Barycentric polynomials {monomial: coefficient} with phi_a(node_b) = delta."""
    nodes = [[Fraction(x, p) for x in a] for a in node_alphas(d, p)]
    mons = monomials(d, p)
    k = len(nodes)
    assert len(mons) == k
    V = [[np.prod([nd[j] ** m[j] for j in range(d + 1)]) for m in mons] for nd in nodes]
    # V C = I: column a of C holds the coefficients of phi_a
    C = solve_rational(V, [[Fraction(int(i == j)) for j in range(k)] for i in range(k)])
    return [{tuple(m): C[i][a] for i, m in enumerate(mons) if C[i][a] != 0} for a in range(k)]


def peval(poly, lam):
    return sum(float(c) * np.prod([lam[j] ** e for j, e in enumerate(mon)]) for mon, c in poly.items())


CASES = [(d, p) for d in (1, 2, 3) for p in (3, 4)]


@pytest.mark.parametrize("d,p", CASES)
def test_basis_against_vandermonde_construction(d, p):
    polys = lagrange_polys(d, p)
    grads = [[pgrad_ref(ph, d, m) for m in range(d)] for ph in polys]
    rng = np.random.default_rng(10 * d + p)
    for _ in range(5):
        xi = rng.dirichlet(np.ones(d + 1))[1:]
        lam = np.concatenate([[1 - xi.sum()], xi])
        phi, dphi = oracle.basis(d, p, xi)
        ref = np.array([peval(ph, lam) for ph in polys])
        dref = np.array([[peval(g, lam) for g in gr] for gr in grads])
        assert np.abs(phi - ref).max() <= 1e-13
        assert np.abs(dphi - dref).max() <= 1e-12


@pytest.mark.parametrize("d,p", CASES)
def test_delta_property_and_partition_of_unity(d, p):
    alphas = node_alphas(d, p)
    for b, a in enumerate(alphas):
        xi = np.array(a[1:], dtype=float) / p
        phi, dphi = oracle.basis(d, p, xi)
        e = np.zeros(len(alphas))
        e[b] = 1.0
        assert np.abs(phi - e).max() <= 1e-13
        assert abs(dphi.sum(axis=0)).max() <= 1e-12
    phi, _ = oracle.basis(d, p, np.full(d, 0.21))
    assert abs(phi.sum() - 1) <= 1e-14


def high_rule(d):
    return {1: 6, 2: 16, 3: 35}[d]


@pytest.mark.parametrize("p", [3, 4])
@pytest.mark.parametrize("domain,dim,verts", AFFINE_CASES)
def test_affine_exact_rational(domain, dim, verts, p):
    import sympy
    X = [[Fraction(c) for c in v] for v in verts]
    n = len(X[0])
    J = [[X[m + 1][c] - X[0][c] for m in range(dim)] for c in range(n)]
    G = [[sum(J[c][i] * J[c][j] for c in range(n)) for j in range(dim)] for i in range(dim)]
    Gi = sympy.Matrix(dim, dim, lambda i, j: sympy.Rational(G[i][j].numerator, G[i][j].denominator)).inv()
    mu = np.sqrt(float(np.linalg.det(np.array([[float(x) for x in r] for r in G]))))
    phis = lagrange_polys(dim, p)
    k = len(phis)
    grads = [[pgrad_ref(ph, dim, m) for m in range(dim)] for ph in phis]
    Mex, Aex = np.zeros((k, k)), np.zeros((k, k))
    Gq = [[Fraction(int(Gi[i, j].p), int(Gi[i, j].q)) for j in range(dim)] for i in range(dim)]
    for a in range(k):
        for b in range(a, k):
            Mex[a, b] = Mex[b, a] = float(pint(pmul(phis[a], phis[b]), dim))
            s = Fraction(0)
            for i in range(dim):
                for j in range(dim):
                    s += Gq[i][j] * pint(pmul(grads[a][i], grads[b][j]), dim)
            Aex[a, b] = Aex[b, a] = float(s)
    Mex *= mu
    Aex *= mu
    # one element whose nodes are the lattice points of the rational vertices
    Vf = np.array([[float(c) for c in v] for v in verts])
    pos = np.array([sum(al[j] / p * Vf[j] for j in range(dim + 1)) for al in node_alphas(dim, p)])
    coords = np.ascontiguousarray(pos.T)
    conn = np.arange(k, dtype=np.int32)[:, None]
    m = dict(domain=domain, dim=dim, order=p, quad=high_rule(dim), coords=coords, conn=conn)
    M = oracle.element_matrices(m, "mass")[0]
    A = oracle.element_matrices(m, "stiffness")[0]
    assert np.abs(A - Aex).max() <= 1e-12 * np.abs(Aex).max()
    if dim == 3 and p == 4:
        # the degree-7 rule integrates the row sums (int phi_a, degree 4) exactly,
        # not the degree-8 products; those equal the rule's own sum
        # mu sum_q w_q phi_a phi_b (xi_q), with phi from the rational construction
        assert np.abs(M.sum(1) - Mex.sum(1)).max() <= 1e-13 * np.abs(Mex.sum(1)).max()
        from oracle import quadrature
        qp, qw = quadrature.rule(3, 35)
        Mq = np.zeros((k, k))
        for xq, wq in zip(qp, qw):
            lamq = np.concatenate([[1 - xq.sum()], xq])
            ph = np.array([peval(f, lamq) for f in phis])
            Mq += wq * np.outer(ph, ph)
        Mq *= mu
        assert np.abs(M - Mq).max() <= 1e-13 * np.abs(Mq).max()
    else:
        assert np.abs(M - Mex).max() <= 1e-13 * np.abs(Mex).max()


@pytest.mark.parametrize("p", [3, 4])
def test_converter_places_lattice_nodes(p):
    V, F = mg.square_tri(2)
    W, G = mg.p1_to_pp(V, F, p, mg.TRI_EDGES)
    for e in range(len(F)):
        X = V[F[e]]
        for a, al in enumerate(node_alphas(2, p)):
            want = sum(al[j] / p * X[j] for j in range(3))
            assert np.abs(W[G[e, a]] - want).max() <= 1e-15
    Vs = np.stack([np.linspace(0, 1, 4), np.zeros(4)], 1)
    Fs = np.stack([np.arange(3), np.arange(1, 4)], 1)
    Ws, Gs = mg.p1_to_pp(Vs, Fs, p, mg.SEG_EDGES)
    for e in range(3):
        for a, al in enumerate(node_alphas(1, p)):
            want = al[0] / p * Vs[Fs[e, 0]] + al[1] / p * Vs[Fs[e, 1]]
            assert np.abs(Ws[Gs[e, a]] - want).max() <= 1e-15


@pytest.mark.parametrize("p", [3, 4])
def test_flat_area_and_kernel(p):
    V, F = mg.square_tri(3)
    W, G = mg.p1_to_pp(V, F, p, mg.TRI_EDGES)
    coords, conn = mg.to_soa(W, G)
    m = dict(domain="bulk", dim=2, order=p, quad=16, coords=coords, conn=conn)
    N = coords.shape[1]
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    A = oracle.to_scipy(N, oracle.assemble(m, "stiffness"))
    assert abs(M.sum() - 1.0) <= 1e-13
    assert np.abs(A @ np.ones(N)).max() <= 1e-12


@pytest.mark.parametrize("p", [3, 4])
def test_sphere_linear_reproduction(p):
    V, F = mg.icosphere_red(1)
    W, G = mg.p1_to_pp(V, F, p, mg.TRI_EDGES)
    W = mg.normalize_rows(W)
    coords, conn = mg.to_soa(W, G)
    m = dict(domain="surface", dim=2, order=p, quad=16, coords=coords, conn=conn)
    N = coords.shape[1]
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    A = oracle.to_scipy(N, oracle.assemble(m, "stiffness"))
    lhs = sum(coords[c] @ (A @ coords[c]) for c in range(3))
    assert abs(lhs - 2 * M.sum()) <= 1e-12 * M.sum()
    assert abs(M.sum() - 4 * np.pi) <= 2e-3 * 4 * np.pi  # curved order-p sphere area


@pytest.mark.parametrize("p", [3, 4])
def test_converter_places_tetrahedral_lattice_nodes(p):
    V, F, _ = mg.kuhn_cube(2, order=1)
    W, G = mg.p1_to_pp(V, F, p, mg.TET_EDGES)
    assert G.shape[1] == len(node_alphas(3, p))
    for e in range(len(F)):
        X = V[F[e]]
        for a, al in enumerate(node_alphas(3, p)):
            want = sum(al[j] / p * X[j] for j in range(4))
            assert np.abs(W[G[e, a]] - want).max() <= 1e-15
    # one node per lattice point: the (2 p + 1)^3 points of the two-cell cube
    assert len(W) == (2 * p + 1) ** 3


@pytest.mark.parametrize("p", [3, 4])
def test_tetrahedral_volume_kernel_and_linear_reproduction(p):
    """Straight Kuhn cube: 1^T M 1 = 1 and A 1 = 0; with the edge, face and
    inner nodes moved off the lattice (curved elements), linear reproduction
    sum_k x_k^T A x_k = 3 * 1^T M 1 still holds."""
    V, F, _ = mg.kuhn_cube(2, order=1)
    W, G = mg.p1_to_pp(V, F, p, mg.TET_EDGES)
    coords, conn = mg.to_soa(W, G)
    m = dict(domain="bulk", dim=3, order=p, quad=35, coords=coords, conn=conn)
    N = coords.shape[1]
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    A = oracle.to_scipy(N, oracle.assemble(m, "stiffness"))
    assert abs(M.sum() - 1.0) <= 1e-13
    assert np.abs(A @ np.ones(N)).max() <= 1e-12
    rng = np.random.default_rng(30 + p)
    Wc = W.copy()
    inner = np.all((W > 1e-12) & (W < 1 - 1e-12), axis=1) & (np.arange(len(W)) >= len(V))
    Wc[inner] += rng.uniform(-0.01, 0.01, size=(int(inner.sum()), 3))
    cc, _ = mg.to_soa(Wc, G)
    mc = dict(m, coords=cc)
    Mc = oracle.to_scipy(N, oracle.assemble(mc, "mass"))
    Ac = oracle.to_scipy(N, oracle.assemble(mc, "stiffness"))
    lhs = sum(cc[c] @ (Ac @ cc[c]) for c in range(3))
    assert abs(lhs - 3 * Mc.sum()) <= 1e-12 * Mc.sum()
    assert abs(Mc.sum() - 1.0) <= 1e-3  # boundary nodes fixed: the volume moves only slightly
