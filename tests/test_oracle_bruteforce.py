"""Brute-force pin of the oracle on tiny curved meshes of all eight types.

A second, deliberately different implementation of the definition
(section 3.2: M_ij = sum_E int_E phi_i phi_j, A_ij = sum_E int_E grad phi_i .
grad phi_j, evaluated with the same rule):

* the nodal basis comes from solving a Vandermonde system on the reference
  nodes (not from barycentric closed forms), differentiated exactly as
  monomials;
* the tangential gradient g of phi is the solution of DF^T g = grad_hat phi
  with g in the tangent space (least squares on [DF^T ; nu^T]), nu taken
  from an SVD -- not the adjugate of L = [t1 t2 t1 x t2];
* entries are computed one global pair (i, j) at a time, looping over the
  elements that contain both nodes -- no COO, no sort;
* with a nodal coefficient (weighted mass M_c, coefficient stiffness A_a)
  the factor c_h(xi_q) = sum_r c_r phi_r(xi_q) is formed from the same
  Vandermonde basis, per pair and point.
"""

import itertools

import numpy as np
import pytest

import meshgen
import oracle
from oracle import quadrature

EDGES = {1: [(0, 1)], 2: [(0, 1), (1, 2), (2, 0)],
         3: [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]}


def ref_nodes(d, p):
    corners = [np.zeros(d)] + [np.eye(d)[i] for i in range(d)]
    if p == 1:
        return np.array(corners)
    return np.array(corners + [(corners[a] + corners[b]) / 2 for a, b in EDGES[d]])


def monos(d, p):
    return [a for a in itertools.product(range(p + 1), repeat=d) if sum(a) <= p]


def vandermonde_basis(d, p):
    X = ref_nodes(d, p)
    ms = monos(d, p)
    Vm = np.array([[np.prod(x ** np.array(a)) for a in ms] for x in X])
    Cf = np.linalg.solve(Vm, np.eye(len(X)))  # column b: coefficients of phi_b

    def ev(xi):
        v = np.array([np.prod(xi ** np.array(a)) for a in ms])
        g = np.zeros((len(ms), d))
        for i, a in enumerate(ms):
            for m in range(d):
                if a[m] > 0:
                    b = list(a)
                    b[m] -= 1
                    g[i, m] = a[m] * np.prod(xi ** np.array(b))
        return Cf.T @ v, Cf.T @ g  # phi (k,), dphi (k, d)
    return ev


def brute(mesh, coef_c=None, coef_a=None):
    """Entry-by-entry M (or M_c with the nodal coefficient coef_c) and A (or
    A_a with coef_a); a nodal coefficient enters as c_h = sum_r c_r phi_r,
    with phi_r the Vandermonde basis at the point."""
    d, p = mesh["dim"], mesh["order"]
    X = mesh["coords"].T
    F = mesh["conn"].T
    n = X.shape[1]
    P, W = quadrature.rule(d, mesh["quad"])
    ev = vandermonde_basis(d, p)
    tabs = [ev(x) for x in P]
    # per element, per q: phi, physical gradients, mu
    geo = []
    for e in range(len(F)):
        xe = X[F[e]]
        per_q = []
        for (phi, dphi) in tabs:
            DF = xe.T @ dphi  # n x d
            mu = np.sqrt(np.linalg.det(DF.T @ DF))
            if n > d:
                U, s, Vt = np.linalg.svd(DF)
                nu = U[:, d:]  # normal space
                lhs = np.concatenate([DF.T, nu.T], 0)
                rhs = np.concatenate([dphi.T, np.zeros((n - d, len(phi)))], 0)
            else:
                lhs, rhs = DF.T, dphi.T
            g = np.linalg.lstsq(lhs, rhs, rcond=None)[0]  # n x k
            per_q.append((phi, g, mu))
        geo.append(per_q)
    N = X.shape[0]
    Mb, Ab = {}, {}
    node_elems = [[] for _ in range(N)]
    for e in range(len(F)):
        for a in range(F.shape[1]):
            node_elems[F[e, a]].append((e, a))
    for i in range(N):
        cols = sorted({int(F[e, b]) for (e, _) in node_elems[i] for b in range(F.shape[1])})
        for j in cols:
            m_ij = 0.0
            a_ij = 0.0
            for (e, a) in node_elems[i]:
                bs = [b for b in range(F.shape[1]) if F[e, b] == j]
                if not bs:
                    continue
                b = bs[0]
                for q, (phi, g, mu) in enumerate(geo[e]):
                    ch = 1.0 if coef_c is None else float(coef_c[F[e]] @ phi)
                    ah = 1.0 if coef_a is None else float(coef_a[F[e]] @ phi)
                    m_ij += W[q] * mu * ch * phi[a] * phi[b]
                    a_ij += W[q] * mu * ah * g[:, a] @ g[:, b]
            Mb[(i, j)] = m_ij
            Ab[(i, j)] = a_ij
    return Mb, Ab


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_entrywise_definition(t):
    mesh = meshgen.small_mesh(*t, size=1)
    # at most a few elements
    T = min(mesh["conn"].shape[1], 6)
    mesh = dict(mesh)
    mesh["conn"] = np.ascontiguousarray(mesh["conn"][:, :T])
    Mb, Ab = brute(mesh)
    N = mesh["coords"].shape[1]
    for kind, ref in (("mass", Mb), ("stiffness", Ab)):
        rp, ci, va = oracle.assemble(mesh, kind)
        got = {}
        for i in range(N):
            for s in range(rp[i], rp[i + 1]):
                got[(i, int(ci[s]))] = va[s]
        assert set(got) == set(ref)
        scale = max(abs(v) for v in ref.values())
        for key, v in ref.items():
            assert abs(got[key] - v) <= 1e-13 * scale, (kind, key, got[key], v)


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_entrywise_definition_with_coefficients(t):
    """M_c and A_a (section 3.2 quadrature forms with the nodal coefficient
    interpolated by the element basis) on the same tiny curved meshes."""
    mesh = meshgen.small_mesh(*t, size=1)
    T = min(mesh["conn"].shape[1], 6)
    mesh = dict(mesh)
    mesh["conn"] = np.ascontiguousarray(mesh["conn"][:, :T])
    c, a = mesh["coef_c"], mesh["coef_a"]
    Mb, Ab = brute(mesh, coef_c=c, coef_a=a)
    check_against(mesh, Mb, Ab, c, a)


def check_against(mesh, Mb, Ab, coef_c, coef_a):
    """Largest scaled difference between the oracle's M_c, A_a and the
    brute-force dictionaries (asserts the pattern agrees)."""
    N = mesh["coords"].shape[1]
    worst = 0.0
    for kind, ref, coef in (("mass", Mb, coef_c), ("stiffness", Ab, coef_a)):
        rp, ci, va = oracle.assemble(mesh, kind, coef=coef)
        got = {}
        for i in range(N):
            for s in range(rp[i], rp[i + 1]):
                got[(i, int(ci[s]))] = va[s]
        assert set(got) == set(ref)
        scale = max(abs(v) for v in ref.values())
        worst = max(worst, max(abs(got[key] - v) for key, v in ref.items()) / scale)
    assert worst <= 1e-13, worst
    return worst

