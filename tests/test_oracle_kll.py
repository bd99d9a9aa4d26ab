"""Pins of the oracle's non-linear terms of the mean-curvature-flow example
(section 6.2): alpha^2 = |grad_Gamma_h nu_h|^2, f_1[c] = int alpha^2 (nu_h)_c phi_j,
f_2 = int alpha^2 H_h phi_j.

* affine fields on flat meshes of every type: nu = B x + b makes the
  tangential gradient B P (P the tangential projector: I - n n^T on a tilted
  plane, t t^T on a straight line, I in the bulk), so alpha^2 = |B P|_F^2 is
  constant and f_1[c] = alpha^2 M nu_c, f_2 = alpha^2 M H with the (pinned)
  mass matrix;
* an independent route on curved meshes: the gradient through the metric
  tensor J G^{-1} g (numpy, per point) instead of the oracle's C^T [g; 0];
* invariants: rotating the mesh and the field together rotates f_1 and leaves
  f_2 alone; scaling the mesh by s scales f by s^(d-2); f_2 is linear in H.

The per-step system of the algorithm (linearly implicit BDF in u = (nu; H),
oracle.kll_system) is pinned by running the scheme: on the unit sphere the
exact flow keeps nu = x/|x| and H = 2/r with r(t)^2 = 1 - 4t, and BDF1 / BDF2
must approach it with first / second order in tau.  A dropped f, a wrong
sign of A or f, or mixed-up components of u break this by orders of
magnitude.
"""

import numpy as np
import pytest

import meshgen
import oracle
from meshgen import meshes as mg


def flat_mesh(domain, dim, order, rng):
    """A flat multi-element mesh of each type with a generic affine embedding."""
    if domain == "surface" and dim == 1:
        n = 5
        V = np.stack([np.linspace(0.0, 1.0, n + 1), np.zeros(n + 1)], 1)
        F = np.stack([np.arange(n), np.arange(1, n + 1)], 1)
        if order == 2:
            V, F, _ = mg.p1_to_p2(V, F, mg.SEG_EDGES)
        A = np.array([[0.8, -0.3], [0.5, 1.1]])
        V = V @ A.T + np.array([0.2, -0.4])
        quad = 2 if order == 1 else 3
    elif domain == "surface" and dim == 2:
        V, F = mg.square_tri(3, order=order)
        E = np.array([[1.0, 0.2, 0.3], [-0.4, 0.9, 0.5]])  # rows: images of e_x, e_y
        V = V @ E + np.array([0.1, 0.2, -0.3])
        quad = 3 if order == 1 else 6
    elif domain == "bulk" and dim == 2:
        V, F = mg.square_tri(3, order=order)
        V = V @ np.array([[1.2, 0.1], [-0.3, 0.9]]).T
        quad = 3 if order == 1 else 6
    else:
        V, F, _ = mg.kuhn_cube(2, order=order)
        V = V @ np.array([[1.0, 0.2, 0.0], [0.1, 0.9, 0.3], [0.0, -0.2, 1.1]]).T
        quad = 4 if order == 1 else 11
    coords, conn = mg.to_soa(V, F)
    return dict(domain=domain, dim=dim, order=order, quad=quad, coords=coords, conn=conn)


def tangential_projector(m):
    X = m["coords"]
    n = X.shape[0]
    if m["domain"] == "bulk":
        return np.eye(n)
    e = m["conn"][:, 0]
    if m["dim"] == 1:
        t = X[:, e[1]] - X[:, e[0]]
        t /= np.linalg.norm(t)
        return np.outer(t, t)
    a, b, c = (X[:, e[i]] for i in range(3))
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm)
    return np.eye(3) - np.outer(nrm, nrm)


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_affine_field_on_flat_mesh(t):
    rng = np.random.default_rng(31)
    m = flat_mesh(*t, rng)
    X = m["coords"]
    n, N = X.shape
    B = rng.normal(size=(n, n))
    b = rng.normal(size=n)
    nu = B @ X + b[:, None]
    H = rng.uniform(0.5, 2.0, size=N)
    alpha2 = np.sum((B @ tangential_projector(m)) ** 2)
    f = oracle.kll(m, nu, H)
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    scale = np.abs(f).max()
    for c in range(n):
        assert np.abs(f[c] - alpha2 * (M @ nu[c])).max() <= 1e-12 * scale, c
    assert np.abs(f[n] - alpha2 * (M @ H)).max() <= 1e-12 * scale


def metric_route(m, nu, H):
    """f through the metric tensor: grad_Gamma (nu_h)_c = J G^{-1} g_c."""
    X, conn = m["coords"], m["conn"]
    n, N = X.shape
    d = m["dim"]
    qp, qw = oracle.quadrature.rule(d, m["quad"])
    f = np.zeros((n + 1, N))
    U = np.vstack([nu, H[None, :]])
    for e in range(conn.shape[1]):
        nodes = conn[:, e]
        x = X[:, nodes]                     # n x k
        ul = U[:, nodes]                    # (n+1) x k
        for xi, w in zip(qp, qw):
            phi, dphi = oracle.basis(d, m["order"], xi)
            J = x @ dphi                    # n x d
            G = J.T @ J
            mu = np.sqrt(np.linalg.det(G))
            grads = J @ np.linalg.solve(G, (ul[:n] @ dphi).T)  # n x n: column c = grad (nu_h)_c
            alpha2 = np.sum(grads ** 2)
            uh = ul @ phi
            f[:, nodes] += w * mu * alpha2 * np.outer(uh, phi)
    return f


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_metric_tensor_route(t):
    m = meshgen.small_mesh(*t, size=2)
    rng = np.random.default_rng(5)
    n, N = m["coords"].shape
    nu, H = rng.normal(size=(n, N)), rng.normal(size=N)
    f = oracle.kll(m, nu, H)
    g = metric_route(m, nu, H)
    assert np.abs(f - g).max() <= 1e-12 * np.abs(g).max()


def random_rotation(n, rng):
    Q, R = np.linalg.qr(rng.normal(size=(n, n)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_rotation_and_scaling(t):
    m = meshgen.small_mesh(*t, size=2)
    rng = np.random.default_rng(8)
    n, N = m["coords"].shape
    nu, H = rng.normal(size=(n, N)), rng.normal(size=N)
    f = oracle.kll(m, nu, H)
    R = random_rotation(n, rng)
    mr = dict(m, coords=R @ m["coords"])
    fr = oracle.kll(mr, R @ nu, H)
    sc = np.abs(f).max()
    assert np.abs(fr[:n] - R @ f[:n]).max() <= 1e-12 * sc
    assert np.abs(fr[n] - f[n]).max() <= 1e-12 * sc
    s = 1.7
    fs = oracle.kll(dict(m, coords=s * m["coords"]), nu, H)
    assert np.abs(fs - s ** (m["dim"] - 2) * f).max() <= 1e-12 * sc * max(1.0, s ** (m["dim"] - 2))


def test_linear_in_H_and_default():
    m = meshgen.small_mesh("surface", 2, 2, size=2)
    rng = np.random.default_rng(2)
    n, N = m["coords"].shape
    nu, H = rng.normal(size=(n, N)), rng.normal(size=N)
    f1 = oracle.kll(m, nu, None)
    fH = oracle.kll(m, nu, H)
    f2H1 = oracle.kll(m, nu, 2 * H + 1)
    assert np.array_equal(f1[:n], fH[:n])
    assert np.abs(f2H1[n] - (2 * fH[n] + f1[n])).max() <= 1e-12 * np.abs(f2H1[n]).max()


def kll_flow(level, tau, steps, bdf):
    """The linearly implicit BDF scheme for the coupled system (section 6.2)
    with the oracle's per-step system and a sparse LU solve; BDF1 for the
    first step of BDF2.  Returns the final positions and u = (nu; H)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    V, F = mg.icosphere_red(level, order=2)
    coords, conn = mg.to_soa(V, F)
    N = coords.shape[1]
    x = [coords.copy()]
    u = [np.vstack([coords / np.linalg.norm(coords, axis=0), 2.0 * np.ones((1, N))])]
    for n in range(steps):
        if bdf == 1 or n == 0:  # delta = (1, -1)
            d0, xt, ut, hist, xh = 1.0, x[-1], u[-1], -u[-1], -x[-1]
        else:  # delta = (3/2, -2, 1/2), extrapolation 2 y^{n-1} - y^{n-2}
            d0, xt, ut = 1.5, 2 * x[-1] - x[-2], 2 * u[-1] - u[-2]
            hist, xh = -2 * u[-1] + 0.5 * u[-2], -2 * x[-1] + 0.5 * x[-2]
        m = dict(domain="surface", dim=2, order=2, quad=6, coords=xt, conn=conn)
        (rp, ci, sv), f, rhs = oracle.kll_system(m, tau, d0, ut[:3], ut[3], hist)
        lu = spla.splu(sp.csr_matrix((sv, ci, rp), shape=(N, N)).tocsc())
        un = np.stack([lu.solve(rhs[c]) for c in range(4)])
        x.append((tau * (-un[3] * un[:3]) - xh) / d0)  # BDF derivative of x = v = -H nu
        u.append(un)
    return x[-1], u[-1]


def test_bdf_scheme_shrinks_sphere_with_its_order():
    tau, steps = 1e-3, 25
    exact = np.sqrt(1.0 - 4.0 * tau * steps)
    err = {}
    for bdf in (1, 2):
        x, u = kll_flow(2, tau, steps, bdf)
        r = np.linalg.norm(x, axis=0)
        err[bdf] = abs(r.mean() - exact)
        assert r.max() - r.min() < 1e-5  # stays round
        assert np.abs(u[3] - 2.0 / r).max() < 2e-3 * (2.0 / exact)
        assert np.abs(np.linalg.norm(u[:3], axis=0) - 1.0).max() < 5e-4
    assert err[1] < 1e-4
    assert err[2] < 5e-6
    assert err[2] < err[1] / 10


def test_kll_system_composition():
    """S = delta0 M + tau A on M's pattern, rhs = tau f - M hist, f the pinned
    non-linear terms; hist = None is a zero history."""
    m = meshgen.small_mesh("surface", 2, 2, size=2)
    n, N = m["coords"].shape
    rng = np.random.default_rng(2)
    nu, H, hist = rng.normal(size=(n, N)), rng.normal(size=N), rng.normal(size=(n + 1, N))
    (rp, ci, sv), f, rhs = oracle.kll_system(m, 0.25, 1.5, nu, H, hist)
    Mc, Ac = oracle.assemble(m, "mass"), oracle.assemble(m, "stiffness")
    assert np.array_equal(rp, Mc[0]) and np.array_equal(ci, Mc[1])
    assert np.abs(sv - (1.5 * Mc[2] + 0.25 * Ac[2])).max() <= 1e-15 * np.abs(sv).max()
    M = oracle.to_scipy(N, Mc).toarray()
    assert np.abs(f - oracle.kll(m, nu, H)).max() == 0
    assert np.abs(rhs - (0.25 * f - hist @ M.T)).max() <= 1e-14 * np.abs(rhs).max()
    _, _, rhs0 = oracle.kll_system(m, 0.25, 1.5, nu, H)
    assert np.array_equal(rhs0, 0.25 * f)
