"""Invariants that fix the oracle on curved meshes of all eight element types.

P4  1^T M 1 = measure (cube volume 1; sum of flat triangle areas for P1 surfaces)
P5  A 1 = 0, A_a 1 = 0
P6  sum_k x_k^T A x_k = d 1^T M 1 (isoparametric elements reproduce linear
    functions and the tangential projection has trace d); weighted analogue
P9  M_c with c = 1 equals M; M_c is linear in c; A_a with a = 1 equals A
P10 symmetry
P11 rigid motions leave M, A unchanged; x -> s x scales M by s^d, A by s^(d-2)
P12 CSR nnz closed forms: closed triangulated surface P1: V + 2E, P2: V + 15E;
    Kuhn cube P2: 230 n^3 + 138 n^2 + 24 n + 1; P1 (n=64): 4,018,753.
"""

import numpy as np
import pytest

import meshgen
import oracle
from meshgen import meshes as mg

TYPES = meshgen.ALL_TYPES


def mats(mesh, coef_c=None, coef_a=None):
    N = mesh["coords"].shape[1]
    M = oracle.to_scipy(N, oracle.assemble(mesh, "mass", coef=coef_c))
    A = oracle.to_scipy(N, oracle.assemble(mesh, "stiffness", coef=coef_a))
    return M, A


@pytest.mark.parametrize("t", TYPES)
def test_linear_reproduction_and_kernel(t):
    mesh = meshgen.small_mesh(*t)
    X = mesh["coords"]
    N = X.shape[1]
    d = mesh["dim"]
    M, A = mats(mesh)
    one = np.ones(N)
    area = one @ (M @ one)
    assert np.abs(A @ one).max() <= 1e-13 * abs(A).max()
    lhs = sum(X[c] @ (A @ X[c]) for c in range(X.shape[0]))
    assert abs(lhs - d * area) <= 1e-13 * d * area
    # weighted versions
    Ma, Aa = mats(mesh, coef_c=mesh["coef_a"], coef_a=mesh["coef_a"])
    assert np.abs(Aa @ one).max() <= 1e-13 * abs(Aa).max()
    lhs = sum(X[c] @ (Aa @ X[c]) for c in range(X.shape[0]))
    assert abs(lhs - d * (one @ (Ma @ one))) <= 1e-13 * d * area * 2
    # symmetry (exact: the oracle computes (a,b) and (b,a) with the same operations)
    assert abs(M - M.T).max() <= 1e-16 * abs(M).max()
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()


@pytest.mark.parametrize("t", TYPES)
def test_coefficient_identities(t):
    mesh = meshgen.small_mesh(*t)
    N = mesh["coords"].shape[1]
    M, A = mats(mesh)
    M1, A1 = mats(mesh, coef_c=np.ones(N), coef_a=np.ones(N))
    assert abs(M - M1).max() <= 1e-15 * abs(M).max()
    assert abs(A - A1).max() <= 1e-14 * abs(A).max()
    c1, c2 = mesh["coef_c"], mesh["coef_a"]
    Ma, _ = mats(mesh, coef_c=c1)
    Mb, _ = mats(mesh, coef_c=c2)
    Mab, _ = mats(mesh, coef_c=2 * c1 - 3 * c2)
    assert abs(Mab - (2 * Ma - 3 * Mb)).max() <= 1e-14 * abs(Mab).max()


@pytest.mark.parametrize("t", TYPES)
def test_rigid_motion_and_scaling(t):
    mesh = meshgen.small_mesh(*t)
    X = mesh["coords"]
    n = X.shape[0]
    d = mesh["dim"]
    M, A = mats(mesh)
    rng = np.random.default_rng(7)
    R = np.linalg.qr(rng.normal(size=(n, n)))[0]
    moved = dict(mesh)
    moved["coords"] = np.ascontiguousarray(R @ X + rng.normal(size=(n, 1)))
    M2, A2 = mats(moved)
    assert abs(M - M2).max() <= 1e-13 * abs(M).max()
    assert abs(A - A2).max() <= 1e-12 * abs(A).max()
    s = 1.7
    scaled = dict(mesh)
    scaled["coords"] = np.ascontiguousarray(s * X)
    M3, A3 = mats(scaled)
    assert abs(M3 - s ** d * M).max() <= 1e-14 * abs(M3).max()
    assert abs(A3 - s ** (d - 2) * A).max() <= 1e-13 * abs(A3).max()


def test_p1_surface_area_is_flat_area():
    m = meshgen.config1()
    V = m["coords"].T
    F = m["conn"].T
    M, _ = mats(m)
    one = np.ones(V.shape[0])
    flat = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1).sum()
    assert abs(one @ (M @ one) - flat) < 1e-13 * flat


@pytest.mark.parametrize("variant", ["affine", "curved"])
def test_cube_volume_is_one(variant):
    m = meshgen.config3(n=4, variant=variant)
    rp, ci, va = oracle.assemble(m, "mass")
    assert abs(va.sum() - 1.0) < 1e-14


def _edges(F):
    E = set()
    for tri in F:
        for i, j in ((0, 1), (1, 2), (2, 0)):
            E.add(tuple(sorted((int(tri[i]), int(tri[j])))))
    return E


@pytest.mark.parametrize("order", [1, 2])
def test_nnz_closed_surface(order):
    V, F = mg.sphere_nvb(5, order=1)
    nV, nE = len(V), len(_edges(F))
    m = meshgen.small_mesh("surface", 2, order, size=3)
    V2, F2 = mg.sphere_nvb(5, order=order)
    coords, conn = mg.to_soa(V2, F2)
    mesh = dict(domain="surface", dim=2, order=order, quad=3, coords=coords, conn=conn)
    rp, ci, va = oracle.assemble(mesh, "mass")
    assert len(ci) == (nV + 2 * nE if order == 1 else nV + 15 * nE)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_nnz_kuhn_p2(n):
    V, F, half = mg.kuhn_cube(n, order=2)
    coords, conn = mg.to_soa(V, F)
    mesh = dict(domain="bulk", dim=3, order=2, quad=4, coords=coords, conn=conn)
    rp, ci, va = oracle.assemble(mesh, "mass")
    assert len(ci) == 230 * n ** 3 + 138 * n ** 2 + 24 * n + 1
    # pattern: sorted columns, diagonal present
    for i in range(len(rp) - 1):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i in row


@pytest.mark.parametrize("t", TYPES)
def test_numeric_only_equals_coo_route(t):
    """Assembling into the prebuilt pattern (slot by binary search) gives the
    values of the COO + stable sort route: the same sums in the same (element)
    order, so the same bits."""
    mesh = meshgen.small_mesh(*t, size=3)
    for kind, coef in (("mass", None), ("stiffness", None), ("mass", mesh["coef_c"]),
                       ("stiffness", mesh["coef_a"])):
        rp, ci, va = oracle.assemble(mesh, kind, coef=coef)
        vn = oracle.assemble_numeric(mesh, kind, (rp, ci), coef=coef)
        assert np.array_equal(vn, va), (kind, coef is not None)
