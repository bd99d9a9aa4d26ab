"""Pins of the oracle's load vector b_j = sum_E sum_q w mu f_h phi_j.

* exact rational integration on single affine elements of every type
  (b = M_exact f for nodal f, M_exact from the barycentric monomial formula);
* the paper's half-disk example and the unit cube: sum_j b_j with f = 1 is
  the area / volume (closed forms);
* partition of unity and interpolation identities against the mass matrix:
  b(1) = M 1 and b(f) = M f (f_h = sum_r f_r phi_r), on curved meshes of
  every type; linearity in f.
"""

from fractions import Fraction

import numpy as np
import pytest

import meshgen
import oracle
from meshgen import meshes as mg
from test_oracle_closed_forms import AFFINE_CASES, basis_poly, pint, pmul, read_half_disk, single


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("domain,dim,verts", AFFINE_CASES)
def test_load_affine_exact_rational(domain, dim, verts, order):
    X = [[Fraction(c) for c in v] for v in verts]
    n = len(X[0])
    J = np.array([[float(X[m + 1][c] - X[0][c]) for m in range(dim)] for c in range(n)])
    mu = np.sqrt(np.linalg.det(J.T @ J))
    phis = basis_poly(dim, order)
    k = len(phis)
    Mex = np.array([[float(pint(pmul(phis[a], phis[b]), dim)) for b in range(k)] for a in range(k)]) * mu
    Vf = np.array([[float(c) for c in v] for v in verts])
    m = single(domain, dim, order, Vf, [list(range(dim + 1))])
    rng = np.random.default_rng(7)
    f = rng.uniform(0.5, 2.0, size=m["coords"].shape[1])
    b = oracle.load(m, f)
    # nodes of the single element are 0..k-1 in element order
    conn = m["conn"][:, 0]
    bex = np.zeros_like(b)
    bex[conn] = Mex @ f[conn]
    assert np.abs(b - bex).max() <= 1e-14 * np.abs(bex).max()


def test_load_half_disk_area():
    V, F, formula = read_half_disk()
    coords, conn = mg.to_soa(V, F)
    mesh = dict(domain="bulk", dim=2, order=2, quad=6, coords=coords, conn=conn)
    expected = eval(formula, {"sqrt": np.sqrt})
    assert abs(oracle.load(mesh).sum() - expected) < 1e-15


def test_load_cube_volume():
    V, F, _ = mg.kuhn_cube(3, order=2)
    coords, conn = mg.to_soa(V, F)
    mesh = dict(domain="bulk", dim=3, order=2, quad=11, coords=coords, conn=conn)
    assert abs(oracle.load(mesh).sum() - 1.0) < 1e-14


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_load_against_mass(t):
    m = meshgen.small_mesh(*t, size=3)
    N = m["coords"].shape[1]
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    ones = oracle.load(m)
    assert np.abs(ones - M @ np.ones(N)).max() <= 1e-14 * np.abs(ones).max()
    rng = np.random.default_rng(3)
    f, g = rng.normal(size=N), rng.normal(size=N)
    bf, bg = oracle.load(m, f), oracle.load(m, g)
    assert np.abs(bf - M @ f).max() <= 1e-13 * np.abs(M @ f).max()
    assert np.abs(oracle.load(m, 2 * f + g) - (2 * bf + bg)).max() <= 1e-13 * np.abs(bf).max()
