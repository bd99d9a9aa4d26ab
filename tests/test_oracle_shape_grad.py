"""Pins of the oracle's shape derivative of J(x) = alpha u^T A(x) v + beta w^T M(x) z.

* central finite differences of the oracle energy (h = 1e-6), relative 1e-6
  per sampled (node, component), scale max(|g_fd|, 1e-3 ||g||_inf);
* translation invariance: sum_r g_r = 0 (each component);
* rotation invariance: sum_r x_r x g_r = 0 (R^3), sum_r x_r ^ g_r = 0 (R^2);
* scaling (Euler's theorem: A is homogeneous of degree d - 2, M of degree d):
  sum_r x_r . g_r = (d - 2) alpha u^T A v + d beta w^T M z;
* the energy equals the quadratic forms of the assembled matrices.
"""

import numpy as np
import pytest

import meshgen
import oracle


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_energy_matches_matrices(t):
    m = meshgen.small_mesh(*t)
    N = m["coords"].shape[1]
    u, v = m["u"], m["v"]
    A = oracle.to_scipy(N, oracle.assemble(m, "stiffness"))
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    J = oracle.energy(m, u, v, 0.7, v, u, -1.3)
    ref = 0.7 * u @ (A @ v) - 1.3 * v @ (M @ u)
    assert abs(J - ref) <= 1e-13 * (abs(0.7 * u @ (A @ v)) + abs(1.3 * v @ (M @ u)))


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_against_central_differences(t):
    m = meshgen.small_mesh(*t)
    X = m["coords"]
    n, N = X.shape
    u, v = m["u"], m["v"]
    args = (u, u, 1.0, v, v, 1.0)
    g = oracle.shape_grad(m, *args)
    gmax = np.abs(g).max()
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(12):
        r = int(rng.integers(N))
        c = int(rng.integers(n))
        mp_, mm_ = dict(m), dict(m)
        Xp, Xm = X.copy(), X.copy()
        Xp[c, r] += h
        Xm[c, r] -= h
        mp_["coords"], mm_["coords"] = Xp, Xm
        fd = (oracle.energy(mp_, *args, long_double=True)
              - oracle.energy(mm_, *args, long_double=True)) / (2 * h)
        assert abs(g[c, r] - fd) <= 1e-7 * max(abs(fd), 1e-3 * gmax), (r, c, g[c, r], fd)


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_invariances(t):
    m = meshgen.small_mesh(*t)
    X = m["coords"]
    n = X.shape[0]
    d = m["dim"]
    u, v, w, z = m["u"], m["v"], m["coef_c"], m["coef_a"]
    alpha, beta = 0.8, 1.9
    g = oracle.shape_grad(m, u, v, alpha, w, z, beta)
    scale = np.abs(g).max() * np.abs(X).max() * X.shape[1]
    assert np.abs(g.sum(1)).max() <= 1e-13 * np.abs(g).max() * X.shape[1]
    if n == 3:
        rot = np.cross(X.T, g.T).sum(0)
        assert np.abs(rot).max() <= 1e-13 * scale
    else:
        rot = (X[0] * g[1] - X[1] * g[0]).sum()
        assert abs(rot) <= 1e-13 * scale
    N = X.shape[1]
    A = oracle.to_scipy(N, oracle.assemble(m, "stiffness"))
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    euler = (d - 2) * alpha * u @ (A @ v) + d * beta * w @ (M @ z)
    assert abs((X * g).sum() - euler) <= 1e-12 * scale
