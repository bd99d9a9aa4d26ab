"""Pins of the oracle's reference basis (section 3.1: nodal Lagrange basis,
phi_j(x_i) = delta_ij, node order of section 4.1)."""

import numpy as np
import pytest

import oracle

TYPES = [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2)]

SEG_EDGES = [(0, 1)]
TRI_EDGES = [(0, 1), (1, 2), (2, 0)]
TET_EDGES = [(0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3)]


def ref_nodes(d, p):
    corners = [np.zeros(d)] + [np.eye(d)[i] for i in range(d)]
    if p == 1:
        return np.array(corners)
    edges = {1: SEG_EDGES, 2: TRI_EDGES, 3: TET_EDGES}[d]
    mids = [(corners[a] + corners[b]) / 2 for a, b in edges]
    return np.array(corners + mids)


@pytest.mark.parametrize("d,p", TYPES)
def test_nodal(d, p):
    X = ref_nodes(d, p)
    for b, x in enumerate(X):
        phi, _ = oracle.basis(d, p, x)
        e = np.zeros(len(X))
        e[b] = 1
        assert np.allclose(phi, e, atol=1e-15)


@pytest.mark.parametrize("d,p", TYPES)
def test_partition_of_unity_and_gradients(d, p):
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.dirichlet(np.ones(d + 1))[1:]
        phi, dphi = oracle.basis(d, p, x)
        assert abs(phi.sum() - 1) < 1e-14
        assert np.allclose(dphi.sum(0), 0, atol=1e-13)
        # gradients against central differences of the values
        h = 1e-6
        for m in range(d):
            e = np.zeros(d)
            e[m] = h
            fd = (oracle.basis(d, p, x + e)[0] - oracle.basis(d, p, x - e)[0]) / (2 * h)
            assert np.allclose(dphi[:, m], fd, atol=1e-8)
        # reproduces linear functions: sum_a xi(node_a) phi_a = xi
        X = ref_nodes(d, p)
        assert np.allclose(X.T @ phi, x, atol=1e-14)
        assert np.allclose(X.T @ dphi, np.eye(d), atol=1e-13)
