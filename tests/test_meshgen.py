"""The seeded workloads have the stated sizes and are valid meshes."""

import numpy as np
import pytest

import meshgen
from meshgen import meshes as mg


def _edge_count(F):
    e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    return len(uniq), cnt


@pytest.mark.parametrize("rounds", [1, 2, 5, 8])
def test_nvb_conforming_closed_surface(rounds):
    V, F = mg.sphere_nvb(rounds)
    assert len(F) == 20 * 2 ** rounds
    nE, cnt = _edge_count(F)
    assert np.all(cnt == 2)  # conforming, closed
    assert len(V) - nE + len(F) == 2  # Euler characteristic of S^2
    assert len(V) == len(F) // 2 + 2
    # outward orientation kept
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    assert np.all(np.einsum("ij,ij->i", n, V[F].mean(1)) > 0)


@pytest.mark.parametrize("freq", [1, 3, 10])
def test_geodesic_sphere(freq):
    V, F = mg.geodesic_sphere(freq)
    assert len(F) == 20 * freq ** 2 and len(V) == 10 * freq ** 2 + 2
    nE, cnt = _edge_count(F)
    assert np.all(cnt == 2)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    assert np.all(np.einsum("ij,ij->i", n, V[F].mean(1)) > 0)


def test_red_refinement_sizes():
    V, F = mg.icosphere_red(4)
    assert (len(V), len(F)) == (2562, 5120)


def test_config_sizes_small():
    c1 = meshgen.config1()
    assert c1["coords"].shape == (3, 2562) and c1["conn"].shape == (3, 5120)
    r = np.linalg.norm(c1["coords"], axis=0)
    assert np.all(np.abs(r - 1) <= 1e-3 + 1e-15)


@pytest.mark.slow
def test_config_sizes_large():
    c2 = meshgen.config2()
    assert c2["coords"].shape == (3, 1310722) and c2["conn"].shape == (6, 655360)
    x, y, z = c2["coords"]
    assert np.abs(x ** 2 + y ** 2 / 0.64 + z ** 2 / 0.36 - 1).max() < 1e-14
    c5 = meshgen.config5()
    assert c5["coords"].shape == (3, 327682) and c5["conn"].shape == (6, 163840)


def test_kuhn_cube_p2_counts():
    V, F, half = mg.kuhn_cube(4, order=2)
    assert F.shape == (6 * 64, 10) and len(V) == 9 ** 3
    # positive orientation of every tet
    P = V[F[:, :4]]
    det = np.linalg.det(np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], 1))
    assert np.all(det > 0)
    # every P2 node is the midpoint of its edge
    for s, (i, j) in enumerate(mg.TET_EDGES):
        assert np.allclose(V[F[:, 4 + s]], 0.5 * (V[F[:, i]] + V[F[:, j]]))


def test_config4_sizes():
    freq = meshgen.config4_sizes()
    assert len(freq) == 256 and freq.min() >= 10 and freq.max() <= 100


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_small_meshes_valid(t):
    m = meshgen.small_mesh(*t)
    k = m["conn"].shape[0]
    assert k == {1: 2, 2: 3, 3: 4}[t[1]] if t[2] == 1 else True
    assert m["conn"].min() >= 0 and m["conn"].max() < m["coords"].shape[1]
    # no repeated node inside an element
    Fs = np.sort(m["conn"].T, axis=1)
    assert np.all(np.diff(Fs, axis=1) > 0)


def test_vectorised_spherical_harmonics():
    from meshgen import configs as cf
    rng = np.random.default_rng(0)
    P = rng.normal(size=(500, 3))
    P /= np.linalg.norm(P, axis=1)[:, None]
    Y = cf.real_sph_harm_all(4, P)
    for l in range(5):
        for m in range(-l, l + 1):
            assert np.abs(Y[(l, m)] - cf.real_sph_harm(l, m, P)).max() < 1e-12
