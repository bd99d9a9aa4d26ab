"""The five seeded workloads and the small test meshes.

Every workload is a plain dict of NumPy arrays plus a few descriptors:

``domain``  "surface" or "bulk";  ``dim`` manifold dimension d;
``order``   1 or 2;  ``quad`` number of quadrature points of the rule;
``coords``  float64 (n_amb, N);  ``conn`` int32 (k, T);
optional nodal fields ``coef_c`` (weighted mass), ``coef_a`` (stiffness
coefficient), ``u``, ``v`` (adjoint test vectors).

Seeds: ``numpy.random.default_rng(SeedSequence(20260000 + k))`` for
workload k = 1..5; per-mesh sub-streams are spawned from it.
"""

from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y

from . import meshes as mg

SEED_BASE = 20260000


def _rng(k: int):
    return np.random.default_rng(np.random.SeedSequence(SEED_BASE + k))


def _pack(name, domain, dim, order, quad, V, F, **fields):
    coords, conn = mg.to_soa(V, F)
    d = dict(name=name, domain=domain, dim=dim, order=order, quad=quad,
             coords=coords, conn=conn)
    for key, val in fields.items():
        if val is not None:
            d[key] = np.ascontiguousarray(np.asarray(val, dtype=np.float64))
    return d


# --------------------------------------------------------------------------
# smooth radial displacement r = 1 + 0.2 sum_{l<=4} a_lm Y_lm
# --------------------------------------------------------------------------
def real_sph_harm(l: int, m: int, P: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic Y_lm at unit vectors P (N, 3), via
    SciPy (reference for the vectorised evaluation below)."""
    theta = np.arccos(np.clip(P[:, 2], -1.0, 1.0))
    phi = np.arctan2(P[:, 1], P[:, 0])
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    s = np.sqrt(2.0) * (-1.0) ** abs(m)
    return s * (np.real(y) if m > 0 else np.imag(y))


def real_sph_harm_all(lmax: int, P: np.ndarray):
    """All real orthonormal Y_lm, l <= lmax, at unit vectors P: dict (l, m) -> values.

    Associated Legendre functions without the Condon-Shortley phase by the
    standard three-term recurrence; Y_l0 = N_l0 P_l^0, Y_lm = sqrt2 N_lm P_l^m
    cos(m phi), Y_l,-m = sqrt2 N_lm P_l^m sin(m phi), N_lm^2 = (2l+1)/(4 pi)
    (l-m)!/(l+m)!  (the same functions as real_sph_harm)."""
    from math import factorial, pi, sqrt
    x = np.clip(P[:, 2], -1.0, 1.0)
    phi = np.arctan2(P[:, 1], P[:, 0])
    sx = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    out = {}
    for m in range(lmax + 1):
        pmm = np.full_like(x, float(np.prod(np.arange(1, 2 * m, 2)) if m > 0 else 1.0)) * sx ** m
        prev2, prev1 = None, pmm
        for l in range(m, lmax + 1):
            if l == m:
                plm = pmm
            elif l == m + 1:
                plm = x * (2 * m + 1) * pmm
            else:
                plm = ((2 * l - 1) * x * prev1 - (l + m - 1) * prev2) / (l - m)
            if l > m:
                prev2, prev1 = prev1, plm
            nlm = sqrt((2 * l + 1) / (4 * pi) * factorial(l - m) / factorial(l + m))
            if m == 0:
                out[(l, 0)] = nlm * plm
            else:
                out[(l, m)] = sqrt(2.0) * nlm * plm * np.cos(m * phi)
                out[(l, -m)] = sqrt(2.0) * nlm * plm * np.sin(m * phi)
    return out


def sh_coefficients(rng, lmax=4, sigma=0.3):
    return {(l, m): rng.normal(0.0, sigma) for l in range(lmax + 1) for m in range(-l, l + 1)}


def sh_radius(P_unit: np.ndarray, coeffs) -> np.ndarray:
    Y = real_sph_harm_all(max(l for l, _ in coeffs), P_unit)
    r = np.ones(len(P_unit))
    for (l, m), a in coeffs.items():
        r += 0.2 * a * Y[(l, m)]
    return r


def displaced_sphere(V, F, rng):
    """Project every node to S^2, then move it to r(x_hat) x_hat."""
    U = mg.normalize_rows(V)
    r = sh_radius(U, sh_coefficients(rng))
    return U * r[:, None], F


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config1():
    """P1 sphere: icosahedron red-refined 4x, radial noise +-1e-3, 3-point rule;
    c = 1 + 0.5 x1 x2 at the perturbed nodes."""
    rng = _rng(1)
    V, F = mg.icosphere_red(4, order=1)
    V, F, _ = mg.sfc_reorder(V, F)
    V = V * (1.0 + rng.uniform(-1e-3, 1e-3, size=len(V)))[:, None]
    c = 1.0 + 0.5 * V[:, 0] * V[:, 1]
    return _pack("p1_sphere_5120", "surface", 2, 1, 3, V, F, coef_c=c)


def config2():
    """P2 ellipsoid: icosahedron NVB x15 (655,360 triangles), P2 midpoints on
    S^2, all nodes scaled by diag(1, 0.8, 0.6); 6-point rule; c ~ U[0.5, 2]."""
    rng = _rng(2)
    V, F = mg.sphere_nvb(15, order=2)
    V, F, _ = mg.sfc_reorder(V, F)
    V = V * np.array([1.0, 0.8, 0.6])
    c = rng.uniform(0.5, 2.0, size=len(V))
    return _pack("p2_ellipsoid_655360", "surface", 2, 2, 6, V, F, coef_c=c)


def config3(n: int = 64, variant: str = "affine"):
    """P2 tetrahedra on [0,1]^3, n^3 Kuhn cells (6 tets each), 11-point rule.

    variant "affine": interior cell vertices jittered by U[-0.1h, 0.1h],
    edge nodes at midpoints of the jittered edges (elements stay affine).
    variant "curved": additionally every interior edge node is jittered by
    U[-0.05h, 0.05h] (amplitude 0.1 of the P2 node spacing h/2).
    a(x) = 1 + 0.5 sin(2 pi x) cos(2 pi y) z sampled at the nodes."""
    rng = _rng(3)
    h = 1.0 / n
    V, F, half = mg.kuhn_cube(n, order=2)
    V = mg.kuhn_jitter(V, half, n, 0.1 * h, rng)
    if variant == "curved":
        odd = ~np.all(half % 2 == 0, axis=1)
        inter = np.all((half > 0) & (half < 2 * n), axis=1)
        sel = odd & inter
        V[sel] += rng.uniform(-0.05 * h, 0.05 * h, size=(int(sel.sum()), 3))
    V, F, _ = mg.sfc_reorder(V, F)
    a = 1.0 + 0.5 * np.sin(2 * np.pi * V[:, 0]) * np.cos(2 * np.pi * V[:, 1]) * V[:, 2]
    return _pack(f"p2_kuhn_cube_{n}", "bulk", 3, 2, 11, V, F, coef_a=a)


def config4_sizes(count: int = 256):
    rng = _rng(4)
    T = np.exp(rng.uniform(np.log(2000.0), np.log(200000.0), size=count))
    freq = np.clip(np.round(np.sqrt(T / 20.0)), 10, 100).astype(int)
    return freq


def config4(count: int = 256):
    """256 geodesic spheres of log-uniform size, displaced by a random smooth
    radial field; even index P1 (3-point rule), odd index P2 (6-point rule)."""
    freq = config4_sizes(count)
    seqs = np.random.SeedSequence(SEED_BASE + 4).spawn(count)
    out = []
    for i in range(count):
        rng = np.random.default_rng(seqs[i])
        order = 1 if i % 2 == 0 else 2
        V, F = mg.sphere_geodesic(int(freq[i]), order=order)
        V, F, _ = mg.sfc_reorder(V, F)
        V, F = displaced_sphere(V, F, rng)
        out.append(_pack(f"batch_{i}_n{freq[i]}_p{order}", "surface", 2, order,
                         3 if order == 1 else 6, V, F))
    return out


def config5():
    """P2 sphere from NVB x13 (163,840 triangles) displaced by the radial
    field, u, v ~ N(0, 1) per node, 6-point rule."""
    rng = _rng(5)
    V, F = mg.sphere_nvb(13, order=2)
    V, F, _ = mg.sfc_reorder(V, F)
    V, F = displaced_sphere(V, F, rng)
    u = rng.normal(size=len(V))
    v = rng.normal(size=len(V))
    return _pack("p2_sphere_adjoint_163840", "surface", 2, 2, 6, V, F, u=u, v=v)


# --------------------------------------------------------------------------
# small meshes of all eight element types (tests)
# --------------------------------------------------------------------------
def small_mesh(domain: str, dim: int, order: int, size: int = 2, seed: int = 0,
               curved: bool = True):
    """A small valid mesh of the requested element type.

    surface d=1: closed curve (perturbed circle) in R^2
    surface d=2: perturbed red-refined icosphere in R^3
    bulk d=2:    jittered unit square
    bulk d=3:    jittered Kuhn cube
    With ``curved`` the P2 edge nodes are moved off the straight midpoints."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 99, seed, dim, order]))
    if domain == "surface" and dim == 1:
        V, F = mg.circle(4 * size + 3, order=order)
        V = V * (1.0 + 0.05 * rng.uniform(-1, 1, size=len(V)))[:, None]
        quad = 2 if order == 1 else 3
        n_amb = 2
    elif domain == "surface" and dim == 2:
        V, F = mg.icosphere_red(max(size - 1, 0), order=order)
        V = V * (1.0 + 0.05 * rng.uniform(-1, 1, size=len(V)))[:, None]
        quad = 3 if order == 1 else 6
        n_amb = 3
    elif domain == "bulk" and dim == 2:
        V, F = mg.square_tri(size + 1, order=1)
        h = 1.0 / (size + 1)
        inter = np.all((V > 1e-12) & (V < 1 - 1e-12), axis=1)
        V[inter] += rng.uniform(-0.15 * h, 0.15 * h, size=(int(inter.sum()), 2))
        if order == 2:
            V, F, _ = mg.p1_to_p2(V, F, mg.TRI_EDGES)
            if curved:
                mid = np.arange(len(V)) >= (size + 2) ** 2
                V[mid] += rng.uniform(-0.05 * h, 0.05 * h, size=(int(mid.sum()), 2))
        quad = 3 if order == 1 else 6
        n_amb = 2
    elif domain == "bulk" and dim == 3:
        n = max(size, 1)
        V, F, half = mg.kuhn_cube(n, order=order)
        if order == 1:
            half = half * 2
        V = mg.kuhn_jitter(V, half, n, 0.1 / n, rng) if order == 2 else V
        if order == 1:
            inter = np.all((V > 1e-12) & (V < 1 - 1e-12), axis=1)
            V[inter] += rng.uniform(-0.1 / n, 0.1 / n, size=(int(inter.sum()), 3))
        if order == 2 and curved:
            odd = ~np.all(half % 2 == 0, axis=1)
            V[odd] += rng.uniform(-0.04 / n, 0.04 / n, size=(int(odd.sum()), 3))
        quad = 4 if order == 1 else 11
        n_amb = 3
    else:
        raise ValueError((domain, dim))
    assert V.shape[1] == n_amb
    coef_c = 1.0 + 0.5 * np.sin(3 * V[:, 0]) * np.cos(2 * V[:, -1])
    coef_a = 1.5 + 0.5 * np.cos(2 * V[:, 0] + V[:, 1])
    u = rng.normal(size=len(V))
    v = rng.normal(size=len(V))
    return _pack(f"small_{domain}{dim}d_p{order}", domain, dim, order, quad, V, F,
                 coef_c=coef_c, coef_a=coef_a, u=u, v=v)


ALL_TYPES = [("surface", 1, 1), ("surface", 1, 2), ("surface", 2, 1), ("surface", 2, 2),
             ("bulk", 2, 1), ("bulk", 2, 2), ("bulk", 3, 1), ("bulk", 3, 2)]
