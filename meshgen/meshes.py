"""Seeded synthetic meshes (host only, NumPy).

This module builds the inputs that both the CPU oracle and the GPU library
read.  It holds no finite-element arithmetic: only mesh topology
(refinement, P1 -> P2 node insertion), node placement (projections,
jitter) and node/element orderings.

Array conventions (the paper's node array N and element array E, section 4,
stored structure-of-arrays and 0-based):

* ``coords``: float64, shape ``(n_amb, N)`` -- row ``c`` holds coordinate
  ``c`` of every node (the paper's column-major ``N(:, c)``).
* ``conn``: int32, shape ``(k, T)`` -- row ``a`` holds the global id of
  local node ``a`` of every element.  Corners come first in
  anticlockwise order, then the edge nodes (section 4.1):
  segment (end0, end1, mid);
  triangle edges (0,1), (1,2), (2,0);
  tetrahedron edges (0,1), (1,2), (0,2), (0,3), (1,3), (2,3).
"""

from __future__ import annotations

import itertools

import numpy as np

TRI_EDGES = ((0, 1), (1, 2), (2, 0))
TET_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))
SEG_EDGES = ((0, 1),)


# --------------------------------------------------------------------------
# small helpers
# --------------------------------------------------------------------------
def to_soa(V: np.ndarray, F: np.ndarray):
    """(N, n_amb), (T, k) -> SoA float64 (n_amb, N) and int32 (k, T)."""
    coords = np.ascontiguousarray(np.asarray(V, dtype=np.float64).T)
    conn = np.ascontiguousarray(np.asarray(F, dtype=np.int64).T.astype(np.int32))
    return coords, conn


def normalize_rows(V: np.ndarray) -> np.ndarray:
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def _edge_keys(a: np.ndarray, b: np.ndarray, n: int) -> np.ndarray:
    lo = np.minimum(a, b).astype(np.int64)
    hi = np.maximum(a, b).astype(np.int64)
    return lo * n + hi


# --------------------------------------------------------------------------
# icosahedron and sphere refinements
# --------------------------------------------------------------------------
def icosahedron():
    """Unit icosahedron: V (12, 3), F (20, 3) oriented with outward normals."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    V = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            V.append((0.0, s1, s2 * p))
            V.append((s1, s2 * p, 0.0))
            V.append((s2 * p, 0.0, s1))
    V = np.array(V, dtype=np.float64)
    F = []
    for a, b, c in itertools.combinations(range(12), 3):
        if (abs(np.linalg.norm(V[a] - V[b]) - 2.0) < 1e-9
                and abs(np.linalg.norm(V[b] - V[c]) - 2.0) < 1e-9
                and abs(np.linalg.norm(V[c] - V[a]) - 2.0) < 1e-9):
            n = np.cross(V[b] - V[a], V[c] - V[a])
            F.append((a, b, c) if n @ (V[a] + V[b] + V[c]) > 0 else (a, c, b))
    F = np.array(F, dtype=np.int64)
    assert F.shape == (20, 3)
    return normalize_rows(V), F


def red_refine(V, F, project=True):
    """Each triangle -> 4 (edge midpoints), midpoints optionally put on S^2."""
    nV = len(V)
    v0, v1, v2 = F[:, 0], F[:, 1], F[:, 2]
    keys = np.concatenate([_edge_keys(v0, v1, nV), _edge_keys(v1, v2, nV),
                           _edge_keys(v2, v0, nV)])
    uniq, inv = np.unique(keys, return_inverse=True)
    a, b = uniq // nV, uniq % nV
    M = 0.5 * (V[a] + V[b])
    if project:
        M = normalize_rows(M)
    T = len(F)
    m01, m12, m20 = (nV + inv[:T], nV + inv[T:2 * T], nV + inv[2 * T:])
    F2 = np.concatenate([
        np.stack([v0, m01, m20], 1), np.stack([m01, v1, m12], 1),
        np.stack([m20, m12, v2], 1), np.stack([m01, m12, m20], 1)])
    return np.concatenate([V, M]), F2


def _dual_perfect_matching(F):
    """A perfect matching of the face-adjacency graph (small meshes only)."""
    T = len(F)
    edge_faces = {}
    for f in range(T):
        for (i, j) in TRI_EDGES:
            e = tuple(sorted((int(F[f, i]), int(F[f, j]))))
            edge_faces.setdefault(e, []).append(f)
    nbr = [[] for _ in range(T)]
    for e, fs in edge_faces.items():
        assert len(fs) == 2
        nbr[fs[0]].append((fs[1], e))
        nbr[fs[1]].append((fs[0], e))
    mate = [None] * T

    def solve():
        free = [f for f in range(T) if mate[f] is None]
        if not free:
            return True
        f = free[0]
        for g, e in nbr[f]:
            if mate[g] is None:
                mate[f] = mate[g] = e
                if solve():
                    return True
                mate[f] = mate[g] = None
        return False

    assert solve()
    return mate


def nvb_initial_labelling(F):
    """Rotate each face so that local vertex 0 is opposite its refinement edge.

    The refinement edges form a perfect matching of the dual graph, which is
    the compatibility condition that keeps uniform newest-vertex bisection
    conforming at every level.
    """
    mate = _dual_perfect_matching(F)
    F2 = F.copy()
    for f in range(len(F)):
        e = set(mate[f])
        for r in range(3):
            t = np.roll(F[f], -r)
            if {int(t[1]), int(t[2])} == e:
                F2[f] = t
                break
        else:
            raise AssertionError("labelling failed")
    return F2


def nvb_refine(V, F, rounds, project=True):
    """Uniform newest-vertex bisection; F rows are (newest, r0, r1)."""
    for _ in range(rounds):
        nV = len(V)
        v0, v1, v2 = F[:, 0], F[:, 1], F[:, 2]
        uniq, inv = np.unique(_edge_keys(v1, v2, nV), return_inverse=True)
        a, b = uniq // nV, uniq % nV
        M = 0.5 * (V[a] + V[b])
        if project:
            M = normalize_rows(M)
        m = nV + inv
        F = np.concatenate([np.stack([m, v0, v1], 1), np.stack([m, v2, v0], 1)])
        V = np.concatenate([V, M])
    return V, F


def geodesic_sphere(freq: int):
    """Frequency-n geodesic icosphere: every icosahedron face cut into n^2
    triangles, all nodes projected to S^2.  T = 20 n^2, V = 10 n^2 + 2."""
    V0, F0 = icosahedron()
    n = int(freq)
    ii, jj = [], []
    for i in range(n + 1):
        for j in range(n + 1 - i):
            ii.append(i)
            jj.append(j)
    ii = np.array(ii)
    jj = np.array(jj)
    loc = -np.ones((n + 1, n + 1), dtype=np.int64)
    loc[ii, jj] = np.arange(len(ii))
    P = len(ii)
    # integer barycentric key of every (face, local point)
    ids = np.repeat(F0, P, axis=0).reshape(20, P, 3)
    w = np.stack([n - ii - jj, ii, jj], 1)[None].repeat(20, 0)
    ids = np.where(w == 0, 15, ids)
    order = np.argsort(ids, axis=2, kind="stable")
    ids_s = np.take_along_axis(ids, order, 2)
    w_s = np.take_along_axis(w, order, 2)
    key = np.zeros((20, P), dtype=np.int64)
    for s in range(3):
        key |= ((ids_s[:, :, s] << 8) | w_s[:, :, s]) << (12 * s)
    uniq, first, inv = np.unique(key.ravel(), return_index=True, return_inverse=True)
    inv = inv.reshape(20, P)
    pts = np.zeros((len(uniq), 3))
    flat_w = w.reshape(-1, 3)
    flat_f = np.repeat(np.arange(20), P)
    src = F0[flat_f[first]]
    ww = flat_w[first].astype(np.float64) / n
    pts = (ww[:, 0:1] * V0[src[:, 0]] + ww[:, 1:2] * V0[src[:, 1]]
           + ww[:, 2:3] * V0[src[:, 2]])
    pts = normalize_rows(pts)
    tris = []
    for i in range(n):
        for j in range(n - i):
            tris.append((loc[i, j], loc[i + 1, j], loc[i, j + 1]))
            if i + j <= n - 2:
                tris.append((loc[i + 1, j], loc[i + 1, j + 1], loc[i, j + 1]))
    tris = np.array(tris, dtype=np.int64)
    F = inv[:, tris].reshape(-1, 3)
    return pts, F


# --------------------------------------------------------------------------
# P1 -> P2
# --------------------------------------------------------------------------
def p1_to_p2(V, F, edges):
    """Append one node per distinct edge (at the straight midpoint)."""
    nV = len(V)
    keys = np.concatenate([_edge_keys(F[:, i], F[:, j], nV) for (i, j) in edges])
    uniq, inv = np.unique(keys, return_inverse=True)
    a, b = uniq // nV, uniq % nV
    M = 0.5 * (V[a] + V[b])
    T = len(F)
    mids = np.stack([nV + inv[s * T:(s + 1) * T] for s in range(len(edges))], 1)
    return np.concatenate([V, M]), np.concatenate([F, mids], 1), (a, b)


# --------------------------------------------------------------------------
# P1 -> P3, P4 (segments and triangles)
# --------------------------------------------------------------------------
TET_FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))


def tet_lattice_alphas(p):
    """Barycentric multi-indices (|alpha| = p) of the local nodes of an order-p
    tetrahedron: vertices; per edge of TET_EDGES its p - 1 nodes from the
    edge's first vertex; per face of TET_FACES its inner nodes (p = 3: (1,1,1);
    p = 4: (2,1,1), (1,2,1), (1,1,2) on the face's vertices); the inner node
    (1,1,1,1) for p = 4."""
    out = []
    for i in range(4):
        a = [0] * 4
        a[i] = p
        out.append(a)
    for u, v in TET_EDGES:
        for i in range(1, p):
            a = [0] * 4
            a[u], a[v] = p - i, i
            out.append(a)
    for f in TET_FACES:
        inner = [(1, 1, 1)] if p == 3 else [(2, 1, 1), (1, 2, 1), (1, 1, 2)] if p == 4 else []
        for w in inner:
            a = [0] * 4
            for j, vert in enumerate(f):
                a[vert] = w[j]
            out.append(a)
    if p == 4:
        out.append([1, 1, 1, 1])
    return out


def _tet_to_pp(V, F, p):
    """Order-p lattice nodes of straight tetrahedra.  A node is identified by
    its barycentric position over global vertex ids, so nodes on shared edges
    and faces are created once."""
    alphas = tet_lattice_alphas(p)
    ids = {}
    coords = list(V)
    conn = np.zeros((len(F), len(alphas)), dtype=np.int64)
    for e, g in enumerate(F):
        for a, al in enumerate(alphas):
            key = tuple(sorted((int(g[j]), al[j]) for j in range(4) if al[j] > 0))
            if len(key) == 1:
                conn[e, a] = key[0][0]
                continue
            n = ids.get(key)
            if n is None:
                n = len(coords)
                ids[key] = n
                coords.append(sum(al[j] * V[g[j]] for j in range(4)) / p)
            conn[e, a] = n
    return np.array(coords), conn


def p1_to_pp(V, F, p, edges):
    """Lattice nodes of order p (3 or 4) on straight segments / triangles /
    tetrahedra.

    Local order: vertices; then for each local edge (u, v) of ``edges`` its
    p - 1 nodes from u to v (barycentric position (p - i, i) / p on the
    edge, i = 1..p-1); then interior triangle nodes, p = 3: (1,1,1)/3,
    p = 4: (2,1,1)/4, (1,2,1)/4, (1,1,2)/4; tetrahedra: edge nodes, then
    the face and interior nodes of tet_lattice_alphas.  Nodes on an edge
    are created once per distinct edge, from its lower to its higher vertex
    id, and each element takes them in its own direction."""
    if F.shape[1] == 4:
        assert tuple(map(tuple, edges)) == TET_EDGES
        return _tet_to_pp(np.asarray(V, dtype=np.float64), np.asarray(F), p)
    nV, T = len(V), len(F)
    keys = np.concatenate([_edge_keys(F[:, i], F[:, j], nV) for (i, j) in edges])
    uniq, inv = np.unique(keys, return_inverse=True)
    lo, hi = uniq // nV, uniq % nV
    ne = len(uniq)
    # node i (1..p-1) of distinct edge g sits at (p - i, i) / p from lo to hi
    newV = [V]
    for i in range(1, p):
        newV.append(((p - i) * V[lo] + i * V[hi]) / p)
    cols = [F]
    for s_, (u, v) in enumerate(edges):
        g = inv[s_ * T:(s_ + 1) * T]
        forward = F[:, u] < F[:, v]
        for i in range(1, p):
            idx = np.where(forward, i, p - i)       # position counted from lo
            cols.append((nV + (idx - 1) * ne + g)[:, None])
    out_V = np.concatenate(newV)
    if F.shape[1] == 3:
        base = len(out_V)
        A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
        if p == 3:
            interior = [(A + B + C) / 3.0]
        else:
            interior = [(2 * A + B + C) / 4.0, (A + 2 * B + C) / 4.0, (A + B + 2 * C) / 4.0]
        for n_i, P in enumerate(interior):
            cols.append((base + n_i * T + np.arange(T))[:, None])
        out_V = np.concatenate([out_V] + interior)
    return out_V, np.concatenate(cols, 1)


# --------------------------------------------------------------------------
# locality ordering (space-filling curve)
# --------------------------------------------------------------------------
def _spread3(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64) & np.uint64(0x1FFFFF)
    x = (x | (x << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x1249249249249249)
    return x


def morton_keys(P: np.ndarray) -> np.ndarray:
    P = np.asarray(P, dtype=np.float64)
    if P.shape[1] < 3:
        P = np.concatenate([P, np.zeros((len(P), 3 - P.shape[1]))], 1)
    lo = P.min(0)
    span = np.maximum(P.max(0) - lo, 1e-300)
    q = np.floor((P - lo) / span * (2 ** 21 - 1)).astype(np.int64)
    return _spread3(q[:, 0]) | (_spread3(q[:, 1]) << np.uint64(1)) | (_spread3(q[:, 2]) << np.uint64(2))


def sfc_reorder(V, F, extra=()):
    """Renumber nodes and elements along a Morton curve (locality order).

    ``extra`` are per-node arrays permuted alongside ``V``."""
    perm = np.argsort(morton_keys(V), kind="stable")
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    V2 = V[perm]
    F2 = inv[F]
    cen = V2[F2[:, :min(F2.shape[1], 4)]].mean(1) if F2.shape[1] > 1 else V2[F2[:, 0]]
    eperm = np.argsort(morton_keys(cen), kind="stable")
    F2 = F2[eperm]
    return V2, F2, [np.asarray(x)[perm] for x in extra]


# --------------------------------------------------------------------------
# named mesh families
# --------------------------------------------------------------------------
def icosphere_red(refinements: int, order: int = 1):
    V, F = icosahedron()
    for _ in range(refinements):
        V, F = red_refine(V, F, project=True)
    if order == 2:
        V, F, _ = p1_to_p2(V, F, TRI_EDGES)
        V = normalize_rows(V)
    return V, F


def sphere_nvb(rounds: int, order: int = 1):
    V, F = icosahedron()
    F = nvb_initial_labelling(F)
    V, F = nvb_refine(V, F, rounds, project=True)
    if order == 2:
        V, F, _ = p1_to_p2(V, F, TRI_EDGES)
        V = normalize_rows(V)
    return V, F


def sphere_geodesic(freq: int, order: int = 1):
    V, F = geodesic_sphere(freq)
    if order == 2:
        V, F, _ = p1_to_p2(V, F, TRI_EDGES)
        V = normalize_rows(V)
    return V, F


def circle(n: int, order: int = 1):
    """Closed polygon with n segments on the unit circle (a curve in R^2)."""
    t = 2 * np.pi * np.arange(n) / n
    V = np.stack([np.cos(t), np.sin(t)], 1)
    F = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    if order == 2:
        V, F, _ = p1_to_p2(V, F, SEG_EDGES)
        V = normalize_rows(V)
    return V, F


def square_tri(n: int, order: int = 1):
    """Unit square, n x n cells, each cut into two anticlockwise triangles."""
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="xy")
    V = np.stack([X.ravel(), Y.ravel()], 1)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[:-1, 1:].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[1:, :-1].ravel()
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    if order == 2:
        V, F, _ = p1_to_p2(V, F, TRI_EDGES)
    return V, F


def half_disk_paper():
    """The two-element P2 half-disk of the paper's worked example (section 4.1,
    element and coordinate tables), 0-based.  The printed coordinates of
    nodes 6 and 9 are read as (-sqrt2/2, sqrt2/2) and (sqrt2/2, sqrt2/2), the
    points on the unit circle that the accompanying figure shows."""
    r = 0.5 * 2.0 ** 0.5
    V = np.array([[-1, 0], [0, 0], [0, 1], [-0.5, 0], [0, 0.5], [-r, r],
                  [1, 0], [0.5, 0], [r, r]], dtype=np.float64)
    F = np.array([[1, 2, 3, 4, 5, 6], [2, 7, 3, 8, 9, 5]], dtype=np.int64) - 1
    return V, F


def kuhn_cube(n: int, order: int = 1):
    """[0,1]^3 with n^3 cells, each split into the 6 Kuhn tetrahedra that share
    the cell diagonal (0,0,0)-(1,1,1).  Returns (V, F, half) where ``half`` is
    the integer half-grid coordinate (0..2n) of every node.

    P2 nodes are the half-grid points: every half-grid point is the midpoint
    of exactly one Kuhn edge (axis edge, face diagonal or cell diagonal)."""
    m = 2 * n + 1  # half-grid points per axis
    def hid(I, J, K):
        return I + m * (J + m * K)
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = []
    unit = np.eye(3, dtype=np.int64)
    for perm in itertools.permutations(range(3)):
        p0 = np.zeros(3, dtype=np.int64)
        p1 = unit[perm[0]]
        p2 = p1 + unit[perm[1]]
        p3 = np.ones(3, dtype=np.int64)
        corners = [p0, p1, p2, p3]
        # orientation: positive determinant of (p1-p0, p2-p0, p3-p0)
        det = np.linalg.det(np.stack([p1 - p0, p2 - p0, p3 - p0]).astype(float))
        if det < 0:
            corners = [p0, p2, p1, p3]
        tets.append(corners)
    F = []
    for corners in tets:
        cols = []
        for c in corners:
            cols.append(np.stack([2 * (ci + c[0]), 2 * (cj + c[1]), 2 * (ck + c[2])], 1))
        if order == 2:
            for (i, j) in TET_EDGES:
                cols.append((cols[i] + cols[j]) // 2)
        F.append(np.stack([hid(x[:, 0], x[:, 1], x[:, 2]) for x in cols], 1))
    F = np.concatenate(F)
    # keep only the nodes that are used, in half-grid lexicographic order
    used = np.unique(F)
    remap = -np.ones(m ** 3, dtype=np.int64)
    remap[used] = np.arange(len(used))
    F = remap[F]
    I = used % m
    J = (used // m) % m
    K = used // (m * m)
    half = np.stack([I, J, K], 1)
    V = half.astype(np.float64) / (2 * n)
    return V, F, half


def kuhn_jitter(V, half, n, amp, rng):
    """Move every interior cell vertex by U[-amp, amp]^3; every other
    half-grid node is put at the midpoint of its (now moved) Kuhn edge, so
    that all elements stay affine.  Boundary vertices do not move."""
    V = V.copy()
    m = 2 * n + 1
    even = np.all(half % 2 == 0, axis=1)
    interior = np.all((half > 0) & (half < 2 * n), axis=1)
    vid = -np.ones(m ** 3, dtype=np.int64)
    hkey = half[:, 0] + m * (half[:, 1] + m * half[:, 2])
    vid[hkey] = np.arange(len(V))
    mv = even & interior
    V[mv] += rng.uniform(-amp, amp, size=(int(mv.sum()), 3))
    odd = ~even
    h = half[odd]
    lo = np.where(h % 2 == 1, h - 1, h)
    hi = np.where(h % 2 == 1, h + 1, h)
    a = vid[lo[:, 0] + m * (lo[:, 1] + m * lo[:, 2])]
    b = vid[hi[:, 0] + m * (hi[:, 1] + m * hi[:, 2])]
    V[odd] = 0.5 * (V[a] + V[b])
    return V
