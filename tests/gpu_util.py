"""Helpers shared by the GPU tests (comparison against the oracle, small
curved meshes of orders 1 to 4)."""

import numpy as np

import oracle
from meshgen import meshes as mg

# Row-scaled relative tolerance on every stored value:
# |v_gpu - v_ref| <= TOL * max_k |ref_ik| over the row.  Entrywise relative
# error is ill-posed for entries that vanish by cancellation (for example the
# exact zeros of the affine P2 mass matrix), so the row maximum is the scale.
TOL = 1e-12


def row_scale(rp, vals):
    n = len(rp) - 1
    scale = np.zeros(n)
    nz = np.diff(rp) > 0
    scale[nz] = np.maximum.reduceat(np.abs(vals), rp[:-1][nz])
    return scale


def assert_csr_close(rp, ci, got, ref_csr, tol=TOL, what=""):
    orp, oci, ova = ref_csr
    assert np.array_equal(np.asarray(rp, dtype=np.int64), orp), f"{what}: row_ptr differs"
    assert np.array_equal(np.asarray(ci, dtype=np.int64), oci.astype(np.int64)), \
        f"{what}: col_idx differs"
    sc = np.repeat(row_scale(orp, ova), np.diff(orp))
    err = np.abs(np.asarray(got) - ova) / np.where(sc > 0, sc, 1.0)
    worst = float(err.max()) if len(err) else 0.0
    assert worst <= tol, f"{what}: row-scaled error {worst:.3e} > {tol}"
    return worst


def assert_rows_close(rp, ci, got, ref_rows_csr, rows, tol=TOL, what=""):
    """Compare selected rows only (oracle assembled with a row mask)."""
    orp, oci, ova = ref_rows_csr
    worst = 0.0
    for i in rows:
        a, b = rp[i], rp[i + 1]
        oa, ob = orp[i], orp[i + 1]
        assert np.array_equal(ci[a:b], oci[oa:ob]), f"{what}: columns of row {i} differ"
        ref = ova[oa:ob]
        sc = np.abs(ref).max()
        w = float(np.abs(got[a:b] - ref).max() / sc)
        worst = max(worst, w)
    assert worst <= tol, f"{what}: row-scaled error {worst:.3e} > {tol}"
    return worst



def grad_abs_scale(oracle, m, *args):
    """Per node r the sum, over the elements containing r, of the largest
    entry of that element's own shape-gradient contribution (each computed by
    the oracle on the one-element mesh), broadcast over the components: the
    scale of the rounding error of the summed gradient,
    |fl(sum_e g_e) - sum_e g_e| <= c eps sum_e |g_e|.  Gradient entries cancel
    between elements (interior nodes of flat meshes nearly balance), so the
    largest entry of the whole gradient is not the right scale for them; the
    element's largest entry (like the row maximum of a matrix) is."""
    n, N = m["coords"].shape
    S = np.zeros(N)
    T = m["conn"].shape[1]
    for e in range(T):
        one = dict(m)
        one["conn"] = np.ascontiguousarray(m["conn"][:, e:e + 1])
        S[m["conn"][:, e]] += np.abs(oracle.shape_grad(one, *args)).max()
    return np.broadcast_to(S, (n, N))


def order_mesh(domain, d, p, seed=0):
    """A small curved mesh of order p with random nodal coefficients."""
    rng = np.random.default_rng(100 + 10 * d + p + seed)
    if domain == "surface" and d == 1:
        V, F = mg.circle(11)
        V, F = mg.p1_to_pp(V, F, p, mg.SEG_EDGES)
        V = mg.normalize_rows(V) * (1.0 + 0.05 * rng.uniform(-1, 1, size=len(V)))[:, None]
        quad = 5 if p == 3 else 6
    elif domain == "surface" and d == 2:
        V, F = mg.icosphere_red(1)
        V, F = mg.p1_to_pp(V, F, p, mg.TRI_EDGES)
        V = mg.normalize_rows(V) * (1.0 + 0.05 * rng.uniform(-1, 1, size=len(V)))[:, None]
        quad = 16
    elif domain == "bulk" and d == 3:
        V, F, _ = mg.kuhn_cube(2, order=1)
        V, F = mg.p1_to_pp(V, F, p, mg.TET_EDGES)
        # every non-vertex node inside the cube moved by a twentieth of the node
        # spacing h / p (h = 1/2; a tenth folds Kuhn quartics): curved elements
        inter = np.all((V > 1e-12) & (V < 1 - 1e-12), axis=1)
        amp = 0.05 / (2 * p)
        V[inter] += rng.uniform(-amp, amp, size=(int(inter.sum()), 3))
        quad = 35
    else:
        V, F = mg.square_tri(3)
        V, F = mg.p1_to_pp(V, F, p, mg.TRI_EDGES)
        inter = np.all((V > 1e-12) & (V < 1 - 1e-12), axis=1)
        # a tenth of the node spacing h / p (h = 1/3): larger moves fold
        # quartic elements (det J changing sign inside one element)
        amp = 0.1 / (3 * p)
        V[inter] += rng.uniform(-amp, amp, size=(int(inter.sum()), 2))
        quad = 16
    coords, conn = mg.to_soa(V, F)
    if domain == "bulk":
        # every element valid: det J of one sign at points spread over the element
        if d == 2:
            xi = np.array([(i / 8, j / 8) for i in range(9) for j in range(9 - i)])
        else:
            xi = np.array([(i / 6, j / 6, l / 6) for i in range(7) for j in range(7 - i) for l in range(7 - i - j)])
        for e in range(conn.shape[1]):
            x = coords[:, conn[:, e]]
            dets = [np.linalg.det(x @ oracle.basis(d, p, pt)[1]) for pt in xi]
            assert min(dets) > 0 or max(dets) < 0, f"folded element {e}"
    N = coords.shape[1]
    return dict(domain=domain, dim=d, order=p, quad=quad, coords=coords, conn=conn,
                coef_a=rng.uniform(0.5, 2.0, size=N), coef_c=rng.uniform(0.5, 2.0, size=N))


# meshes with one node of very high valence (rows longer than 255 entries)
FAN_QUAD = {1: 3, 2: 6, 3: 16, 4: 16}


def raise_order(V, F, p, edges):
    if p == 1:
        return V, F
    if p == 2:
        V2, F2, _ = mg.p1_to_p2(V, F, edges)
        return V2, F2
    return mg.p1_to_pp(V, F, p, edges)


def fan(n, p, surface, seed=0):
    """A disk around one centre vertex shared by n triangles (two rings of n
    vertices at radii near 1 and 2), raised to order p; on a surface the
    points are lifted onto a cone.  The centre's row holds 1 + n (p = 1),
    1 + 3n (p = 2), 1 + 6n (p = 3) or 1 + 10n (p = 4) entries."""
    rng = np.random.default_rng(500 + 10 * n + p + seed)
    t = 2 * np.pi * np.arange(n) / n
    r1 = 1.0 + 0.05 * rng.uniform(-1, 1, n)
    r2 = 2.0 + 0.05 * rng.uniform(-1, 1, n)
    V = np.vstack([[0.0, 0.0], np.c_[r1 * np.cos(t), r1 * np.sin(t)], np.c_[r2 * np.cos(t), r2 * np.sin(t)]])
    i = np.arange(n)
    j = (i + 1) % n
    F = np.vstack([np.c_[np.zeros(n, dtype=np.int64), 1 + i, 1 + j],
                   np.c_[1 + i, 1 + n + i, 1 + j],
                   np.c_[1 + j, 1 + n + i, 1 + n + j]])
    V, F = raise_order(V, F, p, mg.TRI_EDGES)
    if surface:
        z = 0.4 * (2.0 - np.hypot(V[:, 0], V[:, 1]))
        V = np.c_[V, z]
    coords, conn = mg.to_soa(V, F)
    domain = "surface" if surface else "bulk"
    return dict(domain=domain, dim=2, order=p, quad=FAN_QUAD[p], coords=coords, conn=conn,
                coef=1.0 + 0.5 * np.sin(coords[0]) * np.cos(coords[1]))


def star(n, p):
    """P2 (or P1) tetrahedra around one centre vertex: a polygon of n rim
    vertices at z = 0 and two apices, 2n tetrahedra sharing the centre."""
    rng = np.random.default_rng(900 + n + p)
    t = 2 * np.pi * np.arange(n) / n
    r = 1.0 + 0.05 * rng.uniform(-1, 1, n)
    V = np.vstack([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0],
                   np.c_[r * np.cos(t), r * np.sin(t), 0.02 * rng.uniform(-1, 1, n)]])
    i = np.arange(n)
    j = (i + 1) % n
    F = np.vstack([np.c_[np.zeros(n, dtype=np.int64), np.ones(n, dtype=np.int64), 3 + i, 3 + j],
                   np.c_[np.zeros(n, dtype=np.int64), np.full(n, 2), 3 + j, 3 + i]])
    V, F = raise_order(V, F, p, mg.TET_EDGES)
    coords, conn = mg.to_soa(V, F)
    return dict(domain="bulk", dim=3, order=p, quad=11 if p == 2 else 4, coords=coords, conn=conn,
                coef=1.0 + 0.5 * np.sin(coords[0]) * np.cos(coords[1]) * coords[2])
