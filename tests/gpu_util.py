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
