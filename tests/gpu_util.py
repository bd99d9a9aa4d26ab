"""Helpers shared by the GPU tests (comparison against the oracle)."""

import numpy as np

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
