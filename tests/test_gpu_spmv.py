"""lfem_spmv (products of assembled matrices with nodal vectors) and the
torch.sparse_csr_tensor view of an assembled matrix, against the oracle's
matrices."""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import meshgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def csr(ref, n):
    rp, ci, va = ref
    return sp.csr_matrix((va, ci, rp), shape=(n, n))


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
@pytest.mark.parametrize("nvec", [1, 3, 6])
def test_spmv_vs_oracle(lf, t, nvec):
    m = meshgen.small_mesh(*t, size=3)
    N = m["coords"].shape[1]
    dm = lf.DeviceMesh.from_dict(m)
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A)
    x = np.random.default_rng(7).normal(size=(nvec, N))
    xd = torch.as_tensor(x, device="cuda")
    for key, kind in (("M", "mass"), ("A", "stiffness")):
        y = dm.matvec(out[key], xd if nvec > 1 else xd[0], alpha=-0.75).cpu().numpy().reshape(nvec, N)
        V = csr(oracle.assemble(m, kind), N)
        ref = -0.75 * (V @ x.T).T
        # rounding bound of each row's sum: a few ulps of sum_j |V_ij x_j|
        bound = 1e-13 * np.abs(0.75 * (abs(V) @ np.abs(x).T).T) + 1e-300
        assert np.all(np.abs(y - ref) <= bound), (t, key)
    # deterministic: the same bits twice
    y1 = dm.matvec(out["A"], xd)
    y2 = dm.matvec(out["A"], xd)
    assert torch.equal(y1, y2)
    dm.close()


def test_sparse_csr_tensor(lf):
    m = meshgen.small_mesh("surface", 2, 2, size=3)
    N = m["coords"].shape[1]
    dm = lf.DeviceMesh.from_dict(m)
    c = torch.as_tensor(m["coef_c"], device="cuda")
    for kind, coef, okind, ocoef in (("mass", None, "mass", None), ("stiffness", None, "stiffness", None),
                                     ("weighted", c, "mass", m["coef_c"])):
        S = lf.assemble(dm, kind, coef)
        assert S.layout == torch.sparse_csr and S.shape == (N, N) and S.dtype == torch.float64
        rp, ci, va = oracle.assemble(m, okind, coef=ocoef)
        assert np.array_equal(S.crow_indices().cpu().numpy(), rp)
        assert np.array_equal(S.col_indices().cpu().numpy(), ci)
        sc = np.repeat(np.maximum.reduceat(np.abs(va), rp[:-1]), np.diff(rp))
        assert np.all(np.abs(S.values().cpu().numpy() - va) <= 1e-12 * sc), kind
    # the two matrices share the index tensors of the pattern
    S1, S2 = lf.assemble(dm, "mass"), lf.assemble(dm, "stiffness")
    assert S1.crow_indices().data_ptr() == S2.crow_indices().data_ptr()
    with pytest.raises(ValueError):
        lf.assemble(dm, "weighted")
    dm.close()


def test_spmv_errors(lf):
    m = meshgen.small_mesh("surface", 1, 1, size=2)
    dm = lf.DeviceMesh.from_dict(m)
    out = dm.assemble(lf.LFEM_M)
    x = torch.ones(dm.N, dtype=torch.float64, device="cuda")
    with pytest.raises(lf.LfemError) as ei:
        lf.lfem_spmv(dm.pattern, out["M"], x, 1.0, x, 1)
    assert ei.value.status == lf.LFEM_EINVAL
    with pytest.raises(lf.LfemError):
        lf.lfem_spmv(dm.pattern, out["M"], x, 1.0, torch.empty_like(x), 0)
    dm.close()
