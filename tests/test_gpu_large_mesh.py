"""A planar P1 mesh of more than 2^25 elements: a 4100 x 4100 grid of
squares on the unit square, each split into two triangles (33,620,000
triangles, 16,818,201 nodes), interior vertices jittered.  Element counts of
this size need incidence codes of more than 25 bits for the element; the
codes are the positions a * T + e in the connectivity.  Checked on sampled
rows against the oracle (row-masked assembly), by 1^T M 1 = area, A 1 = 0
row by row, and by the load vector of f = 1 summing to the area."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_rows_close

pytestmark = pytest.mark.gpu

N_SIDE = 4100  # 2 * 4100^2 = 33,620,000 > 2^25 = 33,554,432 triangles


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def grid_mesh(n, seed=11):
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = np.arange(n + 1) * h
    X, Y = np.meshgrid(g, g, indexing="ij")  # node id i * (n + 1) + j
    X, Y = X.ravel(), Y.ravel()
    inner = (X > 0.5 * h) & (X < 1 - 0.5 * h) & (Y > 0.5 * h) & (Y < 1 - 0.5 * h)
    X = X + np.where(inner, rng.uniform(-0.2 * h, 0.2 * h, X.size), 0.0)
    Y = Y + np.where(inner, rng.uniform(-0.2 * h, 0.2 * h, Y.size), 0.0)
    i, j = np.meshgrid(np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), indexing="ij")
    v00 = (i * (n + 1) + j).ravel()
    v10, v01 = v00 + (n + 1), v00 + 1
    v11 = v10 + 1
    conn = np.empty((3, 2 * n * n), dtype=np.int32)
    conn[0, 0::2], conn[1, 0::2], conn[2, 0::2] = v00, v10, v11
    conn[0, 1::2], conn[1, 1::2], conn[2, 1::2] = v00, v11, v01
    coords = np.stack([X, Y])
    return dict(domain="bulk", dim=2, order=1, quad=3, coords=coords, conn=conn)


def test_more_than_2_25_elements(lf):
    m = grid_mesh(N_SIDE)
    T = m["conn"].shape[1]
    assert T > 2 ** 25
    print(f"grid mesh: {T} triangles, {m['coords'].shape[1]} nodes", flush=True)
    dm = lf.DeviceMesh.from_dict(m)
    dm.build_pattern()
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A)
    torch.cuda.synchronize()
    print("assembled", flush=True)
    assert abs(float(out["M"].sum().item()) - 1.0) < 1e-10
    rp_t, ci_t = dm.pattern_tensors()
    rows_t = torch.repeat_interleave(torch.arange(dm.N, device="cuda"), (rp_t[1:] - rp_t[:-1]).long())
    a1 = torch.zeros(dm.N, dtype=torch.float64, device="cuda").index_add_(0, rows_t, out["A"])
    amax = torch.zeros(dm.N, dtype=torch.float64, device="cuda").index_reduce_(0, rows_t, out["A"].abs(), "amax")
    assert float((a1.abs() / amax).max().item()) < 1e-12
    del rows_t, a1, amax
    b = dm.load()
    assert abs(float(b.sum().item()) - 1.0) < 1e-10
    rp, ci = rp_t.cpu().numpy(), ci_t.cpu().numpy()
    N = dm.N
    rows = np.unique(np.r_[np.random.default_rng(5).integers(0, N, 200), 0, N - 1, N // 2])
    for key, kind in (("M", "mass"), ("A", "stiffness")):
        ref = oracle.assemble(m, kind, rows=rows)
        assert_rows_close(rp, ci, out[key].cpu().numpy(), ref, rows, what=f"large grid {key}")
    dm.close()
