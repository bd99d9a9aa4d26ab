"""Per-step system of Dziuk's mean-curvature-flow scheme (section 6.3):
S = M + tau A and rhs = M x at the current coordinates.

* parity: S against the oracle's M + tau A (same CSR pattern; 1e-12
  row-scaled), rhs against the oracle's M times x (1e-12 of sum_j |M_ij x_j|);
* a HIP-graph capture of the step replayed while the coordinates move in
  place gives bitwise the eager results, replay after replay;
* the scheme run with a host solve shrinks the unit sphere like the exact
  flow, r(t)^2 = 1 - 4t."""

import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import assert_csr_close
from meshgen import meshes as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_system_matches_oracle(lf, t):
    m = meshgen.small_mesh(*t, size=3)
    say("case", t)
    dm = lf.DeviceMesh.from_dict(m)
    n, N = m["coords"].shape
    tau = 0.0123
    x = np.random.default_rng(3).normal(size=(n, N))
    out = dm.dziuk_system(tau, torch.as_tensor(x, device="cuda"))
    own = dm.dziuk_system(tau)  # x = the mesh's coordinates
    rp, ci = (v.cpu().numpy() for v in dm.pattern_tensors())
    Mo, Ao = oracle.assemble(m, "mass"), oracle.assemble(m, "stiffness")
    So = (Mo[0], Mo[1], Mo[2] + tau * Ao[2])
    assert_csr_close(rp, ci, out["S"].cpu().numpy(), So, what=f"{t} S")
    M = oracle.to_scipy(N, Mo)
    absM = abs(M)
    for got, xx in ((out["rhs"], x), (own["rhs"], m["coords"])):
        got = got.cpu().numpy()
        for c in range(n):
            ref = M @ xx[c]
            scale = absM @ np.abs(xx[c])
            assert np.all(np.abs(got[c] - ref) <= 1e-12 * np.maximum(scale, 1e-300)), (t, c)
    dm.close()


def test_graph_replay_moving_mesh(lf):
    V, F = mg.icosphere_red(3, order=2)
    coords, conn = mg.to_soa(V, F)
    m = dict(domain="surface", dim=2, order=2, quad=6, coords=coords, conn=conn)
    dm = lf.DeviceMesh.from_dict(m)
    tau = 1e-3
    static = dm.dziuk_system(tau)  # eager call: builds every lazy structure
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dm.dziuk_system(tau, out=static)
    rng = np.random.default_rng(4)
    for rep in range(3):
        moved = coords * (1.0 + 0.05 * rng.uniform(-1, 1, size=coords.shape[1]))
        dm.coords.copy_(torch.as_tensor(moved))
        g.replay()
        torch.cuda.synchronize()
        eager = dm.dziuk_system(tau)
        torch.cuda.synchronize()
        for key in ("M", "A", "S", "rhs"):
            assert torch.equal(static[key], eager[key]), (rep, key)
        # and the replayed system is that of the moved mesh
        Mo = oracle.assemble(dict(m, coords=moved), "mass")
        rp, ci = (v.cpu().numpy() for v in dm.pattern_tensors())
        assert_csr_close(rp, ci, static["M"].cpu().numpy(), Mo, what=f"replay {rep} M")
    dm.close()


def test_mean_curvature_flow_shrinks_sphere(lf):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    V, F = mg.icosphere_red(3, order=2)
    coords, conn = mg.to_soa(V, F)
    m = dict(domain="surface", dim=2, order=2, quad=6, coords=coords, conn=conn)
    dm = lf.DeviceMesh.from_dict(m)
    rp, ci = (v.cpu().numpy() for v in dm.pattern_tensors())
    N = dm.N
    tau, steps = 1e-3, 25
    for _ in range(steps):
        out = dm.dziuk_system(tau)
        S = sp.csr_matrix((out["S"].cpu().numpy(), ci, rp), shape=(N, N)).tocsc()
        rhs = out["rhs"].cpu().numpy()
        lu = spla.splu(S)
        x_new = np.stack([lu.solve(rhs[c]) for c in range(3)])
        dm.coords.copy_(torch.as_tensor(x_new))
    r = np.linalg.norm(dm.coords.cpu().numpy(), axis=0)
    exact = np.sqrt(1.0 - 4.0 * tau * steps)
    say("radius", r.mean(), r.min(), r.max(), "exact", exact)
    assert abs(r.mean() - exact) < 3e-3
    assert r.max() - r.min() < 1e-2  # stays round
    dm.close()


def test_empty_mesh_and_bad_tau(lf):
    m = dict(meshgen.small_mesh("surface", 2, 2, size=2))
    m["conn"] = np.zeros((6, 0), dtype=np.int32)
    dm = lf.DeviceMesh.from_dict(m)
    out = dm.dziuk_system(0.01)
    torch.cuda.synchronize()
    assert bool((out["rhs"] == 0).all())
    with pytest.raises(lf.LfemError) as e:
        dm.dziuk_system(float("nan"))
    assert e.value.status == lf.LFEM_EINVAL
    dm.close()
