"""Per-step systems of the paper's two mean-curvature-flow schemes.

Dziuk's scheme (section 6.3): S = M + tau A and rhs = M x at the current
coordinates.

* parity: S against the oracle's M + tau A (same CSR pattern; 1e-12
  row-scaled), rhs against the oracle's M times x (1e-12 of sum_j |M_ij x_j|);
* a HIP-graph capture of the step replayed while the coordinates move in
  place gives bitwise the eager results, replay after replay;
* the scheme run with a host solve shrinks the unit sphere like the exact
  flow, r(t)^2 = 1 - 4t.

The BDF algorithm of section 6.2 in u = (nu; H): S = delta0 M + tau A,
f = (f_1; f_2), rhs = tau f - M hist.
* parity of S, f and rhs with oracle.kll_system on every element type
  (rhs within 1e-12 of tau |f| + |M| |hist| entrywise), with and without
  the history term;
* a captured step replayed while the surface moves in place gives bitwise
  the eager results;
* BDF2 with host solves shrinks the unit sphere at second order in tau and
  follows the oracle's run of the same scheme to 1e-10."""

import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import assert_csr_close, assert_rows_close
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


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_kll_system_matches_oracle(lf, t):
    m = meshgen.small_mesh(*t, size=3)
    say("case", t, "kll system")
    dm = lf.DeviceMesh.from_dict(m)
    n, N = m["coords"].shape
    rng = np.random.default_rng(7)
    nu, H, hist = rng.normal(size=(n, N)), rng.normal(size=N), rng.normal(size=(n + 1, N))
    tau, d0 = 0.0123, 1.5
    dev = (torch.as_tensor(v, device="cuda") for v in (nu, H, hist))
    nut, Ht, histt = dev
    rp, ci = (v.cpu().numpy() for v in dm.pattern_tensors())
    M = oracle.to_scipy(N, oracle.assemble(m, "mass"))
    for with_hist in (True, False):
        out = dm.kll_system(tau, d0, nut, Ht, histt if with_hist else None)
        So, fo, rhso = oracle.kll_system(m, tau, d0, nu, H, hist if with_hist else None)
        assert_csr_close(rp, ci, out["S"].cpu().numpy(), So, what=f"{t} S")
        f = out["f"].cpu().numpy()
        for c in range(n + 1):
            assert np.abs(f[c] - fo[c]).max() <= 1e-12 * np.abs(fo[c]).max(), (t, c)
        got = out["rhs"].cpu().numpy()
        scale = tau * np.abs(fo) + (np.stack([abs(M) @ np.abs(hist[c]) for c in range(n + 1)]) if with_hist else 0)
        assert np.all(np.abs(got - rhso) <= 1e-12 * np.maximum(scale, 1e-300)), (t, with_hist)
    dm.close()


def test_kll_graph_replay_moving_mesh(lf):
    V, F = mg.icosphere_red(3, order=2)
    coords, conn = mg.to_soa(V, F)
    m = dict(domain="surface", dim=2, order=2, quad=6, coords=coords, conn=conn)
    dm = lf.DeviceMesh.from_dict(m)
    N = coords.shape[1]
    rng = np.random.default_rng(8)
    nu = torch.as_tensor(coords / np.linalg.norm(coords, axis=0), device="cuda")
    H = torch.full((N,), 2.0, dtype=torch.float64, device="cuda")
    hist = torch.as_tensor(rng.normal(size=(4, N)), device="cuda")
    static = dm.kll_system(1e-3, 1.5, nu, H, hist)  # eager call: builds every lazy structure
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dm.kll_system(1e-3, 1.5, nu, H, hist, out=static)
    for rep in range(3):
        moved = coords * (1.0 + 0.05 * rng.uniform(-1, 1, size=N))
        dm.coords.copy_(torch.as_tensor(moved))
        g.replay()
        torch.cuda.synchronize()
        eager = dm.kll_system(1e-3, 1.5, nu, H, hist)
        torch.cuda.synchronize()
        for key in ("M", "A", "S", "f", "rhs"):
            assert torch.equal(static[key], eager[key]), (rep, key)
    dm.close()


def test_kll_bdf2_flow_matches_oracle_run(lf):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    V, F = mg.icosphere_red(2, order=2)
    coords, conn = mg.to_soa(V, F)
    m = dict(domain="surface", dim=2, order=2, quad=6, coords=coords, conn=conn)
    dm = lf.DeviceMesh.from_dict(m)
    rp, ci = (v.cpu().numpy() for v in dm.pattern_tensors())
    N = dm.N
    tau, steps = 1e-3, 25

    def run(system):
        x = [coords.copy()]
        u = [np.vstack([coords / np.linalg.norm(coords, axis=0), 2.0 * np.ones((1, N))])]
        for n in range(steps):
            if n == 0:
                d0, xt, ut, hist, xh = 1.0, x[-1], u[-1], -u[-1], -x[-1]
            else:
                d0, xt, ut = 1.5, 2 * x[-1] - x[-2], 2 * u[-1] - u[-2]
                hist, xh = -2 * u[-1] + 0.5 * u[-2], -2 * x[-1] + 0.5 * x[-2]
            sv, rhs = system(d0, xt, ut, hist)
            lu = spla.splu(sp.csr_matrix((sv, ci, rp), shape=(N, N)).tocsc())
            un = np.stack([lu.solve(rhs[c]) for c in range(4)])
            x.append((tau * (-un[3] * un[:3]) - xh) / d0)
            u.append(un)
        return x[-1], u[-1]

    def gpu_system(d0, xt, ut, hist):
        dm.coords.copy_(torch.as_tensor(xt))
        dev = [torch.as_tensor(np.ascontiguousarray(v), device="cuda") for v in (ut[:3], ut[3], hist)]
        out = dm.kll_system(tau, d0, *dev)
        return out["S"].cpu().numpy(), out["rhs"].cpu().numpy()

    def oracle_system(d0, xt, ut, hist):
        (orp, oci, sv), _, rhs = oracle.kll_system(dict(m, coords=xt), tau, d0, ut[:3], ut[3], hist)
        assert np.array_equal(orp, rp) and np.array_equal(oci, ci)
        return sv, rhs

    xg, ug = run(gpu_system)
    xo, uo = run(oracle_system)
    r = np.linalg.norm(xg, axis=0)
    exact = np.sqrt(1.0 - 4.0 * tau * steps)
    say("radius", r.mean(), "exact", exact, "diff to oracle run", np.abs(xg - xo).max())
    assert abs(r.mean() - exact) < 5e-6
    assert np.abs(xg - xo).max() < 1e-10 and np.abs(ug - uo).max() < 1e-10
    dm.close()


def test_kll_system_bad_arguments(lf):
    m = meshgen.small_mesh("surface", 2, 2, size=2)
    dm = lf.DeviceMesh.from_dict(m)
    n, N = m["coords"].shape
    nu = torch.zeros(n, N, dtype=torch.float64, device="cuda")
    H = torch.zeros(N, dtype=torch.float64, device="cuda")
    for tau, d0 in ((float("nan"), 1.0), (1.0, float("inf"))):
        with pytest.raises(lf.LfemError) as e:
            dm.kll_system(tau, d0, nu, H)
        assert e.value.status == lf.LFEM_EINVAL
    with pytest.raises(lf.LfemError) as e:
        dm.kll_system(1e-3, 1.0, nu, None)
    assert e.value.status == lf.LFEM_EINVAL
    dm.close()


def test_kll_system_config2_sampled(lf):
    """The BDF step on the 655,360-element P2 ellipsoid with its normals as nu,
    a nodal H and a random history: f over every node, S and rhs on sampled
    rows, against the oracle."""
    m = meshgen.config2()
    say("config2 kll system")
    dm = lf.DeviceMesh.from_dict(m)
    X = m["coords"]
    n, N = X.shape
    g = X / np.array([1.0, 0.64, 0.36])[:, None]
    nu = g / np.linalg.norm(g, axis=0)
    H = m["coef_c"]
    hist = np.random.default_rng(12).normal(size=(n + 1, N))
    tau, d0 = 2e-3, 1.5
    out = dm.kll_system(tau, d0, *(torch.as_tensor(np.ascontiguousarray(v), device="cuda") for v in (nu, H, hist)))
    fo = oracle.kll(m, nu, H)
    f = out["f"].cpu().numpy()
    for c in range(n + 1):
        assert np.abs(f[c] - fo[c]).max() <= 1e-12 * np.abs(fo[c]).max(), c
    rp, ci = (v.cpu().numpy() for v in dm.pattern_tensors())
    rows = np.unique(np.random.default_rng(14).integers(0, N, 300))
    Mr = oracle.assemble(m, "mass", rows=rows)
    Ar = oracle.assemble(m, "stiffness", rows=rows)
    Sr = (Mr[0], Mr[1], d0 * Mr[2] + tau * Ar[2])
    assert_rows_close(rp, ci, out["S"].cpu().numpy(), Sr, rows, what="c2 S")
    rhs = out["rhs"].cpu().numpy()
    for i in rows:
        a, b = Mr[0][i], Mr[0][i + 1]
        cols, mv = Mr[1][a:b], Mr[2][a:b]
        for c in range(n + 1):
            ref = tau * fo[c, i] - mv @ hist[c, cols]
            scale = tau * abs(fo[c, i]) + np.abs(mv) @ np.abs(hist[c, cols])
            assert abs(rhs[c, i] - ref) <= 1e-12 * scale, (i, c)
    dm.close()
