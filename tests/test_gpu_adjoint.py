"""GPU shape adjoint: lfem_shape_grad / lfem_energy against the oracle's closed
form and against central finite differences; the autograd Function."""

import numpy as np
import pytest
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


def cuda(x):
    return None if x is None else torch.as_tensor(np.ascontiguousarray(x), device="cuda")


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_small_vs_oracle(lf, t):
    m = meshgen.small_mesh(*t, size=3)
    dm = lf.DeviceMesh.from_dict(m)
    u, v, w, z = (cuda(m[k]) for k in ("u", "v", "coef_c", "coef_a"))
    g = torch.empty_like(dm.coords)
    lf.lfem_shape_grad(dm.handle, u, v, 0.7, w, z, -1.2, g)
    ref = oracle.shape_grad(m, m["u"], m["v"], 0.7, m["coef_c"], m["coef_a"], -1.2)
    err = np.linalg.norm(g.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-12
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    lf.lfem_energy(dm.handle, u, v, 0.7, w, z, -1.2, J)
    Jref = oracle.energy(m, m["u"], m["v"], 0.7, m["coef_c"], m["coef_a"], -1.2)
    assert abs(J.item() - Jref) <= 1e-12 * abs(Jref)
    # one term only (w, z null)
    lf.lfem_shape_grad(dm.handle, u, v, 1.0, None, None, 0.0, g)
    ref = oracle.shape_grad(m, m["u"], m["v"], 1.0, None, None, 0.0)
    assert np.linalg.norm(g.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    dm.close()


def patch(m, node):
    """The elements containing `node` as a stand-alone mesh (same node ids)."""
    sel = np.any(m["conn"] == node, axis=0)
    p = dict(m)
    p["conn"] = np.ascontiguousarray(m["conn"][:, sel])
    return p


def test_config5_adjoint(lf):
    m = meshgen.config5()
    print("config5", m["conn"].shape, flush=True)
    dm = lf.DeviceMesh.from_dict(m)
    u, v = cuda(m["u"]), cuda(m["v"])
    g = torch.empty_like(dm.coords)
    lf.lfem_shape_grad(dm.handle, u, u, 1.0, v, v, 1.0, g)
    g2 = torch.empty_like(dm.coords)
    lf.lfem_shape_grad(dm.handle, u, u, 1.0, v, v, 1.0, g2)
    assert torch.equal(g, g2)  # deterministic gather
    G = g.cpu().numpy()
    ref = oracle.shape_grad(m, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0)
    assert np.linalg.norm(G - ref) <= 1e-12 * np.linalg.norm(ref)
    # 200 seeded coordinates against central differences of the local patch energy
    # (elements containing the node), evaluated in long double.  The h = 1e-6
    # difference is Richardson-extrapolated with the h = 2e-6 one to remove its
    # O(h^2) truncation term, which reaches ~1e-6 relative on the steepest patches.
    rng = np.random.default_rng(20260005)
    N = m["coords"].shape[1]
    gmax = np.abs(G).max()

    def central(p, r, c, h):
        Xp = p["coords"].copy()
        Xp[c, r] += h
        Xm = p["coords"].copy()
        Xm[c, r] -= h
        pp, pm = dict(p), dict(p)
        pp["coords"], pm["coords"] = Xp, Xm
        return (oracle.energy(pp, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0, long_double=True)
                - oracle.energy(pm, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0,
                                long_double=True)) / (2 * h)

    # Metrics: (1) floored relative error |G - fd| / max(|fd|, 1e-3 max|G|)
    # over all 200 samples (a component near zero has no meaningful relative
    # error); (2) plain relative error |G - fd| / |fd| over the samples with
    # |fd| >= 1e-2 max|G|.  Each for the extrapolated and the plain h = 1e-6
    # central difference.
    worst = worst_plain = 0.0
    rel = rel_plain = 0.0
    n_large = 0
    for _ in range(200):
        r = int(rng.integers(N))
        c = int(rng.integers(3))
        p = patch(m, r)
        f1 = central(p, r, c, 1e-6)
        f2 = central(p, r, c, 2e-6)
        fd = (4.0 * f1 - f2) / 3.0
        scale = max(abs(fd), 1e-3 * gmax)
        worst = max(worst, abs(G[c, r] - fd) / scale)
        worst_plain = max(worst_plain, abs(G[c, r] - f1) / scale)
        if abs(fd) >= 1e-2 * gmax:
            n_large += 1
            rel = max(rel, abs(G[c, r] - fd) / abs(fd))
            rel_plain = max(rel_plain, abs(G[c, r] - f1) / abs(f1))
    print(f"adjoint vs FD (floored): extrapolated {worst:.3e}, plain h=1e-6 {worst_plain:.3e}; "
          f"unfloored over {n_large} samples with |fd| >= 1e-2 max|G|: extrapolated {rel:.3e}, "
          f"plain h=1e-6 {rel_plain:.3e}", flush=True)
    assert n_large >= 100, n_large
    assert worst <= 1e-6, worst
    assert rel <= 1e-6, rel
    assert worst_plain <= 1e-5, worst_plain
    assert rel_plain <= 1e-5, rel_plain
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    lf.lfem_energy(dm.handle, u, u, 1.0, v, v, 1.0, J)
    Jref = oracle.energy(m, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0)
    assert abs(J.item() - Jref) <= 1e-12 * abs(Jref)
    dm.close()


def test_autograd_function(lf):
    m = meshgen.small_mesh("surface", 2, 2, size=3)
    dm = lf.DeviceMesh.from_dict(m)
    u, v = cuda(m["u"]), cuda(m["v"])
    x = dm.coords.clone().requires_grad_(True)
    J = lf.ShapeEnergy.apply(x, dm, u, u, v, v, 1.0, 1.0)
    (gx,) = torch.autograd.grad(3.0 * J, x)
    ref = oracle.shape_grad(m, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0)
    assert np.linalg.norm(gx.cpu().numpy() - 3.0 * ref) <= 1e-12 * np.linalg.norm(3.0 * ref)
    Jref = oracle.energy(m, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0)
    assert abs(J.item() - Jref) <= 1e-12 * abs(Jref)
    # a moved mesh: the Function reads the coordinates it is given
    x2 = (dm.coords * 1.1).clone().requires_grad_(True)
    J2 = lf.ShapeEnergy.apply(x2, dm, u, u, v, v, 1.0, 1.0)
    m2 = dict(m)
    m2["coords"] = m["coords"] * 1.1
    assert abs(J2.item() - oracle.energy(m2, m["u"], m["u"], 1.0, m["v"], m["v"], 1.0)) \
        <= 1e-12 * abs(J2.item())
    dm.close()


def test_autograd_nodal_vectors_and_restore(lf):
    """Gradients with respect to u, v, w, z (alpha A v, alpha A u, beta M z,
    beta M w) against the oracle's matrices, and the mesh's own coordinates
    restored after forward and backward."""
    import scipy.sparse as sp
    m = meshgen.small_mesh("surface", 2, 2, size=3)
    N = m["coords"].shape[1]
    dm = lf.DeviceMesh.from_dict(m)
    own = dm.coords
    u, v, w, z = (cuda(m[k]).requires_grad_(True) for k in ("u", "v", "coef_c", "coef_a"))
    x = (dm.coords * 1.05).clone().requires_grad_(True)
    J = lf.ShapeEnergy.apply(x, dm, u, v, w, z, 0.7, -1.2)
    assert dm.coords is own
    gx, gu, gv, gw, gz = torch.autograd.grad(2.0 * J, (x, u, v, w, z))
    assert dm.coords is own
    mx = dict(m)
    mx["coords"] = m["coords"] * 1.05
    rp, ci, va = oracle.assemble(mx, "stiffness")
    A = sp.csr_matrix((va, ci, rp), shape=(N, N))
    rp, ci, va = oracle.assemble(mx, "mass")
    M = sp.csr_matrix((va, ci, rp), shape=(N, N))
    for got, ref in ((gu, 2 * 0.7 * (A @ m["v"])), (gv, 2 * 0.7 * (A @ m["u"])),
                     (gw, 2 * -1.2 * (M @ m["coef_a"])), (gz, 2 * -1.2 * (M @ m["coef_c"]))):
        assert np.linalg.norm(got.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    gref = oracle.shape_grad(mx, m["u"], m["v"], 0.7, m["coef_c"], m["coef_a"], -1.2)
    assert np.linalg.norm(gx.cpu().numpy() - 2 * gref) <= 1e-12 * np.linalg.norm(2 * gref)
    # the handle reads the mesh's own coordinates again
    rp, ci = (t.cpu().numpy() for t in dm.pattern_tensors())
    got = dm.assemble(lf.LFEM_M)["M"].cpu().numpy()
    from gpu_util import assert_csr_close
    assert_csr_close(rp, ci, got, oracle.assemble(m, "mass"), what="mass after ShapeEnergy")
    dm.close()

