"""lfem_shape_grad_noalloc (the shape gradient with its staging in the
library's fixed workspace) against lfem_shape_grad, through the C ABI: two
calls in a row on the same GPU, the second on a smaller mesh (the workspace
keeps the first call's contents), plus the size limit."""

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
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def grads(lf, m):
    """(lfem_shape_grad, lfem_shape_grad_noalloc) of alpha u^T A v + beta w^T M z."""
    dm = lf.DeviceMesh.from_dict(m)
    u, v, w, z = (cuda(m[k]) for k in ("u", "v", "coef_c", "coef_a"))
    ref = torch.full_like(dm.coords, float("nan"))
    got = torch.full_like(dm.coords, float("nan"))
    lf.lfem_shape_grad(dm.handle, u, v, 0.7, w, z, -1.2, ref)
    lf.lfem_shape_grad_noalloc(dm.handle, u, v, 0.7, w, z, -1.2, got)
    torch.cuda.synchronize()
    out = ref.cpu().numpy(), got.cpu().numpy()
    dm.close()
    return out


def large_mesh():
    """P2 sphere of 163,840 curved triangles (2.95 M staged doubles, 70 % of
    the workspace) with nodal fields."""
    m = meshgen.config5()
    rng = np.random.default_rng(20260077)
    N = m["coords"].shape[1]
    m["coef_c"] = rng.uniform(0.5, 2.0, N)
    m["coef_a"] = rng.normal(size=N)
    return m


def test_noalloc_two_calls_second_smaller(lf):
    print("noalloc: P2 sphere 163840 triangles, then small P2 surface", flush=True)
    big = large_mesh()
    ref, got = grads(lf, big)
    assert np.array_equal(ref, got)  # same kernels, same order: the same bits
    small = meshgen.small_mesh("surface", 2, 2, size=3)
    ref2, got2 = grads(lf, small)
    assert np.array_equal(ref2, got2)
    # and the bar against the oracle on the small mesh
    o = oracle.shape_grad(small, small["u"], small["v"], 0.7, small["coef_c"], small["coef_a"], -1.2)
    assert np.linalg.norm(got2 - o) <= 1e-12 * np.linalg.norm(o)


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_noalloc_every_type(lf, t):
    m = meshgen.small_mesh(*t, size=3)
    ref, got = grads(lf, m)
    assert np.array_equal(ref, got), t


def test_noalloc_size_limit(lf):
    """More than 4,194,304 staged doubles: LFEM_ERANGE from the host check,
    before any launch; the entry point still works afterwards."""
    from meshgen import meshes as mg
    V, F = mg.sphere_nvb(14, order=2)  # 327,680 P2 triangles: 5.9 M staged doubles
    coords, conn = mg.to_soa(V, F)
    dm = lf.DeviceMesh.from_dict(dict(domain="surface", dim=2, order=2, quad=6, coords=coords, conn=conn))
    u = torch.ones(dm.N, dtype=torch.float64, device="cuda")
    g = torch.empty_like(dm.coords)
    with pytest.raises(lf.LfemError) as ei:
        lf.lfem_shape_grad_noalloc(dm.handle, u, u, 1.0, None, None, 0.0, g)
    assert ei.value.status == lf.LFEM_ERANGE
    dm.close()
    small = meshgen.small_mesh("bulk", 3, 2, size=2)
    ref, got = grads(lf, small)
    assert np.array_equal(ref, got)
