"""The autotuner's result cache, its atomic candidate and the manual schedule
knob, through the C ABI: every choice still assembles matrices equal to the
oracle's (and, for the deterministic scatters, bitwise equal to an explicit
request of the chosen variant)."""

import os

import pytest
import torch

import oracle
from gpu_util import assert_csr_close, order_mesh
from meshgen import meshes as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def sphere(lf, freq, scale):
    V, F = mg.sphere_geodesic(freq, order=2)
    V, F, _ = mg.sfc_reorder(V, F)
    coords, conn = mg.to_soa(V * scale, F)
    m = dict(domain="surface", dim=2, order=2, quad=6, coords=coords, conn=conn)
    d = lf.DeviceMesh.from_dict(m)
    d.build_pattern()
    return m, d


def check(lf, m, d, what=None):
    out = d.assemble(lf.LFEM_M | lf.LFEM_A)
    rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
    for key, kind in (("M", "mass"), ("A", "stiffness")):
        assert_csr_close(rp, ci, out[key].cpu().numpy(), oracle.assemble(m, kind), what=f"{what} {key}")
    return out


def tune(lf, d, flags, capfd):
    os.environ["LFEM_TUNE_VERBOSE"] = "1"
    try:
        capfd.readouterr()
        v, cap = lf.lfem_pattern_autotune_ex(d.handle, d.pattern, lf.LFEM_M | lf.LFEM_A, flags)
        torch.cuda.synchronize()
        err = capfd.readouterr().err
    finally:
        del os.environ["LFEM_TUNE_VERBOSE"]
    return v, cap, err


def test_cache_hit_and_refresh(lf, capfd):
    lf.lfem_tune_cache_clear()
    m1, d1 = sphere(lf, 12, 1.0)
    m2, d2 = sphere(lf, 12, 1.7)  # same element type, rule and size bucket
    v1, cap1, err1 = tune(lf, d1, 0, capfd)
    assert "[lfem tune]" in err1  # timed
    assert "atomic" not in err1
    v2, cap2, err2 = tune(lf, d2, 0, capfd)
    assert "[lfem tune]" not in err2  # applied from the cache
    assert (v1, cap1) == (v2, cap2)
    info = lf.lfem_pattern_info(d2.pattern)
    assert info["scatter"] == v2
    if v2 == lf.LFEM_SCATTER_BLOCKED:
        assert info["block_cap"] == cap2
    else:
        assert cap2 == 0
    out = check(lf, m2, d2, "cached choice")
    explicit = d2.assemble(lf.LFEM_M | lf.LFEM_A, scatter=v2)
    assert torch.equal(out["M"], explicit["M"]) and torch.equal(out["A"], explicit["A"])
    # LFEM_TUNE_NO_CACHE times again
    _, _, err3 = tune(lf, d2, lf.LFEM_TUNE_NO_CACHE, capfd)
    assert "[lfem tune]" in err3
    # a different size bucket is not a hit
    m3, d3 = sphere(lf, 25, 1.0)
    _, _, err4 = tune(lf, d3, 0, capfd)
    assert "[lfem tune]" in err4
    # after clearing, the first mesh is timed again
    lf.lfem_tune_cache_clear()
    _, _, err5 = tune(lf, d1, 0, capfd)
    assert "[lfem tune]" in err5
    for d in (d1, d2, d3):
        d.close()


def test_atomic_candidate(lf, capfd):
    m, d = sphere(lf, 12, 1.0)
    v, cap, err = tune(lf, d, lf.LFEM_TUNE_ALLOW_ATOMIC | lf.LFEM_TUNE_NO_CACHE, capfd)
    assert "[lfem tune] atomic" in err
    assert v in (lf.LFEM_SCATTER_BLOCKED, lf.LFEM_SCATTER_STAGED, lf.LFEM_SCATTER_ATOMIC)
    assert lf.lfem_pattern_info(d.pattern)["scatter"] == v
    check(lf, m, d, "atomic allowed")
    d.close()


def test_schedule_knob(lf):
    m, d = sphere(lf, 12, 1.0)
    info = lf.lfem_pattern_info(d.pattern)
    ref = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    ref_s = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_STAGED)
    for cap in (1024, 2048, 8192):
        lf.lfem_pattern_schedule(d.handle, d.pattern, lf.LFEM_SCATTER_BLOCKED, cap)
        got = lf.lfem_pattern_info(d.pattern)
        assert got["scatter"] == lf.LFEM_SCATTER_BLOCKED and got["block_cap"] == cap
        assert got["max_block_elems"] > 0
        out = check(lf, m, d, f"block capacity {cap}")
        # the block capacity changes which workgroup sums a value, not its order
        assert torch.equal(out["M"], ref["M"]) and torch.equal(out["A"], ref["A"]), cap
    lf.lfem_pattern_schedule(d.handle, d.pattern, lf.LFEM_SCATTER_STAGED, 0)
    assert lf.lfem_pattern_info(d.pattern)["scatter"] == lf.LFEM_SCATTER_STAGED
    out = d.assemble(lf.LFEM_M | lf.LFEM_A)
    assert torch.equal(out["M"], ref_s["M"]) and torch.equal(out["A"], ref_s["A"])
    lf.lfem_pattern_schedule(d.handle, d.pattern, lf.LFEM_SCATTER_ATOMIC, 0)
    check(lf, m, d, "atomic by knob")
    for bad in (info["max_row"] - 1, 20481):
        with pytest.raises(lf.LfemError) as e:
            lf.lfem_pattern_schedule(d.handle, d.pattern, lf.LFEM_SCATTER_BLOCKED, bad)
        assert e.value.status == lf.LFEM_EINVAL
    with pytest.raises(lf.LfemError) as e:
        lf.lfem_pattern_schedule(d.handle, d.pattern, 7, 0)
    assert e.value.status == lf.LFEM_EINVAL
    d.close()
    # orders 3 and 4 have no block schedule
    mt = order_mesh("bulk", 3, 3)
    dt = lf.DeviceMesh.from_dict(mt)
    dt.build_pattern()
    with pytest.raises(lf.LfemError) as e:
        lf.lfem_pattern_schedule(dt.handle, dt.pattern, lf.LFEM_SCATTER_BLOCKED, 0)
    assert e.value.status == lf.LFEM_EUNSUPPORTED
    v, cap = lf.lfem_pattern_autotune_ex(dt.handle, dt.pattern, lf.LFEM_M | lf.LFEM_A, lf.LFEM_TUNE_NO_CACHE)
    assert v == lf.LFEM_SCATTER_STAGED and cap == 0
    dt.close()


@pytest.mark.parametrize("order", [1, 2])
def test_tetrahedra_default_scatter(lf, order):
    """P2 tetrahedra default to the staged scatter and get no block schedule
    at pattern build (the first blocked request builds one, colour mode); P1
    tetrahedra keep the colour-blocked default.  Every variant matches the
    oracle, and the default equals its variant bit for bit."""
    import meshgen
    m = meshgen.small_mesh("bulk", 3, order, size=3)
    d = lf.DeviceMesh.from_dict(m)
    d.build_pattern()
    info = lf.lfem_pattern_info(d.pattern)
    default = lf.LFEM_SCATTER_STAGED if order == 2 else lf.LFEM_SCATTER_BLOCKED
    assert info["scatter"] == default
    assert (info["blocks"] == 0) == (order == 2)
    auto = d.assemble(lf.LFEM_M | lf.LFEM_A)
    same = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=default)
    assert torch.equal(auto["M"], same["M"]) and torch.equal(auto["A"], same["A"])
    check(lf, m, d, f"P{order} tetrahedra default")
    rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
    for variant in (lf.LFEM_SCATTER_BLOCKED, lf.LFEM_SCATTER_STAGED):
        out = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=variant)
        for key, kind in (("M", "mass"), ("A", "stiffness")):
            assert_csr_close(rp, ci, out[key].cpu().numpy(), oracle.assemble(m, kind), what=f"{variant} {key}")
    info = lf.lfem_pattern_info(d.pattern)
    assert info["blocks"] > 0 and info["max_colors"] > 1  # built by the blocked request
    assert info["scatter"] == default  # the default is unchanged
    d.close()
