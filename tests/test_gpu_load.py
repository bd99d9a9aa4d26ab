"""GPU load vector against the oracle: b_j = sum_E sum_q w mu f_h phi_j.

Tolerance: |b - b_ref| <= 1e-12 max|b_ref| (sums of O(10) positive-weight
terms per node, different but equivalent rounding order)."""

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


def check(got, ref, what):
    err = np.abs(got - ref).max() if ref.size else 0.0
    assert err <= 1e-12 * max(np.abs(ref).max() if ref.size else 0.0, 1e-300), (what, err)


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_small_all_types(lf, t):
    m = meshgen.small_mesh(*t, size=3)
    print("case", t, flush=True)
    dm = lf.DeviceMesh.from_dict(m)
    f = np.random.default_rng(11).uniform(0.5, 2.0, size=dm.N)
    b1 = dm.load().cpu().numpy()
    bf = dm.load(torch.as_tensor(f, device="cuda")).cpu().numpy()
    check(b1, oracle.load(m), f"{t} f=1")
    check(bf, oracle.load(m, f), f"{t} f")
    dm.close()


def test_config2_full_and_determinism(lf):
    m = meshgen.config2()
    print("case c2 load", flush=True)
    dm = lf.DeviceMesh.from_dict(m)
    f = torch.as_tensor(m["coef_c"], device="cuda")
    b = dm.load(f)
    again = dm.load(f)
    torch.cuda.synchronize()
    assert torch.equal(b, again)
    check(b.cpu().numpy(), oracle.load(m, m["coef_c"]), "c2")
    dm.close()


def test_empty_mesh(lf):
    m = meshgen.small_mesh("surface", 2, 2, size=2)
    m = dict(m)
    m["conn"] = np.zeros((6, 0), dtype=np.int32)
    dm = lf.DeviceMesh.from_dict(m)
    b = dm.load()
    torch.cuda.synchronize()
    assert torch.count_nonzero(b).item() == 0
    dm.close()
