"""Meshes with one node of very high valence, whose CSR row holds more than
255 entries: the pattern switches to two-byte slot maps and has no block
schedule (a blocked request runs staged).  The pattern must still equal the
oracle's bit for bit, and the staged and atomic scatters must match
the oracle's values at the usual tolerance, for every element family that
otherwise uses byte slot maps."""

import pytest
import torch

import oracle
from gpu_util import assert_csr_close, fan, star

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


CASES = [("planar P1", lambda: fan(300, 1, False)),
         ("planar P2", lambda: fan(120, 2, False)),
         ("surface P1", lambda: fan(300, 1, True)),
         ("surface P2", lambda: fan(120, 2, True)),
         ("planar P3", lambda: fan(60, 3, False)),
         ("surface P4", lambda: fan(40, 4, True)),
         ("tetrahedra P2", lambda: star(100, 2))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_long_rows_match_oracle(lf, name, make):
    m = make()
    d = lf.DeviceMesh.from_dict(m)
    d.build_pattern()
    info = lf.lfem_pattern_info(d.pattern)
    assert info["max_row"] > 255, info
    assert info["slot_bytes"] == 2 and info["blocks"] == 0
    assert info["scatter"] == lf.LFEM_SCATTER_STAGED
    rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
    coef = torch.as_tensor(m["coef"], device="cuda")
    refs = {"M": oracle.assemble(m, "mass"), "A": oracle.assemble(m, "stiffness", coef=m["coef"]),
            "MC": oracle.assemble(m, "mass", coef=m["coef"])}
    what = lf.LFEM_M | lf.LFEM_A | lf.LFEM_MC
    first = None
    for scatter in (lf.LFEM_SCATTER_AUTO, lf.LFEM_SCATTER_STAGED, lf.LFEM_SCATTER_BLOCKED,
                    lf.LFEM_SCATTER_ATOMIC):
        out = d.assemble(what, coef_a=coef, coef_c=coef, scatter=scatter)
        for key, ref in refs.items():
            assert_csr_close(rp, ci, out[key].cpu().numpy(), ref, what=f"{name} scatter {scatter} {key}")
        if scatter == lf.LFEM_SCATTER_AUTO:
            first = {k: v.clone() for k, v in out.items()}
        elif scatter != lf.LFEM_SCATTER_ATOMIC:
            # the automatic choice and a blocked request both run the staged scatter
            for key in refs:
                assert torch.equal(out[key], first[key]), key
    d.close()


def test_long_rows_tune_debug_and_schedule(lf):
    m = fan(300, 2, True)
    d = lf.DeviceMesh.from_dict(m)
    d.build_pattern()
    rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
    ref_m, ref_a = oracle.assemble(m, "mass"), oracle.assemble(m, "stiffness")
    v, cap = lf.lfem_pattern_autotune_ex(d.handle, d.pattern, lf.LFEM_M | lf.LFEM_A,
                                         lf.LFEM_TUNE_ALLOW_ATOMIC | lf.LFEM_TUNE_NO_CACHE)
    assert v in (lf.LFEM_SCATTER_STAGED, lf.LFEM_SCATTER_ATOMIC) and cap == 0
    with pytest.raises(lf.LfemError) as e:
        lf.lfem_pattern_schedule(d.handle, d.pattern, lf.LFEM_SCATTER_BLOCKED, 1024)
    assert e.value.status == lf.LFEM_EUNSUPPORTED
    lf.lfem_pattern_schedule(d.handle, d.pattern, lf.LFEM_SCATTER_STAGED, 0)
    was = lf.lfem_set_debug(1)
    try:
        out = d.assemble(lf.LFEM_M | lf.LFEM_A)  # every slot checked against its row first
    finally:
        lf.lfem_set_debug(int(was))
    assert_csr_close(rp, ci, out["M"].cpu().numpy(), ref_m, what="debug M")
    assert_csr_close(rp, ci, out["A"].cpu().numpy(), ref_a, what="debug A")
    d.close()


def test_short_rows_keep_byte_slots(lf):
    # 250 triangles around the centre: its row holds 251 entries, byte slots
    m = fan(250, 1, False)
    d = lf.DeviceMesh.from_dict(m)
    d.build_pattern()
    info = lf.lfem_pattern_info(d.pattern)
    assert info["max_row"] == 251 and info["slot_bytes"] == 1 and info["blocks"] > 0
    rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
    out = d.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    assert_csr_close(rp, ci, out["M"].cpu().numpy(), oracle.assemble(m, "mass"), what="M")
    assert_csr_close(rp, ci, out["A"].cpu().numpy(), oracle.assemble(m, "stiffness"), what="A")
    d.close()
