"""GPU parity under the high-order rules of the paper's precomputations
(section 5.2): Gauss with 5 and 6 points on segments, the 16-point degree-8
Dunavant rule on triangles, a symmetric 35-point degree-7 rule on tetrahedra.

The library builds these rules itself (Newton on the Legendre recurrence;
the published 15-digit Dunavant values; Newton in double on the tetrahedral
rule's moment equations); the oracle solves their moment equations in high
precision.  Matrices, load vector and shape gradient are
compared with the oracle at the same tolerances as under the default rules
(1e-12 row-scaled); the rules' own difference is below 1e-14."""

import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import grad_abs_scale
from gpu_util import assert_csr_close, assert_rows_close

pytestmark = pytest.mark.gpu

# (element type, points): curves take Gauss 5 and 6, triangles Dunavant 16
HIGH = [(t, q) for t in meshgen.ALL_TYPES if t[1] == 1 for q in (5, 6)] + \
       [(t, 16) for t in meshgen.ALL_TYPES if t[1] == 2] + \
       [(t, 35) for t in meshgen.ALL_TYPES if t[1] == 3]


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def with_rule(m, q):
    m = dict(m)
    m["quad"] = q
    return m


@pytest.mark.parametrize("t,q", HIGH)
@pytest.mark.parametrize("variant", ["blocked", "staged", "atomic"])
def test_matrices(lf, t, q, variant):
    m = with_rule(meshgen.small_mesh(*t, size=3), q)
    say("case", t, q, variant)
    dm = lf.DeviceMesh.from_dict(m)
    v = {"blocked": lf.LFEM_SCATTER_BLOCKED, "staged": lf.LFEM_SCATTER_STAGED,
         "atomic": lf.LFEM_SCATTER_ATOMIC}[variant]
    ca = torch.as_tensor(m["coef_a"], device="cuda")
    cc = torch.as_tensor(m["coef_c"], device="cuda")
    out = dm.assemble(lf.LFEM_M | lf.LFEM_MC | lf.LFEM_A, coef_a=ca, coef_c=cc, scatter=v)
    out2 = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=v)
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    tol = 1e-12
    checks = [("M", out["M"], oracle.assemble(m, "mass")),
              ("MC", out["MC"], oracle.assemble(m, "mass", coef=m["coef_c"])),
              ("A_a", out["A"], oracle.assemble(m, "stiffness", coef=m["coef_a"])),
              ("M2", out2["M"], oracle.assemble(m, "mass")),
              ("A", out2["A"], oracle.assemble(m, "stiffness"))]
    for name, got, ref in checks:
        assert_csr_close(rp, ci, got.cpu().numpy(), ref, tol=tol, what=f"{t} Q={q} {variant} {name}")
    dm.close()


@pytest.mark.parametrize("t,q", HIGH)
def test_load_and_shape_grad(lf, t, q):
    m = with_rule(meshgen.small_mesh(*t, size=3), q)
    say("case", t, q, "load, shape gradient")
    dm = lf.DeviceMesh.from_dict(m)
    f = m["coef_c"]
    b = dm.load(torch.as_tensor(f, device="cuda")).cpu().numpy()
    bref = oracle.load(m, f)
    assert np.abs(b - bref).max() <= 1e-12 * np.abs(bref).max()
    rng = np.random.default_rng(5)
    u, w = rng.normal(size=dm.N), rng.normal(size=dm.N)
    ut, wt = (torch.as_tensor(x, device="cuda") for x in (u, w))
    g = torch.empty_like(dm.coords)
    lf.lfem_shape_grad(dm.handle, ut, ut, 1.0, wt, wt, 0.5, g)
    ref = oracle.shape_grad(m, u, u, 1.0, w, w, 0.5)
    gg = g.cpu().numpy()
    # entry by entry against 1e-12 of the summed absolute element contributions
    # (the rounding scale of a sum whose terms cancel); normwise printed beside
    S = grad_abs_scale(oracle, m, u, u, 1.0, w, w, 0.5)
    err = float((np.abs(gg - ref) / S).max())
    say(f"  shape gradient error {err:.2e} of sum|g_e|, {np.linalg.norm(gg - ref) / np.linalg.norm(ref):.2e} normwise")
    assert err <= 1e-12
    dm.close()


@pytest.mark.parametrize("t,q", [(("surface", 2, 2), 16), (("surface", 1, 2), 6), (("bulk", 3, 2), 35)])
def test_high_order_rule_differs_from_default(lf, t, q):
    """The rule is really switched: on a curved P2 mesh the high-order rule's
    load vector differs from the default rule's, while both give nearly the
    same total measure, and the high-order total matches the oracle's."""
    m = meshgen.small_mesh(*t, size=3)
    mh = with_rule(m, q)
    dm, dh = lf.DeviceMesh.from_dict(m), lf.DeviceMesh.from_dict(mh)
    b, bh = dm.load().cpu().numpy(), dh.load().cpu().numpy()
    assert not np.array_equal(b, bh)
    assert abs(b.sum() - bh.sum()) <= 1e-3 * abs(bh.sum())
    assert abs(bh.sum() - oracle.load(mh).sum()) <= 1e-13 * abs(bh.sum())
    dm.close()
    dh.close()


def test_batch_member_with_high_order_rule(lf):
    """A high-order rule is outside the persistent kernel: the batch assembles
    that mesh with its own launch in the graph, bitwise as a single call."""
    m = with_rule(meshgen.small_mesh("surface", 2, 2, size=2), 16)
    dm = lf.DeviceMesh.from_dict(m)
    dm.build_pattern()
    b = lf.lfem_batch_create([dm.handle], [dm.pattern], lf.LFEM_M | lf.LFEM_A, 0)
    vals = [torch.full((dm.nnz,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(2)]
    lf.lfem_assemble_batch(b, vals)
    single = dm.assemble(lf.LFEM_M | lf.LFEM_A)
    torch.cuda.synchronize()
    assert torch.equal(vals[0], single["M"]) and torch.equal(vals[1], single["A"])
    lf.lfem_batch_destroy(b)
    dm.close()


def test_tetrahedron_rejects_triangle_rule(lf):
    m = with_rule(meshgen.small_mesh("bulk", 3, 2, size=2), 16)
    with pytest.raises(lf.LfemError) as e:
        lf.DeviceMesh.from_dict(m)
    assert e.value.status == lf.LFEM_EUNSUPPORTED


def test_config3_degree7_full_size_sampled(lf):
    """The 1,572,864-tetrahedron workload under the 35-point degree-7 rule, in
    the launch the benchmark row times (scatter chosen by the autotuner, M and
    A_a in one call): sampled rows against the oracle under the same rule,
    1^T M 1 = 1 and A_a 1 = 0."""
    m = dict(meshgen.config3(), quad=35)
    say("config3 full size, 35-point rule")
    dm = lf.DeviceMesh.from_dict(m)
    dm.build_pattern()
    lf.lfem_pattern_autotune(dm.handle, dm.pattern, lf.LFEM_M | lf.LFEM_A)
    ca = torch.as_tensor(m["coef_a"], device="cuda")
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A, coef_a=ca)
    assert abs(float(out["M"].sum().item()) - 1.0) < 1e-12
    rp_t, ci_t = dm.pattern_tensors()
    rows_t = torch.repeat_interleave(torch.arange(dm.N, device="cuda"), (rp_t[1:] - rp_t[:-1]).long())
    a1 = torch.zeros(dm.N, dtype=torch.float64, device="cuda").index_add_(0, rows_t, out["A"])
    amax = torch.zeros(dm.N, dtype=torch.float64, device="cuda").index_reduce_(0, rows_t, out["A"].abs(), "amax")
    assert float((a1.abs() / amax).max().item()) < 1e-12
    rp, ci = rp_t.cpu().numpy(), ci_t.cpu().numpy()
    rows = np.unique(np.random.default_rng(13).integers(0, dm.N, 200))
    for key, kind, c in (("M", "mass", None), ("A", "stiffness", m["coef_a"])):
        ref = oracle.assemble(m, kind, coef=c, rows=rows)
        assert_rows_close(rp, ci, out[key].cpu().numpy(), ref, rows, what=f"c3 Q=35 {key}")
    dm.close()
