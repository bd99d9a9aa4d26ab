"""GPU parity: the C-ABI library against the CPU oracle, element by element.

CSR pattern bit-exact; values within 1e-12 row-scaled relative (the
quadrature-defined matrices are computed exactly up to rounding order)."""

import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import TOL, assert_csr_close, assert_rows_close

pytestmark = pytest.mark.gpu

VARIANTS = ["blocked", "staged", "atomic"]


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def variant_id(lf, name):
    return {"blocked": lf.LFEM_SCATTER_BLOCKED, "staged": lf.LFEM_SCATTER_STAGED,
            "atomic": lf.LFEM_SCATTER_ATOMIC}[name]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# every selection of matrices and coefficients (the side-slot kernels are
# specialised on which outputs carry a coefficient)
SELECTIONS = ["M", "A", "MC", "Aa", "M+A", "M+MC", "MC+Aa", "M+Aa", "M+MC+A", "M+MC+Aa", "A+MC"]


@pytest.mark.parametrize("t", [t for t in meshgen.ALL_TYPES if t[1] <= 2 and t[2] == 2])
@pytest.mark.parametrize("sel", SELECTIONS)
def test_matrix_and_coefficient_selections(lf, t, sel):
    m = meshgen.small_mesh(*t, size=3)
    say("case", t, sel)
    dm = lf.DeviceMesh.from_dict(m)
    parts = sel.split("+")
    what = ((lf.LFEM_M if "M" in parts else 0) | (lf.LFEM_MC if "MC" in parts else 0) |
            (lf.LFEM_A if ("A" in parts or "Aa" in parts) else 0))
    ca = torch.as_tensor(m["coef_a"], device="cuda") if "Aa" in parts else None
    cc = torch.as_tensor(m["coef_c"], device="cuda") if "MC" in parts else None
    out = dm.assemble(what, coef_a=ca, coef_c=cc, scatter=lf.LFEM_SCATTER_BLOCKED)
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    refs = {"M": ("M", oracle.assemble(m, "mass")),
            "MC": ("MC", oracle.assemble(m, "mass", coef=m["coef_c"])),
            "A": ("A", oracle.assemble(m, "stiffness")),
            "Aa": ("A", oracle.assemble(m, "stiffness", coef=m["coef_a"]))}
    for part in parts:
        key, ref = refs[part]
        assert_csr_close(rp, ci, out[key].cpu().numpy(), ref, what=f"{t} {sel} {part}")
    dm.close()


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
@pytest.mark.parametrize("variant", VARIANTS)
def test_small_all_types(lf, t, variant):
    m = meshgen.small_mesh(*t, size=3)
    say("case", t, variant, m["conn"].shape)
    dm = lf.DeviceMesh.from_dict(m)
    ca = torch.as_tensor(m["coef_a"], device="cuda")
    cc = torch.as_tensor(m["coef_c"], device="cuda")
    v = variant_id(lf, variant)
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A | lf.LFEM_MC, coef_a=ca, coef_c=cc, scatter=v)
    out2 = dm.assemble(lf.LFEM_A, scatter=v)
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    checks = [("M", out["M"], oracle.assemble(m, "mass")),
              ("A_a", out["A"], oracle.assemble(m, "stiffness", coef=m["coef_a"])),
              ("M_c", out["MC"], oracle.assemble(m, "mass", coef=m["coef_c"])),
              ("A", out2["A"], oracle.assemble(m, "stiffness"))]
    for name, got, ref in checks:
        assert_csr_close(rp, ci, got.cpu().numpy(), ref, what=f"{t} {variant} {name}")
    assert dm.degenerate_count() == 0
    dm.close()


@pytest.mark.parametrize("t", meshgen.ALL_TYPES)
def test_single_element_and_ragged(lf, t):
    m = meshgen.small_mesh(*t, size=2)
    for T in (1, 3, 257):
        T = min(T, m["conn"].shape[1])
        sub = dict(m)
        sub["conn"] = np.ascontiguousarray(m["conn"][:, :T])
        dm = lf.DeviceMesh.from_dict(sub)
        for variant in VARIANTS:
            out = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=variant_id(lf, variant))
            rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
            assert_csr_close(rp, ci, out["M"].cpu().numpy(), oracle.assemble(sub, "mass"),
                             what=f"{t} T={T} {variant} M")
            assert_csr_close(rp, ci, out["A"].cpu().numpy(), oracle.assemble(sub, "stiffness"),
                             what=f"{t} T={T} {variant} A")
        dm.close()


def test_isolated_node_and_empty_mesh(lf):
    m = meshgen.small_mesh("surface", 2, 1, size=2)
    # one extra node referenced by no element: an empty row
    m = dict(m)
    m["coords"] = np.ascontiguousarray(np.concatenate([m["coords"], [[2.0], [2.0], [2.0]]], 1))
    dm = lf.DeviceMesh.from_dict(m)
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A)
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    assert rp[-1] == rp[-2]
    assert_csr_close(rp, ci, out["M"].cpu().numpy(), oracle.assemble(m, "mass"), what="isolated")
    dm.close()
    e = dict(m)
    e["conn"] = np.zeros((3, 0), dtype=np.int32)
    dm = lf.DeviceMesh.from_dict(e)
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A)
    assert dm.nnz == 0
    rp, ci = dm.pattern_tensors()
    assert int(rp.max().item()) == 0
    dm.close()


def test_invalid_inputs_rejected(lf):
    m = meshgen.small_mesh("surface", 2, 1, size=2)
    bad = dict(m)
    conn = m["conn"].copy()
    conn[1, 5] = m["coords"].shape[1] + 7  # out of range: the kernels skip it and flag it
    bad["conn"] = conn
    dm = lf.DeviceMesh.from_dict(bad)
    with pytest.raises(lf.LfemError) as ei:
        dm.build_pattern()
    assert ei.value.status == 1
    dm.close()
    rep = dict(m)
    conn = m["conn"].copy()
    conn[1, 2] = conn[0, 2]
    rep["conn"] = conn
    dm = lf.DeviceMesh.from_dict(rep)
    with pytest.raises(lf.LfemError):
        dm.build_pattern()
    dm.close()
    with pytest.raises(lf.LfemError) as ei:
        lf.DeviceMesh("surface", 2, 2, m["coords"], np.zeros((6, 4), np.int32), quad_points=5)
    assert ei.value.status == 6


def test_degenerate_counter(lf):
    V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    F = np.array([[0, 1, 2], [0, 1, 3]])
    dm = lf.DeviceMesh("surface", 2, 1, V.T, F.T.astype(np.int32))
    dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_STAGED)
    assert dm.degenerate_count() == 3  # three quadrature points of the collinear triangle
    dm.close()


@pytest.mark.parametrize("variant", VARIANTS)
def test_config1_full(lf, variant):
    m = meshgen.config1()
    say("config1", variant)
    dm = lf.DeviceMesh.from_dict(m)
    cc = torch.as_tensor(m["coef_c"], device="cuda")
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A | lf.LFEM_MC, coef_c=cc, scatter=variant_id(lf, variant))
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    assert dm.nnz == 17922
    assert_csr_close(rp, ci, out["M"].cpu().numpy(), oracle.assemble(m, "mass"), what="c1 M")
    assert_csr_close(rp, ci, out["A"].cpu().numpy(), oracle.assemble(m, "stiffness"), what="c1 A")
    assert_csr_close(rp, ci, out["MC"].cpu().numpy(), oracle.assemble(m, "mass", coef=m["coef_c"]),
                     what="c1 M_c")
    dm.close()


@pytest.fixture(scope="module")
def c2():
    return meshgen.config2()


def test_config2_full_blocked_and_determinism(lf, c2):
    """The benchmark's workload and launch (blocked scatter, M + A in one pass),
    compared entry by entry with the oracle over the whole 655,360-element
    mesh; two runs must agree bitwise."""
    m = c2
    say("config2 full")
    dm = lf.DeviceMesh.from_dict(m)
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    again = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    assert torch.equal(out["M"], again["M"]) and torch.equal(out["A"], again["A"])
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    assert dm.nnz == 15073282
    assert_csr_close(rp, ci, out["M"].cpu().numpy(), oracle.assemble(m, "mass"), what="c2 M")
    assert_csr_close(rp, ci, out["A"].cpu().numpy(), oracle.assemble(m, "stiffness"), what="c2 A")
    # weighted mass, staged scatter, against sampled oracle rows
    cc = torch.as_tensor(m["coef_c"], device="cuda")
    st = dm.assemble(lf.LFEM_MC, coef_c=cc, scatter=lf.LFEM_SCATTER_STAGED)
    st2 = dm.assemble(lf.LFEM_MC, coef_c=cc, scatter=lf.LFEM_SCATTER_STAGED)
    assert torch.equal(st["MC"], st2["MC"])
    rows = np.unique(np.concatenate([[0, m["coords"].shape[1] - 1],
                                     np.random.default_rng(5).integers(0, m["coords"].shape[1], 500)]))
    ref = oracle.assemble(m, "mass", coef=m["coef_c"], rows=rows)
    assert_rows_close(rp, ci, st["MC"].cpu().numpy(), ref, rows, what="c2 M_c")
    dm.close()


def test_config2_every_value_written_each_launch(lf, c2):
    """Every launch of the persistent blocked kernel (also after a schedule
    rebuild by the autotuner, and with a coefficient) must write every value,
    with the same bits."""
    dm = lf.DeviceMesh.from_dict(c2)
    cc = torch.as_tensor(c2["coef_c"], device="cuda")
    ref = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    refc = dm.assemble(lf.LFEM_MC, coef_c=cc, scatter=lf.LFEM_SCATTER_BLOCKED)
    for rep in range(4):
        if rep == 2:
            lf.lfem_pattern_autotune(dm.handle, dm.pattern, lf.LFEM_M | lf.LFEM_A)
        out = {k: torch.full((int(dm.nnz),), float("nan"), dtype=torch.float64, device="cuda") for k in ("M", "A")}
        dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED, out=out)
        outc = {"MC": torch.full((int(dm.nnz),), float("nan"), dtype=torch.float64, device="cuda")}
        dm.assemble(lf.LFEM_MC, coef_c=cc, scatter=lf.LFEM_SCATTER_BLOCKED, out=outc)
        for key in ("M", "A"):
            assert torch.equal(out[key], ref[key]), (rep, key)
        assert torch.equal(outc["MC"], refc["MC"]), rep
    dm.close()


@pytest.mark.parametrize("t", [t for t in meshgen.ALL_TYPES if t[1] <= 2])
def test_small_every_value_written(lf, t):
    """Small meshes (fewer blocks than workgroups; P1 meshes take the chunked
    variant of the kernel) through the same block distribution."""
    m = meshgen.small_mesh(*t, size=3)
    dm = lf.DeviceMesh.from_dict(m)
    dm.build_pattern()
    for _ in range(3):
        out = {k: torch.full((int(dm.nnz),), float("nan"), dtype=torch.float64, device="cuda") for k in ("M", "A")}
        dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED, out=out)
        assert bool(torch.isfinite(out["M"]).all()) and bool(torch.isfinite(out["A"]).all()), t
    dm.close()


def test_config2_atomic_close(lf, c2):
    dm = lf.DeviceMesh.from_dict(c2)
    a = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_ATOMIC)
    b = dm.assemble(lf.LFEM_M | lf.LFEM_A, scatter=lf.LFEM_SCATTER_BLOCKED)
    rp = dm.pattern_tensors()[0].cpu().numpy()
    for key in ("M", "A"):
        x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
        sc = np.repeat(np.maximum.reduceat(np.abs(y), rp[:-1]), np.diff(rp))
        assert float((np.abs(x - y) / sc).max()) <= TOL
    dm.close()


@pytest.mark.parametrize("variant", ["blocked", "staged"])
def test_config3_small_full(lf, variant):
    m = meshgen.config3(n=8, variant="curved")
    dm = lf.DeviceMesh.from_dict(m)
    ca = torch.as_tensor(m["coef_a"], device="cuda")
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A, coef_a=ca, scatter=variant_id(lf, variant))
    rp, ci = (x.cpu().numpy() for x in dm.pattern_tensors())
    assert dm.nnz == 230 * 512 + 138 * 64 + 24 * 8 + 1
    assert_csr_close(rp, ci, out["M"].cpu().numpy(), oracle.assemble(m, "mass"), what="c3(8) M")
    assert_csr_close(rp, ci, out["A"].cpu().numpy(),
                     oracle.assemble(m, "stiffness", coef=m["coef_a"]), what="c3(8) A_a")
    dm.close()


@pytest.fixture(scope="module")
def c3():
    return meshgen.config3()


@pytest.mark.parametrize("tuned", [False, True])
def test_config3_full_size_sampled(lf, c3, tuned):
    """64^3 Kuhn cube, 1,572,864 P2 tets, 11-point rule, M and A_a in one call:
    with the pattern's default scatter, and (tuned) in the launch the benchmark
    row times (scatter and block size chosen by the autotuner).  Pattern size
    closed form, sampled rows against the oracle, the invariants
    1^T M 1 = 1 and A_a 1 = 0, and the same bits on a second call."""
    m = c3
    say(f"config3 full size, tuned={tuned}")
    dm = lf.DeviceMesh.from_dict(m)
    ca = torch.as_tensor(m["coef_a"], device="cuda")
    dm.build_pattern()
    assert dm.nnz == 60859905
    if tuned:
        say("  autotuned scatter:", lf.lfem_pattern_autotune(dm.handle, dm.pattern, lf.LFEM_M | lf.LFEM_A))
    out = dm.assemble(lf.LFEM_M | lf.LFEM_A, coef_a=ca)
    again = dm.assemble(lf.LFEM_M | lf.LFEM_A, coef_a=ca)
    assert torch.equal(out["M"], again["M"]) and torch.equal(out["A"], again["A"])
    del again
    rp_t, ci_t = dm.pattern_tensors()
    rows_t = torch.repeat_interleave(torch.arange(dm.N, device="cuda"),
                                     (rp_t[1:] - rp_t[:-1]).long())
    one_m_one = float(out["M"].sum().item())
    assert abs(one_m_one - 1.0) < 1e-12
    a1 = torch.zeros(dm.N, dtype=torch.float64, device="cuda").index_add_(0, rows_t, out["A"])
    amax = torch.zeros(dm.N, dtype=torch.float64, device="cuda").index_reduce_(
        0, rows_t, out["A"].abs(), "amax")
    assert float((a1.abs() / amax).max().item()) < 1e-12
    rp, ci = rp_t.cpu().numpy(), ci_t.cpu().numpy()
    rows = np.unique(np.random.default_rng(3).integers(0, dm.N, 300))
    for key, kind, c in (("M", "mass", None), ("A", "stiffness", m["coef_a"])):
        ref = oracle.assemble(m, kind, coef=c, rows=rows)
        assert_rows_close(rp, ci, out[key].cpu().numpy(), ref, rows, what=f"c3 {key}")
    dm.close()
