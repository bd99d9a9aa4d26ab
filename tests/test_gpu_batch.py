"""Batched multi-mesh assembly (one HIP graph replay: the persistent kernel for
its family of meshes, a launch of its own for every other member) against
per-mesh launches (bitwise: same schedule, same summation order) and against
the oracle."""

import numpy as np
import pytest
import torch

import meshgen
import oracle
from gpu_util import assert_csr_close, fan, order_mesh
from meshgen import meshes as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14035_amd as lf
    return lf


def mixed_meshes():
    out = []
    for t in meshgen.ALL_TYPES:
        if t[1] <= 2:
            out.append(meshgen.small_mesh(*t, size=3))
    for freq, order in ((7, 1), (9, 2), (16, 2)):
        V, F = mg.sphere_geodesic(freq, order=order)
        V, F, _ = mg.sfc_reorder(V, F)
        coords, conn = mg.to_soa(V * 1.3, F)
        out.append(dict(domain="surface", dim=2, order=order, quad=3 if order == 1 else 6,
                        coords=coords, conn=conn))
    return out


def run_batch(lf, dms, what, autotune=0, vals=None):
    nmat = (1 if what & lf.LFEM_M else 0) + (1 if what & lf.LFEM_A else 0)
    b = lf.lfem_batch_create([d.handle for d in dms], [d.pattern for d in dms], what, autotune)
    if vals is None:
        vals = [torch.full((max(d.nnz, 1),), float("nan"), dtype=torch.float64, device="cuda")
                for d in dms for _ in range(nmat)]
    lf.lfem_assemble_batch(b, vals)
    torch.cuda.synchronize()
    return b, vals


@pytest.mark.parametrize("what", ["MA", "M", "A"])
def test_batch_matches_single_and_oracle(lf, what):
    w = {"MA": lf.LFEM_M | lf.LFEM_A, "M": lf.LFEM_M, "A": lf.LFEM_A}[what]
    ms = mixed_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    b, vals = run_batch(lf, dms, w)
    nmat = len(what)
    for i, (m, d) in enumerate(zip(ms, dms)):
        single = d.assemble(w, scatter=lf.LFEM_SCATTER_BLOCKED)
        rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
        for j, key in enumerate(k for k in ("M", "A") if k in what):
            got = vals[i * nmat + j][:d.nnz]
            assert torch.equal(got, single[key]), (i, key)
            kind = "mass" if key == "M" else "stiffness"
            assert_csr_close(rp, ci, got.cpu().numpy(), oracle.assemble(m, kind),
                             what=f"batch mesh {i} {key}")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_new_outputs_autotune_and_replay(lf):
    ms = mixed_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w, autotune=1)
    ref = [v.clone() for v in vals]
    # replay with the same outputs, then with new output tensors
    lf.lfem_assemble_batch(b, vals)
    vals2 = [torch.zeros_like(v) for v in vals]
    lf.lfem_assemble_batch(b, vals2)
    torch.cuda.synchronize()
    for r, v1, v2 in zip(ref, vals, vals2):
        assert torch.equal(r, v1) and torch.equal(r, v2)
    # results equal a fresh per-mesh assembly with the tuned schedules
    for i, d in enumerate(dms):
        single = d.assemble(w, scatter=lf.LFEM_SCATTER_BLOCKED)
        assert torch.equal(vals2[2 * i][:d.nnz], single["M"])
        assert torch.equal(vals2[2 * i + 1][:d.nnz], single["A"])
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_edge_cases(lf):
    one = meshgen.small_mesh("surface", 2, 2, size=2)
    d = lf.DeviceMesh.from_dict(one)
    d.build_pattern()
    b, vals = run_batch(lf, [d], lf.LFEM_M)
    ref = d.assemble(lf.LFEM_M, scatter=lf.LFEM_SCATTER_BLOCKED)["M"]
    assert torch.equal(vals[0][:d.nnz], ref)
    lf.lfem_batch_destroy(b)
    # a mesh without elements in the batch
    empty = dict(one)
    empty["conn"] = np.zeros((6, 0), dtype=np.int32)
    de = lf.DeviceMesh.from_dict(empty)
    de.build_pattern()
    b = lf.lfem_batch_create([d.handle, de.handle], [d.pattern, de.pattern], lf.LFEM_M)
    v = torch.empty(d.nnz, dtype=torch.float64, device="cuda")
    lf.lfem_assemble_batch(b, [v, torch.empty(1, dtype=torch.float64, device="cuda")])
    torch.cuda.synchronize()
    assert torch.equal(v, ref)
    lf.lfem_batch_destroy(b)
    # argument errors
    with pytest.raises(lf.LfemError) as ei:
        lf.lfem_batch_create([d.handle], [d.pattern], 8)
    assert ei.value.status == lf.LFEM_EINVAL
    with pytest.raises(lf.LfemError) as ei:  # the weighted mass without its weight
        lf.lfem_batch_create([d.handle], [d.pattern], lf.LFEM_MC)
    assert ei.value.status == lf.LFEM_EINVAL
    for x in (d, de):
        x.close()


def test_batch_follows_moved_coordinates(lf):
    """lfem_mesh_set_coords on a batched mesh: the next batch call assembles at
    the new coordinates (a new tensor, the old one released)."""
    ms = mixed_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w)
    i = len(dms) - 1  # the frequency-16 P2 sphere
    moved = dict(ms[i])
    moved["coords"] = ms[i]["coords"] * 0.7
    dms[i].set_coords(torch.as_tensor(moved["coords"], device="cuda"))
    torch.cuda.empty_cache()
    lf.lfem_assemble_batch(b, vals)
    torch.cuda.synchronize()
    rp, ci = (x.cpu().numpy() for x in dms[i].pattern_tensors())
    for j, kind in enumerate(("mass", "stiffness")):
        assert_csr_close(rp, ci, vals[2 * i + j][:dms[i].nnz].cpu().numpy(), oracle.assemble(moved, kind),
                         what=f"moved mesh {kind}")
    # the unmoved meshes are unchanged
    for k, d in enumerate(dms[:-1]):
        single = d.assemble(w, scatter=lf.LFEM_SCATTER_BLOCKED)
        assert torch.equal(vals[2 * k][:d.nnz], single["M"])
        assert torch.equal(vals[2 * k + 1][:d.nnz], single["A"])
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_after_pattern_retuned(lf):
    """A pattern's schedule rebuilt after the batch was created (autotuning the
    pattern): the batch rebuilds its work list and still matches per-mesh
    launches with the new schedules bitwise, and the oracle."""
    ms = mixed_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w)
    for d in dms[-2:]:
        lf.lfem_pattern_autotune(d.handle, d.pattern, w)
    vals2 = [torch.full_like(v, float("nan")) for v in vals]
    lf.lfem_assemble_batch(b, vals2)
    torch.cuda.synchronize()
    for i, (m, d) in enumerate(zip(ms, dms)):
        single = d.assemble(w, scatter=lf.LFEM_SCATTER_BLOCKED)
        assert torch.equal(vals2[2 * i][:d.nnz], single["M"]), i
        assert torch.equal(vals2[2 * i + 1][:d.nnz], single["A"]), i
        rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
        assert_csr_close(rp, ci, vals2[2 * i + 1][:d.nnz].cpu().numpy(), oracle.assemble(m, "stiffness"),
                         what=f"retuned batch mesh {i}")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_config4_full_batch(lf):
    """All 256 meshes of the batched workload (displaced geodesic spheres,
    P1/P2 alternating, 11.4 M triangles), autotuned as the benchmark runs it:
    every output bitwise equal to the per-mesh launch with the same schedule,
    and a few meshes (the smallest P1 and P2, a mid-size P2) against the
    oracle in full."""
    ms = meshgen.config4()
    print("config4: 256 meshes", flush=True)
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w, autotune=1)
    print("config4: batch done, comparing with per-mesh launches", flush=True)
    for i, d in enumerate(dms):
        single = d.assemble(w, scatter=lf.LFEM_SCATTER_BLOCKED)
        assert torch.equal(vals[2 * i][:d.nnz], single["M"]), i
        assert torch.equal(vals[2 * i + 1][:d.nnz], single["A"]), i
        del single
    sizes = [d.T for d in dms]
    p1 = [i for i in range(len(ms)) if ms[i]["order"] == 1]
    p2 = [i for i in range(len(ms)) if ms[i]["order"] == 2]
    picks = {min(p1, key=sizes.__getitem__), min(p2, key=sizes.__getitem__),
             sorted(p2, key=sizes.__getitem__)[len(p2) // 2]}
    for i in sorted(picks):
        print(f"config4: oracle check mesh {i} ({sizes[i]} triangles, P{ms[i]['order']})", flush=True)
        rp, ci = (x.cpu().numpy() for x in dms[i].pattern_tensors())
        for j, kind in enumerate(("mass", "stiffness")):
            assert_csr_close(rp, ci, vals[2 * i + j][:dms[i].nnz].cpu().numpy(), oracle.assemble(ms[i], kind),
                             what=f"config4 mesh {i} {kind}")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def mixed_family_meshes():
    """Members inside and outside the persistent kernel's family: P1 curve and
    P2 surface (inside), a P2 surface under the 16-point rule, P2 and cubic
    tetrahedra, a quartic planar mesh, a cubic curve and a P2 surface with a
    row of more than 255 entries (no block schedule) (outside)."""
    out = [meshgen.small_mesh("surface", 1, 1, size=3), meshgen.small_mesh("surface", 2, 2, size=3),
           dict(meshgen.small_mesh("surface", 2, 2, size=2), quad=16),
           meshgen.small_mesh("bulk", 3, 2, size=2), order_mesh("bulk", 3, 3), order_mesh("bulk", 2, 4),
           order_mesh("surface", 1, 3), fan(120, 2, True)]  # the fan's centre row exceeds 255 entries
    rng = np.random.default_rng(7)
    for m in out:
        N = m["coords"].shape[1]
        m.setdefault("coef_a", rng.uniform(0.5, 2.0, size=N))
        m.setdefault("coef_c", rng.uniform(0.5, 2.0, size=N))
    return out


def check_members(lf, ms, dms, vals, keys, coefs, label):
    nmat = len(keys)
    for i, (m, d) in enumerate(zip(ms, dms)):
        ca, cc = coefs[i]
        w = sum({"M": lf.LFEM_M, "A": lf.LFEM_A, "MC": lf.LFEM_MC}[k] for k in keys)
        single = d.assemble(w, coef_a=ca, coef_c=cc)
        rp, ci = (x.cpu().numpy() for x in d.pattern_tensors())
        for j, key in enumerate(keys):
            got = vals[i * nmat + j][:d.nnz]
            assert torch.equal(got, single[key]), (label, i, key)
            if key == "M":
                ref = oracle.assemble(m, "mass")
            elif key == "MC":
                ref = oracle.assemble(m, "mass", coef=m["coef_c"])
            else:
                ref = oracle.assemble(m, "stiffness", coef=m["coef_a"] if ca is not None else None)
            assert_csr_close(rp, ci, got.cpu().numpy(), ref, what=f"{label} mesh {i} {key}")


@pytest.mark.parametrize("autotune", [0, 1])
def test_batch_mixed_members(lf, autotune):
    """Plain M and A over members in and outside the persistent kernel's
    family, one graph replay; each output bitwise equal to lfem_assemble with
    the tuned scatter and within tolerance of the oracle; replays with new
    outputs (graph captured again) equal the first."""
    ms = mixed_family_meshes()
    print("mixed batch:", [(m["domain"], m["dim"], m["order"], m.get("quad")) for m in ms], flush=True)
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w, autotune=autotune)
    check_members(lf, ms, dms, vals, ("M", "A"), [(None, None)] * len(ms), "mixed")
    ref = [v.clone() for v in vals]
    vals2 = [torch.full_like(v, float("nan")) for v in vals]
    for _ in range(2):
        lf.lfem_assemble_batch(b, vals2)
    lf.lfem_assemble_batch(b, vals)
    torch.cuda.synchronize()
    for r, v1, v2 in zip(ref, vals, vals2):
        assert torch.equal(r, v1) and torch.equal(r, v2)
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_coefficients_and_weighted_mass(lf):
    """M, A_a and M_c for every member (all outside the persistent kernel,
    which runs plain M and A); coefficient values changed between replays are
    read by the next replay."""
    ms = mixed_family_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    ca = [torch.as_tensor(m["coef_a"], device="cuda") for m in ms]
    cc = [torch.as_tensor(m["coef_c"], device="cuda") for m in ms]
    w = lf.LFEM_M | lf.LFEM_A | lf.LFEM_MC
    b = lf.lfem_batch_create_ex([d.handle for d in dms], [d.pattern for d in dms], w, ca, cc)
    vals = [torch.full((max(d.nnz, 1),), float("nan"), dtype=torch.float64, device="cuda")
            for d in dms for _ in range(3)]
    lf.lfem_assemble_batch(b, vals)
    torch.cuda.synchronize()
    check_members(lf, ms, dms, vals, ("M", "A", "MC"), list(zip(ca, cc)), "coefficients")
    # new coefficient values in the same tensors: the next replay reads them
    for i, m in enumerate(ms):
        m["coef_a"] = m["coef_a"] * 1.5 + 0.25
        m["coef_c"] = m["coef_c"] * 0.5 + 1.0
        ca[i].copy_(torch.as_tensor(m["coef_a"]))
        cc[i].copy_(torch.as_tensor(m["coef_c"]))
    lf.lfem_assemble_batch(b, vals)
    torch.cuda.synchronize()
    check_members(lf, ms, dms, vals, ("M", "A", "MC"), list(zip(ca, cc)), "new coefficients")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_partial_coefficients(lf):
    """A_a on some members only: the members without a coefficient stay in
    the persistent kernel (plain A), the others get their own launch."""
    ms = mixed_family_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    ca = [torch.as_tensor(m["coef_a"], device="cuda") if i % 2 else None for i, m in enumerate(ms)]
    w = lf.LFEM_M | lf.LFEM_A
    b = lf.lfem_batch_create_ex([d.handle for d in dms], [d.pattern for d in dms], w, ca, None, 1)
    vals = [torch.full((max(d.nnz, 1),), float("nan"), dtype=torch.float64, device="cuda")
            for d in dms for _ in range(2)]
    lf.lfem_assemble_batch(b, vals)
    torch.cuda.synchronize()
    check_members(lf, ms, dms, vals, ("M", "A"), [(c, None) for c in ca], "partial coefficients")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_member_state_changes(lf):
    """Changes the graph must follow: a member outside the persistent kernel
    moved to new coordinates, and its pattern's staging buffers reallocated by
    a wider assembly on the same pattern between replays."""
    ms = mixed_family_meshes()
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    b, vals = run_batch(lf, dms, lf.LFEM_M)
    # the cubic tetrahedra (always staged): a three-matrix assembly needs a
    # larger staging buffer than the batch's one-matrix launch
    i = 4
    cc = torch.as_tensor(ms[i]["coef_c"], device="cuda")
    dms[i].assemble(lf.LFEM_M | lf.LFEM_A | lf.LFEM_MC, coef_c=cc)
    # the P2 tetrahedra (staged by default): the same, which also regrows the
    # array of vertex diagonals that their long-list reduction reads
    k = 3
    cc3 = torch.as_tensor(ms[k]["coef_c"], device="cuda")
    dms[k].assemble(lf.LFEM_M | lf.LFEM_A | lf.LFEM_MC, coef_c=cc3)
    # the quartic planar mesh moved
    j = 5
    ms[j] = dict(ms[j], coords=ms[j]["coords"] * 1.25)
    dms[j].set_coords(torch.as_tensor(ms[j]["coords"], device="cuda"))
    vals2 = [torch.full_like(v, float("nan")) for v in vals]
    lf.lfem_assemble_batch(b, vals2)
    torch.cuda.synchronize()
    check_members(lf, ms, dms, vals2, ("M",), [(None, None)] * len(ms), "state changes")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_prebuilt_arguments(lf):
    """BatchOutputs (the output pointer array marshalled once) and
    prepare_assemble (a per-mesh call marshalled once) give the same bits as
    the per-call forms."""
    ms = mixed_meshes()[:4]
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w)
    outs = lf.BatchOutputs([torch.full_like(v, float("nan")) for v in vals])
    lf.lfem_assemble_batch(b, outs)
    lf.lfem_assemble_batch(b, outs)
    torch.cuda.synchronize()
    for r, v in zip(vals, outs.vals):
        assert torch.equal(r, v)
    for i, d in enumerate(dms):
        vm = torch.full((d.nnz,), float("nan"), dtype=torch.float64, device="cuda")
        va = torch.full_like(vm, float("nan"))
        call = lf.prepare_assemble(d.handle, d.pattern, w, None, None, vm, va, None, lf.LFEM_SCATTER_BLOCKED)
        call()
        call()
        torch.cuda.synchronize()
        assert torch.equal(vm, vals[2 * i][:d.nnz]) and torch.equal(va, vals[2 * i + 1][:d.nnz])
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()


def test_batch_member_schedule_built_later(lf):
    """A P2-tetrahedron member (staged by default, no block schedule at
    pattern build) whose block schedule is built after the batch was created,
    by an explicit blocked request on its pattern: the batch notices the new
    schedule generation, keeps the member on its staged launch, and its
    replays still equal per-mesh assembly."""
    ms = [meshgen.small_mesh("surface", 2, 2, size=3), meshgen.small_mesh("bulk", 3, 2, size=3)]
    dms = [lf.DeviceMesh.from_dict(m) for m in ms]
    for d in dms:
        d.build_pattern()
    assert lf.lfem_pattern_info(dms[1].pattern)["blocks"] == 0
    w = lf.LFEM_M | lf.LFEM_A
    b, vals = run_batch(lf, dms, w)
    check_members(lf, ms, dms, vals, ("M", "A"), [(None, None)] * len(ms), "before")
    blocked = dms[1].assemble(w, scatter=lf.LFEM_SCATTER_BLOCKED)  # builds the colour schedule
    assert lf.lfem_pattern_info(dms[1].pattern)["blocks"] > 0
    vals2 = [torch.full_like(v, float("nan")) for v in vals]
    lf.lfem_assemble_batch(b, vals2)
    torch.cuda.synchronize()
    for v1, v2 in zip(vals, vals2):
        assert torch.equal(v1, v2)
    check_members(lf, ms, dms, vals2, ("M", "A"), [(None, None)] * len(ms), "after")
    rp, ci = (x.cpu().numpy() for x in dms[1].pattern_tensors())
    assert_csr_close(rp, ci, blocked["A"].cpu().numpy(), oracle.assemble(ms[1], "stiffness"), what="blocked A")
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()
