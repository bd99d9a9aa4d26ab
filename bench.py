#!/usr/bin/env python3
"""Benchmark: FP64 M + A assembly of the P2 ellipsoid surface mesh on one GPU.

Workload: icosahedron refined by 15 rounds of newest-vertex bisection
(655,360 curved six-node triangles, 1,310,722 nodes), P2 nodes on the
ellipsoid x^2 + y^2/0.64 + z^2/0.36 = 1, 6-point degree-4 rule.  One step is
one numeric assembly of the mass and stiffness matrices into the prebuilt CSR
pattern (15,073,282 values each) in a single fused launch; inputs are
resident in device memory.  The symbolic phase (pattern, slot map, block
schedule) runs once before timing and is reported separately.

Prints one JSON line.  Only one GPU is supported.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elements/s for M+A assembly (P2 surface), % HBM roofline, batched vs plain"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s


KERNEL_SOURCES = ("numeric_impl.hpp", "numeric_surface.hip", "side.hpp", "blocked.hpp", "element.hpp",
                  "symbolic.hip", "lfem_internal.hpp")
KERNEL_NAME = "k_side<P2 surface, Q=6, M, A>"


def kernel_source_digest() -> str:
    """Digest of the sources that define the timed kernel and its schedule."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_14035_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(digest: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "k_side_p2_ellipsoid_655360_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_digest:\s*(\S+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


def cpu_baseline(mesh):
    """The oracle as it stands, single-threaded, on the whole workload:
    mass + stiffness by element loop, COO, stable sort, CSR (median of 3)."""
    import oracle
    oracle.lib()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.assemble(mesh, "mass")
        oracle.assemble(mesh, "stiffness")
        times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    T = mesh["conn"].shape[1]
    # numeric part alone: the local matrices of every element, no scatter
    loc = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.element_matrices(mesh, "mass")
        oracle.element_matrices(mesh, "stiffness")
        loc.append(time.perf_counter() - t0)
    tl = statistics.median(loc)
    # numeric-only, like for like with the GPU's numeric phase: M and A into the
    # prebuilt pattern, each slot found by binary search in its row
    rp, ci, _ = oracle.assemble(mesh, "mass")
    num = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.assemble_numeric(mesh, "mass", (rp, ci))
        oracle.assemble_numeric(mesh, "stiffness", (rp, ci))
        num.append(time.perf_counter() - t0)
    tn = statistics.median(num)
    return {"value": T / t, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"whole workload ({T} elements, M and A, COO + stable sort + CSR), "
                      f"median of 3 runs: {t:.2f} s",
            "numeric_only": {"value": T / tn, "unit": "elements/s", "cores": 1, "seconds": tn,
                             "sample": "the same M and A summed into the prebuilt CSR pattern "
                                       "(binary-search slot lookup per row), median of 3 runs"},
            "local_matrices_only_elements_per_s": T / tl,
            "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count()}


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batched_vs_plain(lf, torch, meshgen, reps=5):
    """256 displaced geodesic spheres (P1/P2 alternating): M + A of every mesh by
    one replay of the batched graph vs 256 per-mesh launches on one stream."""
    meshes = meshgen.config4()
    dms = [lf.DeviceMesh.from_dict(m) for m in meshes]
    for d in dms:
        d.build_pattern()
    what = lf.LFEM_M | lf.LFEM_A
    vals = [torch.empty(max(d.nnz, 1), dtype=torch.float64, device="cuda") for d in dms for _ in range(2)]
    stream = torch.cuda.current_stream()

    # both sides with their arguments marshalled once (the per-call Python
    # marshalling would otherwise sit inside the timed region: about 15 us per
    # per-mesh call, about 0.1 ms for the batch's 512 output pointers); the
    # same with per-call marshalling is reported beside them
    def plain_python():
        for i, d in enumerate(dms):
            lf.lfem_assemble(d.handle, d.pattern, what, None, None, vals[2 * i], vals[2 * i + 1], None,
                             lf.LFEM_SCATTER_BLOCKED, stream)

    calls = [lf.prepare_assemble(d.handle, d.pattern, what, None, None, vals[2 * i], vals[2 * i + 1], None,
                                 lf.LFEM_SCATTER_BLOCKED, stream) for i, d in enumerate(dms)]

    def plain():
        for c in calls:
            c()

    b = lf.lfem_batch_create([d.handle for d in dms], [d.pattern for d in dms], what, 1)
    outs = lf.BatchOutputs(vals)

    def batched_python():
        lf.lfem_assemble_batch(b, vals, stream)

    def batched():
        lf.lfem_assemble_batch(b, outs, stream)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return statistics.median(t)

    t_plain = best(plain)   # per-mesh schedules as tuned by the batch
    t_batch = best(batched)
    t_plain_py = best(plain_python)
    t_batch_py = best(batched_python)
    T = sum(d.T for d in dms)
    res = {"meshes": len(dms), "elements": T, "nnz": sum(d.nnz for d in dms), "matrices": "M+A",
           "plain_ms": t_plain, "batched_ms": t_batch, "speedup": t_plain / t_batch,
           "batched_elements_per_s": T / (t_batch * 1e-3),
           "plain_ms_marshalled_per_call": t_plain_py, "batched_ms_marshalled_per_call": t_batch_py}
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()
    return res


def event_times(torch, fn, reps=20, warm=3):
    """HIP-event durations (ms) of fn on the current stream: (min, mean)."""
    stream = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = [a.elapsed_time(b) for a, b in ev]
    return min(t), statistics.mean(t)


def dd_bytes(d, domain, N, T, nnz):
    """Algorithmic bytes of an M + A assembly: coordinates, connectivity, two value arrays."""
    n_amb = d + 1 if domain == "surface" else d
    k = (d + 1) * (d + 2) // 2
    return n_amb * N * 8 + k * T * 4 + 2 * nnz * 8


def row_entry(name, ms, elements, alg_bytes, **extra):
    tmin, tmean = ms
    gbs = alg_bytes / (tmean * 1e-3) / 1e9
    return {"what": name, "ms_min": tmin, "ms_mean": tmean, "elements": elements,
            "elements_per_s": elements / (tmean * 1e-3), "alg_bytes": alg_bytes,
            "achieved_GBs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS, **extra}


def other_rows(lf, torch, meshgen, mesh2, dm2):
    """The other calls of the boundary on their workloads (HIP-event timing of
    the whole call, algorithmic bytes: every input read once, every output
    written once)."""
    import numpy as np
    rows = {}
    N, T = dm2.N, dm2.T
    # the bench workload under the other two scatter variants (FP64 atomics into
    # zeroed values, and the staged slot-sorted reduction)
    oc = {k: torch.empty(dm2.nnz, dtype=torch.float64, device="cuda") for k in ("M", "A")}
    for name, var in (("atomic", lf.LFEM_SCATTER_ATOMIC), ("staged", lf.LFEM_SCATTER_STAGED)):
        rows[f"{name}_c2"] = row_entry(
            f"M + A, P2 ellipsoid (655,360 elements), {name} scatter",
            event_times(torch, lambda: lf.lfem_assemble(dm2.handle, dm2.pattern, lf.LFEM_M | lf.LFEM_A, None, None,
                                                        oc["M"], oc["A"], None, var)),
            T, 3 * N * 8 + 6 * T * 4 + 2 * dm2.nnz * 8, scatter=name)
    del oc
    f = torch.as_tensor(mesh2["coef_c"], device="cuda")
    b = torch.empty(N, dtype=torch.float64, device="cuda")
    rows["load_c2"] = row_entry("load vector b = int f_h phi_j, P2 ellipsoid (655,360 elements)",
                                event_times(torch, lambda: lf.lfem_assemble_load(dm2.handle, f, b)), T,
                                3 * N * 8 + 6 * T * 4 + N * 8 + N * 8)
    X = mesh2["coords"]
    g = X / np.array([1.0, 0.64, 0.36])[:, None]
    nu = torch.as_tensor(g / np.linalg.norm(g, axis=0), device="cuda")
    fk = torch.empty(4, N, dtype=torch.float64, device="cuda")
    rows["kll_c2"] = row_entry("mean-curvature-flow non-linear terms f_1, f_2 (nu = nodal normals), P2 ellipsoid",
                               event_times(torch, lambda: lf.lfem_assemble_kll(dm2.handle, nu, f, fk)), T,
                               3 * N * 8 + 6 * T * 4 + 3 * N * 8 + N * 8 + 4 * N * 8)
    m5 = meshgen.config5()
    dm5 = lf.DeviceMesh.from_dict(m5)
    u = torch.as_tensor(m5["u"], device="cuda")
    v = torch.as_tensor(m5["v"], device="cuda")
    gr = torch.empty(3, dm5.N, dtype=torch.float64, device="cuda")
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    N5, T5 = dm5.N, dm5.T
    rows["shape_grad_c5"] = row_entry(
        "shape gradient of u^T A(x) u + v^T M(x) v, P2 displaced sphere (163,840 elements)",
        event_times(torch, lambda: lf.lfem_shape_grad(dm5.handle, u, u, 1.0, v, v, 1.0, gr)), T5,
        3 * N5 * 8 + 6 * T5 * 4 + 2 * N5 * 8 + 3 * N5 * 8)
    rows["energy_c5"] = row_entry(
        "matrix-free J(x) = u^T A(x) u + v^T M(x) v, same mesh",
        event_times(torch, lambda: lf.lfem_energy(dm5.handle, u, u, 1.0, v, v, 1.0, J)), T5,
        3 * N5 * 8 + 6 * T5 * 4 + 2 * N5 * 8 + 8)
    dm5.close()
    # one step of Dziuk's mean-curvature-flow scheme (M, A, S = M + tau A, rhs = M x) on a P2
    # sphere of the size of the paper's finest MCF meshes, eager and replayed from a HIP graph
    from meshgen import meshes as mg
    Vs, Fs = mg.sphere_nvb(9, order=2)
    Vs, Fs, _ = mg.sfc_reorder(Vs, Fs)
    cs, ks = mg.to_soa(Vs, Fs)
    dms = lf.DeviceMesh.from_dict(dict(domain="surface", dim=2, order=2, quad=6, coords=cs, conn=ks))
    so = dms.dziuk_system(1e-3)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dms.dziuk_system(1e-3, out=so)
    Ns, Ts, nnzs = dms.N, dms.T, dms.nnz
    # assembly: coordinates and connectivity in, M and A out; row pass: M, A, pattern, x in, S, rhs out
    bstep = (3 * Ns * 8 + 6 * Ts * 4 + 2 * nnzs * 8) + (2 * nnzs * 8 + (Ns + 1) * 4 + nnzs * 4 + 3 * Ns * 8
                                                      + nnzs * 8 + 3 * Ns * 8)
    rows["dziuk_step_eager"] = row_entry(
        f"Dziuk MCF step (M, A, S = M + tau A, rhs = M x), P2 sphere ({Ts} elements), one call",
        event_times(torch, lambda: dms.dziuk_system(1e-3, out=so)), Ts, bstep)
    rows["dziuk_step_graph"] = row_entry(
        f"the same step replayed from a captured HIP graph", event_times(torch, graph.replay), Ts, bstep)
    del graph
    # one step of the BDF algorithm of section 6.2 on the same sphere: M, A, the non-linear terms f
    # of nu~, H~, S = delta0 M + tau A and rhs = tau f - M hist for the four components of (nu; H)
    nus = torch.as_tensor(cs / np.linalg.norm(cs, axis=0), device="cuda")
    Hs = torch.full((Ns,), 2.0, dtype=torch.float64, device="cuda")
    hs = torch.as_tensor(np.random.default_rng(11).normal(size=(4, Ns)), device="cuda")
    ko = dms.kll_system(1e-3, 1.5, nus, Hs, hs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dms.kll_system(1e-3, 1.5, nus, Hs, hs, out=ko)
    # assembly as above; terms: coordinates, connectivity, nu, H in, f out; rows: M, A, pattern, hist,
    # f in, S and rhs out
    bkll = ((3 * Ns * 8 + 6 * Ts * 4 + 2 * nnzs * 8) + (3 * Ns * 8 + 6 * Ts * 4 + 4 * Ns * 8 + 4 * Ns * 8)
            + (2 * nnzs * 8 + (Ns + 1) * 4 + nnzs * 4 + 8 * Ns * 8 + nnzs * 8 + 4 * Ns * 8))
    rows["kll_step_eager"] = row_entry(
        f"BDF MCF step of section 6.2 (M, A, f, S = delta0 M + tau A, rhs = tau f - M hist), same sphere",
        event_times(torch, lambda: dms.kll_system(1e-3, 1.5, nus, Hs, hs, out=ko)), Ts, bkll)
    rows["kll_step_graph"] = row_entry(
        f"the same step replayed from a captured HIP graph", event_times(torch, graph.replay), Ts, bkll)
    del graph
    dms.close()
    # order sweep: M + A on spheres of order p = 1..4 with about the same number of nodes, default
    # rule and scatter of each order
    for p_ord, (kind, r) in {1: ("red", 8), 2: ("nvb", 14), 3: ("nvb", 13), 4: ("nvb", 12)}.items():
        V, F = mg.icosphere_red(r) if kind == "red" else mg.sphere_nvb(r)
        if p_ord == 2:
            V, F, _ = mg.p1_to_p2(V, F, mg.TRI_EDGES)
        elif p_ord > 2:
            V, F = mg.p1_to_pp(V, F, p_ord, mg.TRI_EDGES)
        V = mg.normalize_rows(V)
        V, F, _ = mg.sfc_reorder(V, F)  # locality order, as for the other workloads
        cp, kp = mg.to_soa(V, F)
        dmp = lf.DeviceMesh.from_dict(dict(domain="surface", dim=2, order=p_ord, quad=0, coords=cp, conn=kp))
        dmp.build_pattern()
        op = {k: torch.empty(dmp.nnz, dtype=torch.float64, device="cuda") for k in ("M", "A")}
        Np, Tp, nnzp = dmp.N, dmp.T, dmp.nnz
        ms = event_times(torch, lambda: lf.lfem_assemble(dmp.handle, dmp.pattern, lf.LFEM_M | lf.LFEM_A, None,
                                                         None, op["M"], op["A"], None, lf.LFEM_SCATTER_AUTO))
        info = lf.lfem_pattern_info(dmp.pattern)
        rows[f"order{p_ord}_sphere"] = row_entry(
            f"M + A on an order-{p_ord} sphere ({Tp} triangles, {Np} nodes)", ms, Tp,
            3 * Np * 8 + kp.shape[0] * Tp * 4 + 2 * nnzp * 8, nodes=Np, nnz=nnzp,
            nodes_per_s=Np / (ms[1] * 1e-3), scatter={1: "blocked", 2: "staged", 3: "atomic"}[info["scatter"]])
        dmp.close()
    # the paper's dimension analysis (section 6.4) compares P2 codes across dimensions, surface and
    # bulk: M + A for a P2 curve, sphere, square and cube at about 400k elements each (autotuned)
    dim_meshes = {
        "curve": ("surface", 1, lambda: mg.circle(393216, order=2)),
        "sphere": ("surface", 2, lambda: mg.sphere_nvb(14, order=2)),
        "square": ("bulk", 2, lambda: mg.square_tri(453, order=2)),
        "cube": ("bulk", 3, lambda: mg.kuhn_cube(40, order=2)[:2]),
    }
    for name, (dom, dd, make) in dim_meshes.items():
        V, F = make()
        V, F, _ = mg.sfc_reorder(V, F)
        cd, kd = mg.to_soa(V, F)
        dmd = lf.DeviceMesh.from_dict(dict(domain=dom, dim=dd, order=2, quad=0, coords=cd, conn=kd))
        dmd.build_pattern()
        variant = lf.lfem_pattern_autotune(dmd.handle, dmd.pattern, lf.LFEM_M | lf.LFEM_A)
        od = {k: torch.empty(dmd.nnz, dtype=torch.float64, device="cuda") for k in ("M", "A")}
        Nd, Td, nnzd = dmd.N, dmd.T, dmd.nnz
        ms = event_times(torch, lambda: lf.lfem_assemble(dmd.handle, dmd.pattern, lf.LFEM_M | lf.LFEM_A, None,
                                                         None, od["M"], od["A"], None, lf.LFEM_SCATTER_AUTO),
                         reps=10, warm=2)
        rows[f"p2_{name}"] = row_entry(
            f"P2 M + A, {dom} d={dd} ({name}, {Td} elements, {Nd} nodes)", ms, Td,
            dd_bytes(dd, dom, Nd, Td, nnzd), nodes=Nd, nnz=nnzd, ns_per_element=ms[1] * 1e6 / Td,
            scatter={1: "blocked", 2: "staged", 3: "atomic"}[variant])
        dmd.close()
    rows.update(tets_rows(lf, torch, meshgen))
    return rows


def tets_rows(lf, torch, meshgen, atomic=False):
    """P2 tetrahedra, M + A_a on the 64^3 Kuhn cube: 11-point rule (and the
    35-point degree-7 rule), each with its autotuned scatter; with `atomic`
    also the FP64-atomic scatter under the 11-point rule."""
    rows = {}
    m3 = meshgen.config3()
    dm3 = lf.DeviceMesh.from_dict(m3)
    dm3.build_pattern()
    ca = torch.as_tensor(m3["coef_a"], device="cuda")
    scatter = lf.lfem_pattern_autotune(dm3.handle, dm3.pattern, lf.LFEM_M | lf.LFEM_A)
    o3 = {k: torch.empty(dm3.nnz, dtype=torch.float64, device="cuda") for k in ("M", "A")}
    N3, T3, nnz3 = dm3.N, dm3.T, dm3.nnz
    rows["tets_c3"] = row_entry(
        "P2 tetrahedra M + A_a (a(x) nodal), unit cube 64^3 x 6 (1,572,864 elements), 11-point rule",
        event_times(torch, lambda: lf.lfem_assemble(dm3.handle, dm3.pattern, lf.LFEM_M | lf.LFEM_A, ca, None,
                                                    o3["M"], o3["A"], None, scatter), reps=5, warm=1),
        T3, 3 * N3 * 8 + 10 * T3 * 4 + N3 * 8 + 2 * nnz3 * 8,
        scatter={1: "blocked", 2: "staged", 3: "atomic"}.get(scatter, str(scatter)), nnz=nnz3)
    # FP64 flops per element of the local matrices: per point the Jacobian (10 nodes x 9 entries
    # FMA), cofactors, determinant and K = C^T C / det^2 (~120), the coefficient (10 FMA), then
    # per pair (55) one mass and six stiffness FMAs; 2 flops per FMA
    flops_e = 11 * (2 * 90 + 120 + 2 * 10 + 55 * 2 * 7)
    t3 = rows["tets_c3"]["ms_mean"] * 1e-3
    rows["tets_c3"].update({"flops_per_element": flops_e, "tflops": flops_e * T3 / t3 / 1e12,
                            "frac_fp64_peak": flops_e * T3 / t3 / 78.6e12})
    b3 = rows["tets_c3"]["alg_bytes"]
    rows["tets_c3"]["roofline"] = {
        "bound": "alu", "achieved": flops_e * T3 / t3 / 1e12, "peak": 78.6, "unit": "TFLOP/s",
        "frac": flops_e * T3 / t3 / 78.6e12, "traffic": None,
        "hbm_achieved_GBs": b3 / t3 / 1e9, "hbm_frac": b3 / t3 / 1e9 / HBM_PEAK_GBS,
        "alg_bytes_per_launch": b3, "flops_per_launch": flops_e * T3}
    dm3.close()
    # the same workload under the degree-7 tetrahedral rule (35 points), the degree the paper
    # integrates P2 tetrahedra with (section 5.2)
    dm7 = lf.DeviceMesh.from_dict(dict(m3, quad=35))
    dm7.build_pattern()
    scatter7 = lf.lfem_pattern_autotune(dm7.handle, dm7.pattern, lf.LFEM_M | lf.LFEM_A)
    rows["tets_c3_degree7"] = row_entry(
        "P2 tetrahedra M + A_a, the same mesh and coefficient, 35-point degree-7 rule",
        event_times(torch, lambda: lf.lfem_assemble(dm7.handle, dm7.pattern, lf.LFEM_M | lf.LFEM_A, ca, None,
                                                    o3["M"], o3["A"], None, scatter7), reps=5, warm=1),
        T3, 3 * N3 * 8 + 10 * T3 * 4 + N3 * 8 + 2 * nnz3 * 8,
        scatter={1: "blocked", 2: "staged", 3: "atomic"}.get(scatter7, str(scatter7)), nnz=nnz3)
    flops7 = 35 * (2 * 90 + 120 + 2 * 10 + 55 * 2 * 7)
    t7 = rows["tets_c3_degree7"]["ms_mean"] * 1e-3
    rows["tets_c3_degree7"].update({"flops_per_element": flops7, "tflops": flops7 * T3 / t7 / 1e12,
                                    "frac_fp64_peak": flops7 * T3 / t7 / 78.6e12})
    dm7.close()
    # orders 3 and 4 on tetrahedra (one wave per element, staged reduction): M + A on Kuhn cubes of
    # about 250k nodes, 35-point rule
    from meshgen import meshes as mg
    for p_ord, n_c in ((3, 20), (4, 16)):
        V, F, _ = mg.kuhn_cube(n_c, order=1)
        V, F = mg.p1_to_pp(V, F, p_ord, mg.TET_EDGES)
        V, F, _ = mg.sfc_reorder(V, F)
        cp, kp = mg.to_soa(V, F)
        dmp = lf.DeviceMesh.from_dict(dict(domain="bulk", dim=3, order=p_ord, quad=35, coords=cp, conn=kp))
        dmp.build_pattern()
        op = {k: torch.empty(dmp.nnz, dtype=torch.float64, device="cuda") for k in ("M", "A")}
        Np, Tp, nnzp = dmp.N, dmp.T, dmp.nnz
        ms = event_times(torch, lambda: lf.lfem_assemble(dmp.handle, dmp.pattern, lf.LFEM_M | lf.LFEM_A, None,
                                                         None, op["M"], op["A"], None, lf.LFEM_SCATTER_AUTO),
                         reps=5, warm=1)
        rows[f"tets_order{p_ord}"] = row_entry(
            f"M + A on order-{p_ord} tetrahedra, Kuhn cube {n_c}^3 x 6 ({Tp} elements, {Np} nodes), 35-point rule",
            ms, Tp, 3 * Np * 8 + kp.shape[0] * Tp * 4 + 2 * nnzp * 8, nodes=Np, nnz=nnzp,
            nodes_per_s=Np / (ms[1] * 1e-3), scatter="staged")
        del op
        dmp.close()
    if atomic:
        dma = lf.DeviceMesh.from_dict(m3)
        dma.build_pattern()
        rows["tets_c3_atomic"] = row_entry(
            "P2 tetrahedra M + A_a, 11-point rule, FP64-atomic scatter",
            event_times(torch, lambda: lf.lfem_assemble(dma.handle, dma.pattern, lf.LFEM_M | lf.LFEM_A, ca, None,
                                                        o3["M"], o3["A"], None, lf.LFEM_SCATTER_ATOMIC),
                        reps=5, warm=1),
            T3, 3 * N3 * 8 + 10 * T3 * 4 + N3 * 8 + 2 * nnz3 * 8, scatter="atomic", nnz=nnz3)
        dma.close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scatter", default="blocked", choices=["blocked", "staged", "atomic"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the load / non-linear terms / shape gradient / tetrahedra measurements")
    ap.add_argument("--only-tets", action="store_true",
                    help="run only the P2 tetrahedra rows (64^3 Kuhn cube) and print them as one JSON "
                         "line (for profiling that workload alone)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a 256 MiB device copy 3 times (a kernel of known traffic that "
                         "calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the assembly would shard by "
              "node ranges without communication, but no multi-GPU path is implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    import paper_2605_14035_amd as lf

    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_tets:
        print(json.dumps({"rows": tets_rows(lf, torch, meshgen, atomic=True)}))
        return
    t0 = time.perf_counter()
    mesh = meshgen.config2()
    gen_s = time.perf_counter() - t0
    print(f"[bench] workload generated in {gen_s:.1f} s", file=sys.stderr, flush=True)
    dm = lf.DeviceMesh.from_dict(mesh)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dm.build_pattern()
    torch.cuda.synchronize()
    pattern_s = time.perf_counter() - t0
    N, T, nnz = dm.N, dm.T, dm.nnz
    scatter = {"blocked": lf.LFEM_SCATTER_BLOCKED, "staged": lf.LFEM_SCATTER_STAGED,
               "atomic": lf.LFEM_SCATTER_ATOMIC}[args.scatter]
    out = {"M": torch.empty(nnz, dtype=torch.float64, device="cuda"),
           "A": torch.empty(nnz, dtype=torch.float64, device="cuda")}
    what = lf.LFEM_M | lf.LFEM_A
    stream = torch.cuda.current_stream()

    def step():
        lf.lfem_assemble(dm.handle, dm.pattern, what, None, None, out["M"], out["A"], None,
                         scatter, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed region: K launches back to back on the launch stream, one HIP
    # event pair around all of them (an event pair per launch would put a
    # timestamp packet between consecutive launches)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_start.record(stream)
    for _ in range(args.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = t_start.elapsed_time(t_end) / args.steps
    # the spread of single launches, each between its own event pair (outside
    # the timed region)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ev_sorted = sorted(ev_ms)
    kern_p90 = ev_sorted[min(len(ev_sorted) - 1, int(0.9 * len(ev_sorted)))]
    # the 241 MB of values nearly fit the 256 MB last-level cache: time the
    # same launch with a 512 MB read-modify-write scrub between launches too
    scrub = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    scrubbed = []
    for _ in range(20):
        scrub.mul_(1.0)
        a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_ev.record(stream)
        step()
        b_ev.record(stream)
        torch.cuda.synchronize()
        scrubbed.append(a_ev.elapsed_time(b_ev))
    scrub_ms = statistics.median(scrubbed)
    # practical ceiling: a plain device copy of 256 MiB (read + write), median of 10
    dst = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    src = scrub[:dst.numel()]
    copies = []
    for _ in range(10):
        a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_ev.record(stream)
        dst.copy_(src)
        b_ev.record(stream)
        torch.cuda.synchronize()
        copies.append(a_ev.elapsed_time(b_ev))
    copy_gbs = 2 * dst.numel() * 8 / (statistics.median(copies) * 1e-3) / 1e9
    # and a write-only stream of the same size (84 % of the c2 bytes are writes)
    fills = []
    for _ in range(10):
        a_ev, b_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a_ev.record(stream)
        dst.fill_(1.0)
        b_ev.record(stream)
        torch.cuda.synchronize()
        fills.append(a_ev.elapsed_time(b_ev))
    fill_gbs = dst.numel() * 8 / (statistics.median(fills) * 1e-3) / 1e9
    del scrub, dst, src
    ms_per_step = wall * 1e3 / args.steps
    value = T / (ms_per_step * 1e-3)

    # algorithmic bytes per launch: read coords and connectivity once, write each value once
    b_alg = 3 * N * 8 + 6 * T * 4 + 2 * nnz * 8
    achieved = b_alg / (kern_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    traffic = read_traffic(digest) if args.scatter == "blocked" else None

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "P2 isoparametric surface FE on the ellipsoid x^2+y^2/0.64+z^2/0.36=1, "
                        "icosahedron + 15 newest-vertex bisections, 6-point degree-4 rule, "
                        "mass + Laplace-Beltrami stiffness into a prebuilt CSR pattern",
            "elements": T, "nodes": N, "nnz": nnz, "matrices": "M+A", "quad_points": 6,
            "scatter": args.scatter, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": KERNEL_NAME, "alg_bytes_per_launch": b_alg,
            "kernel_ms_mean": kern_ms, "kernel_ms_mean_single_launch": statistics.mean(ev_ms),
            "kernel_ms_min": min(ev_ms),
            "kernel_ms_median": statistics.median(ev_ms), "kernel_ms_p90": kern_p90,
            "kernel_ms_median_after_512MB_scrub": scrub_ms,
            "frac_after_512MB_scrub": b_alg / (scrub_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "copy_256MiB_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
            "write_256MiB_GBs": fill_gbs, "frac_of_write": achieved / fill_gbs,
            "kernel_source_digest": digest,
        },
        "pattern_build_s": pattern_s,
    }
    if not args.no_rows:
        print("[bench] other rows (load, non-linear terms, shape gradient, MCF steps, orders 1-4, tetrahedra)",
              file=sys.stderr, flush=True)
        result["rows"] = other_rows(lf, torch, meshgen, mesh, dm)
    dm.close()
    if not args.no_batch:
        print("[bench] batched vs plain (256 meshes)", file=sys.stderr, flush=True)
        result["batched_vs_plain"] = batched_vs_plain(lf, torch, meshgen)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(mesh)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
