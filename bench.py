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
    return {"value": T / t, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"whole workload ({T} elements, M and A, COO + stable sort + CSR), "
                      f"median of 3 runs: {t:.2f} s"}


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

    def plain():
        for i, d in enumerate(dms):
            lf.lfem_assemble(d.handle, d.pattern, what, None, None, vals[2 * i], vals[2 * i + 1], None,
                             lf.LFEM_SCATTER_BLOCKED, stream)

    b = lf.lfem_batch_create([d.handle for d in dms], [d.pattern for d in dms], what, 1)

    def batched():
        lf.lfem_assemble_batch(b, vals, stream)

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
    T = sum(d.T for d in dms)
    res = {"meshes": len(dms), "elements": T, "nnz": sum(d.nnz for d in dms), "matrices": "M+A",
           "plain_ms": t_plain, "batched_ms": t_batch, "speedup": t_plain / t_batch,
           "batched_elements_per_s": T / (t_batch * 1e-3)}
    lf.lfem_batch_destroy(b)
    for d in dms:
        d.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scatter", default="blocked", choices=["blocked", "staged", "atomic"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a 256 MiB device copy 3 times (a kernel of known traffic that "
                         "calibrates hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); multi-GPU runs are "
              "not part of this build", file=sys.stderr)
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
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kern_ms = statistics.mean(ev_ms)
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
            "kernel_ms_mean": kern_ms, "kernel_ms_min": min(ev_ms),
            "kernel_source_digest": digest,
        },
        "pattern_build_s": pattern_s,
    }
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
