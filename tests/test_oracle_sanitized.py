"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
stand-alone build of its C source with a small driver runs every entry point
(matrices with and without coefficients, the numeric-only path, energy, shape
gradient, load vector, mean-curvature-flow terms) on small meshes of every
element type and order; no sanitizer finding is allowed, and the outputs equal
those of the ordinary build bitwise (the same C, no reassociation and no
fused multiply-adds in either build)."""

import os
import subprocess

import numpy as np
import pytest

import meshgen
import oracle
from gpu_util import order_mesh
from oracle import quadrature


@pytest.fixture(scope="module")
def exe():
    path = os.path.join(os.path.dirname(oracle.__file__), "oracle_sanitized")
    if not os.path.exists(path):
        oracle.build_sanitized()
    return path


CASES = [("small", t) for t in meshgen.ALL_TYPES] + \
        [("order", (dom, d, p)) for (dom, d) in (("surface", 1), ("surface", 2), ("bulk", 2), ("bulk", 3))
         for p in (3, 4)]


def write_input(path, m, rng):
    surface = 1 if m["domain"] == "surface" else 0
    d, p = int(m["dim"]), int(m["order"])
    qp, qw = quadrature.rule(d, int(m["quad"]))
    coords = np.ascontiguousarray(m["coords"], dtype=np.float64)
    conn = np.ascontiguousarray(m["conn"], dtype=np.int32)
    n_amb, N = coords.shape
    vecs = {name: rng.uniform(-1.0, 1.0, size=N) for name in ("u", "v", "w", "z", "H")}
    coef = rng.uniform(0.5, 2.0, size=N)
    nu = rng.uniform(-1.0, 1.0, size=(n_amb, N))
    with open(path, "wb") as f:
        np.array([surface, d, p, len(qw), N, conn.shape[1]], dtype=np.int64).tofile(f)
        for a in (np.asarray(qp, dtype=np.float64), np.asarray(qw, dtype=np.float64), coords):
            a.tofile(f)
        conn.tofile(f)
        for a in (coef, vecs["u"], vecs["v"], vecs["w"], vecs["z"], nu, vecs["H"]):
            np.ascontiguousarray(a, dtype=np.float64).tofile(f)
    return coef, vecs, nu


@pytest.mark.parametrize("src,t", CASES)
def test_sanitized_oracle(exe, tmp_path, src, t):
    m = meshgen.small_mesh(*t, size=2) if src == "small" else order_mesh(*t)
    rng = np.random.default_rng(11)
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    coef, vecs, nu = write_input(inp, m, rng)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    r = subprocess.run([exe, str(inp), str(outp)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    got = np.fromfile(outp, dtype=np.float64)
    # the same quantities from the ordinary build
    pos = 0
    for kind, c in (("mass", None), ("stiffness", None), ("mass", coef), ("stiffness", coef)):
        rp, ci, ref = oracle.assemble(m, kind, coef=c)
        n = int(got[pos])
        assert n == len(ref)
        assert np.array_equal(got[pos + 1:pos + 1 + n], ref), (kind, c is not None)
        pos += 1 + n
    n = len(ref)
    assert np.array_equal(got[pos:pos + n], oracle.assemble_numeric(m, "stiffness", (rp, ci), coef=coef))
    pos += n
    J = oracle.energy(m, vecs["u"], vecs["v"], 1.0, vecs["w"], vecs["z"], 0.5)
    assert got[pos] == J
    pos += 1
    g = oracle.shape_grad(m, vecs["u"], vecs["v"], 1.0, vecs["w"], vecs["z"], 0.5).ravel()
    assert np.array_equal(got[pos:pos + g.size], g)
    pos += g.size
    b = oracle.load(m, coef)
    assert np.array_equal(got[pos:pos + b.size], b)
    pos += b.size
    f = oracle.kll(m, nu, vecs["H"]).ravel()
    assert np.array_equal(got[pos:pos + f.size], f)
    pos += f.size
    assert pos == got.size
