"""CPU FP64 oracle for isoparametric P1/P2 finite-element assembly.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library ``paper_2605_14035_amd``; the two only read the
same seeded meshes from ``meshgen``.

The arithmetic lives in ``lfem_oracle.c`` (a plain element loop in the order
of the paper's Listing 1) and ``quadrature.py`` (rules solved from their
moment equations).  This module only marshals NumPy arrays through ctypes.

Every function takes a mesh dict as produced by ``meshgen`` (keys
``domain``, ``dim``, ``order``, ``quad``, ``coords`` (n_amb, N) float64,
``conn`` (k, T) int32).
"""

from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

from . import quadrature

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lfem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source in 80-bit long double: finite-difference reference only
_LIB_LD = os.path.join(_HERE, "liboracle_ld.so")

OK, EINVAL, ENOMEM, EDEGENERATE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3 for the baseline x86-64 target, so no
    fused multiply-adds and no reassociation; no vendor libraries), plus the
    long-double build used as a finite-difference reference and the
    sanitizer build of its driver."""
    for path, extra in ((_LIB, []), (_LIB_LD, ["-DORACLE_LONG_DOUBLE"])):
        if force or not os.path.exists(path):
            _compile(path, extra)
    if force or not os.path.exists(_SAN_EXE):
        build_sanitized()
    return _LIB


_DRIVER = os.path.join(_HERE, "sanitize_driver.c")
_SAN_EXE = os.path.join(_HERE, "oracle_sanitized")


def build_sanitized() -> str:
    """The oracle and its stand-alone driver (sanitize_driver.c) compiled with
    AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc), every
    finding fatal; returns the executable's path."""
    tmp = _SAN_EXE + ".tmp"
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", tmp, _DRIVER, _SRC, "-lm"], check=True)
    os.replace(tmp, _SAN_EXE)
    return _SAN_EXE


def _compile(path, extra):
    tmp = path + ".tmp"
    subprocess.run(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", *extra, "-o", tmp, _SRC, "-lm"],
                   check=True)
    os.replace(tmp, path)


@contextlib.contextmanager
def planted(define: str):
    """Test hook: while active, every oracle call (double build) runs a build of
    lfem_oracle.c with -D<define>, a mistake planted on purpose, so that a test
    can show that a pin fails on it.  Built into a temporary directory."""
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, f"liboracle_{define}.so")
        _compile(path, [f"-D{define}"])
        saved = _libs.pop(False, None)
        try:
            _libs[False] = _declare(C.CDLL(path))
            yield
        finally:
            _libs.pop(False, None)
            if saved is not None:
                _libs[False] = saved


_libs = {}


def lib(long_double: bool = False):
    key = bool(long_double)
    if key not in _libs:
        path = _LIB_LD if key else _LIB
        if not os.path.exists(path):
            build(force=False)
        _libs[key] = _declare(C.CDLL(path))
    return _libs[key]


def _declare(L):
    """Argument and return types of the oracle's C functions."""
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lp = C.POINTER(C.c_int64)
    up = C.POINTER(C.c_uint8)
    i64 = C.c_int64
    ci = C.c_int
    L.oracle_basis.argtypes = [ci, ci, dp, dp, dp]
    L.oracle_element_matrices.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, ci,
                                          i64, i64, dp]
    L.oracle_assemble.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, ci, up, i64,
                                  lp, ip, dp, lp]
    L.oracle_energy.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, dp, C.c_double,
                                dp, dp, C.c_double, dp]
    L.oracle_shape_grad.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, dp,
                                    C.c_double, dp, dp, C.c_double, dp]
    L.oracle_load.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, dp]
    L.oracle_kll.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, dp, dp]
    L.oracle_assemble_numeric.argtypes = [ci, ci, ci, ci, dp, dp, i64, dp, i64, ip, dp, ci, lp, ip,
                                          dp]
    for f in (L.oracle_basis, L.oracle_element_matrices, L.oracle_assemble,
              L.oracle_energy, L.oracle_shape_grad, L.oracle_load, L.oracle_kll,
              L.oracle_assemble_numeric):
        f.restype = ci
    return L


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _mesh_args(mesh, qp=None, qw=None):
    surface = 1 if mesh["domain"] == "surface" else 0
    d, p = int(mesh["dim"]), int(mesh["order"])
    if qp is None:
        qp, qw = quadrature.rule(d, int(mesh["quad"]))
    qp = np.ascontiguousarray(qp, dtype=np.float64)
    qw = np.ascontiguousarray(qw, dtype=np.float64)
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    conn = np.ascontiguousarray(mesh["conn"], dtype=np.int32)
    N = coords.shape[1]
    T = conn.shape[1]
    keep = (qp, qw, coords, conn)
    args = [surface, d, p, len(qw), _ptr(qp, C.c_double), _ptr(qw, C.c_double), N,
            _ptr(coords, C.c_double), T, _ptr(conn, C.c_int32)]
    return args, keep, N, T, conn.shape[0]


def _check(st, what):
    if st == EDEGENERATE:
        raise FloatingPointError(f"{what}: degenerate element (measure not positive/finite)")
    if st != OK:
        raise RuntimeError(f"{what}: oracle status {st}")


def basis(d: int, p: int, xi):
    """Values (k,) and reference gradients (k, d) of the nodal basis at xi."""
    xi = np.ascontiguousarray(np.atleast_1d(xi), dtype=np.float64)
    k = lib().oracle_nodes_per_element(d, p)
    if k < 0:
        raise ValueError(f"no nodal basis of order {p} in dimension {d}")
    phi = np.zeros(k)
    dphi = np.zeros((k, d))
    _check(lib().oracle_basis(d, p, _ptr(xi, C.c_double), _ptr(phi, C.c_double),
                              _ptr(dphi, C.c_double)), "basis")
    return phi, dphi


KIND = {"mass": 0, "stiffness": 1}


def element_matrices(mesh, kind: str, coef=None, e0: int = 0, e1=None, rule=None):
    """Local k x k matrices of elements e0..e1-1 (mass or stiffness)."""
    args, keep, N, T, k = _mesh_args(mesh, *(rule or (None, None)))
    e1 = T if e1 is None else e1
    coef = _f64(coef)
    out = np.zeros((e1 - e0, k, k))
    st = lib().oracle_element_matrices(*args, _ptr(coef, C.c_double), KIND[kind], e0, e1,
                                       _ptr(out, C.c_double))
    _check(st, "element_matrices")
    return out


def assemble(mesh, kind: str, coef=None, rows=None, rule=None):
    """Global CSR (row_ptr int64 (N+1,), col_idx int32, vals float64).

    ``rows``: optional iterable of row ids; only those rows are assembled
    (all other rows come out empty)."""
    args, keep, N, T, k = _mesh_args(mesh, *(rule or (None, None)))
    conn = keep[3]
    coef = _f64(coef)
    mask = None
    if rows is not None:
        mask = np.zeros(N, dtype=np.uint8)
        mask[np.asarray(rows, dtype=np.int64)] = 1
        cap = int(mask[conn].sum()) * k
    else:
        cap = k * k * T
    cap = max(cap, 1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    col_idx = np.zeros(cap, dtype=np.int32)
    vals = np.zeros(cap, dtype=np.float64)
    nnz = np.zeros(1, dtype=np.int64)
    st = lib().oracle_assemble(*args, _ptr(coef, C.c_double), KIND[kind],
                               _ptr(mask, C.c_uint8), cap, _ptr(row_ptr, C.c_int64),
                               _ptr(col_idx, C.c_int32), _ptr(vals, C.c_double),
                               _ptr(nnz, C.c_int64))
    _check(st, "assemble")
    n = int(nnz[0])
    return row_ptr, col_idx[:n].copy(), vals[:n].copy()


def assemble_numeric(mesh, kind: str, pattern, coef=None, rule=None):
    """Values of the global matrix in a prebuilt CSR pattern (row_ptr, col_idx)
    of the same element array: element loop with the slot of each local entry
    found by binary search in its row (no COO, no sort)."""
    args, keep, N, T, k = _mesh_args(mesh, *(rule or (None, None)))
    row_ptr = np.ascontiguousarray(pattern[0], dtype=np.int64)
    col_idx = np.ascontiguousarray(pattern[1], dtype=np.int32)
    coef = _f64(coef)
    vals = np.zeros(max(int(row_ptr[-1]), 1))
    st = lib().oracle_assemble_numeric(*args, _ptr(coef, C.c_double), KIND[kind], _ptr(row_ptr, C.c_int64),
                                       _ptr(col_idx, C.c_int32), _ptr(vals, C.c_double))
    _check(st, "assemble_numeric")
    return vals[:int(row_ptr[-1])]


def energy(mesh, u, v, alpha=1.0, w=None, z=None, beta=1.0, long_double=False):
    """alpha u^T A v + beta w^T M z.  ``long_double`` evaluates it with the
    80-bit build (finite-difference reference)."""
    args, keep, N, T, k = _mesh_args(mesh)
    u, v, w, z = _f64(u), _f64(v), _f64(w), _f64(z)
    out = np.zeros(1)
    st = lib(long_double).oracle_energy(*args, _ptr(u, C.c_double), _ptr(v, C.c_double), float(alpha),
                             _ptr(w, C.c_double), _ptr(z, C.c_double), float(beta),
                             _ptr(out, C.c_double))
    _check(st, "energy")
    return float(out[0])


def load(mesh, f=None, rule=None, long_double=False):
    """Load vector b_j = sum_E sum_q w mu f_h phi_j, (N,); f: nodal values or
    None for f = 1."""
    args, keep, N, T, k = _mesh_args(mesh, *(rule or (None, None)))
    f = _f64(f)
    b = np.zeros(N)
    st = lib(long_double).oracle_load(*args, _ptr(f, C.c_double), _ptr(b, C.c_double))
    _check(st, "load")
    return b


def kll(mesh, nu, H=None, rule=None):
    """Non-linear terms of the mean-curvature-flow example (section 6.2):
    alpha^2 = |grad_Gamma_h nu_h|^2 (Frobenius), f_1[c] = int alpha^2 (nu_h)_c phi_j,
    f_2 = int alpha^2 H_h phi_j.  nu: (n_amb, N) nodal vector field, H: (N,) or
    None for 1.  Returns an (n_amb + 1, N) array: rows f_1 components, then f_2."""
    args, keep, N, T, k = _mesh_args(mesh, *(rule or (None, None)))
    n_amb = keep[2].shape[0]
    nu = _f64(np.asarray(nu).reshape(n_amb, N))
    H = _f64(H)
    f = np.zeros((n_amb + 1, N))
    st = lib().oracle_kll(*args, _ptr(nu, C.c_double), _ptr(H, C.c_double), _ptr(f, C.c_double))
    _check(st, "kll")
    return f


def kll_system(mesh, tau, delta0, nu, H, hist=None):
    """Per-step linear system of the mean-curvature-flow algorithm of section
    6.2 (evolving-surface finite elements with linearly implicit BDF): with
    u = (nu; H) in R^{(n_amb + 1) N} and the BDF derivative
    u_dot^n = (1/tau) sum_{j>=0} delta_j u^{n-j}, the equation
    M u_dot^n + A u^n = f(x~, u~) at the extrapolated surface x~ (the mesh's
    coordinates) and extrapolated u~ = (nu; H) reads
        (delta_0 M + tau A) u^n = tau f - M sum_{j>=1} delta_j u^{n-j},
    the same S for every component.  hist: the history term
    sum_{j>=1} delta_j u^{n-j} as an (n_amb + 1, N) array (None: zero).
    Returns (S as CSR (row_ptr, col_idx, vals) on the pattern of M, f, rhs)."""
    Mrp, Mci, Mv = assemble(mesh, "mass")
    Arp, Aci, Av = assemble(mesh, "stiffness")
    if not (np.array_equal(Mrp, Arp) and np.array_equal(Mci, Aci)):
        raise RuntimeError("mass and stiffness patterns differ")
    f = kll(mesh, nu, H)
    rhs = tau * f
    if hist is not None:
        N = len(Mrp) - 1
        M = to_scipy(N, (Mrp, Mci, Mv))
        hist = np.asarray(hist, dtype=np.float64).reshape(f.shape)
        rhs = rhs - np.stack([M @ hist[c] for c in range(f.shape[0])])
    return (Mrp, Mci, delta0 * Mv + tau * Av), f, rhs


def shape_grad(mesh, u, v, alpha=1.0, w=None, z=None, beta=1.0):
    """d/dx [alpha u^T A(x) v + beta w^T M(x) z] as an (n_amb, N) array."""
    args, keep, N, T, k = _mesh_args(mesh)
    n_amb = keep[2].shape[0]
    u, v, w, z = _f64(u), _f64(v), _f64(w), _f64(z)
    g = np.zeros((n_amb, N))
    st = lib().oracle_shape_grad(*args, _ptr(u, C.c_double), _ptr(v, C.c_double), float(alpha),
                                 _ptr(w, C.c_double), _ptr(z, C.c_double), float(beta),
                                 _ptr(g, C.c_double))
    _check(st, "shape_grad")
    return g


def to_scipy(N, csr):
    import scipy.sparse as sp
    row_ptr, col_idx, vals = csr
    return sp.csr_matrix((vals, col_idx, row_ptr), shape=(N, N))
