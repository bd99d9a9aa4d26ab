"""MI355X-native isoparametric finite-element assembly (liblfem.so binding).

The functions below carry the names of the C ABI in ``include/lfem.h`` and
only marshal arguments: PyTorch tensors (device memory, FP64 / int32,
contiguous) are passed as raw device pointers, the current PyTorch stream as
the HIP stream, and a non-OK status becomes ``LfemError``.  Every step of the
computation runs in the library's HIP kernels; importing this package
without a built ``liblfem.so`` raises.
"""

from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import (LFEM_A, LFEM_BULK, LFEM_EDEGENERATE, LFEM_EHIP, LFEM_EINVAL, LFEM_ENOMEM,
                   LFEM_ERANGE, LFEM_EUNSUPPORTED, LFEM_M, LFEM_MC, LFEM_OK, LFEM_SCATTER_ATOMIC,
                   LFEM_SCATTER_AUTO, LFEM_SCATTER_BLOCKED, LFEM_SCATTER_STAGED, LFEM_SURFACE,
                   LFEM_TUNE_ALLOW_ATOMIC, LFEM_TUNE_NO_CACHE, LfemError)

_L = _lib.load()

__all__ = [
    "LFEM_A", "LFEM_BULK", "LFEM_M", "LFEM_MC", "LFEM_SCATTER_ATOMIC", "LFEM_SCATTER_AUTO",
    "LFEM_OK", "LFEM_EINVAL", "LFEM_ENOMEM", "LFEM_EHIP", "LFEM_ERANGE", "LFEM_EDEGENERATE",
    "LFEM_EUNSUPPORTED",
    "LFEM_SCATTER_BLOCKED", "LFEM_SCATTER_STAGED", "LFEM_SURFACE", "LFEM_TUNE_ALLOW_ATOMIC",
    "LFEM_TUNE_NO_CACHE", "LfemError",
    "lfem_mesh_create", "lfem_mesh_set_coords", "lfem_pattern_build", "lfem_pattern_get",
    "lfem_pattern_info", "lfem_assemble", "lfem_assemble_mass", "lfem_assemble_stiffness", "lfem_assemble_weighted",
    "lfem_pattern_autotune", "lfem_pattern_autotune_ex", "lfem_tune_cache_clear", "lfem_pattern_schedule", "lfem_batch_create", "lfem_batch_create_ex", "lfem_assemble_batch", "lfem_shape_grad",
    "lfem_shape_grad_noalloc", "lfem_energy", "lfem_assemble_load", "lfem_assemble_kll", "lfem_spmv", "lfem_dziuk_system", "lfem_kll_system", "lfem_reference_table", "lfem_status_get", "lfem_status_reset", "lfem_last_error", "lfem_version", "lfem_set_debug",
    "lfem_mesh_destroy", "lfem_pattern_destroy", "lfem_batch_destroy", "copy_from_device", "BatchOutputs",
    "prepare_assemble",
    "library_path",
]


def library_path() -> str:
    return _lib.LIB_PATH


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live in device memory")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def lfem_mesh_create(domain: int, dim: int, order: int, coords: torch.Tensor, conn: torch.Tensor,
                     quad_points: int = 0, stream=None) -> C.c_void_p:
    """coords: float64 (n_amb, N); conn: int32 (k, T).  Both must outlive the mesh."""
    out = C.c_void_p()
    N = coords.shape[1] if coords.dim() == 2 else 0
    T = conn.shape[1] if conn.dim() == 2 else 0
    st = _L.lfem_mesh_create(int(domain), int(dim), int(order), N,
                             _ptr(coords, torch.float64, "coords"), T,
                             _ptr(conn, torch.int32, "conn"), int(quad_points), _stream(stream),
                             C.byref(out))
    _lib.check(st, "lfem_mesh_create")
    return out


def lfem_mesh_set_coords(mesh, coords: torch.Tensor):
    _lib.check(_L.lfem_mesh_set_coords(mesh, _ptr(coords, torch.float64, "coords")),
               "lfem_mesh_set_coords")


def lfem_pattern_build(mesh, stream=None) -> C.c_void_p:
    out = C.c_void_p()
    _lib.check(_L.lfem_pattern_build(mesh, _stream(stream), C.byref(out)), "lfem_pattern_build")
    return out


def lfem_pattern_get(pattern):
    """(n_rows, nnz, row_ptr device address, col_idx device address)."""
    n, nnz = C.c_int64(), C.c_int64()
    rp, ci = C.c_void_p(), C.c_void_p()
    _lib.check(_L.lfem_pattern_get(pattern, C.byref(n), C.byref(nnz), C.byref(rp), C.byref(ci)),
               "lfem_pattern_get")
    return n.value, nnz.value, rp.value, ci.value


def lfem_pattern_info(pattern) -> dict:
    info = _lib.PatternInfo()
    _lib.check(_L.lfem_pattern_info(pattern, C.byref(info)), "lfem_pattern_info")
    return {name: getattr(info, name) for name, _ in _lib.PatternInfo._fields_}


_hip = None


def copy_from_device(dst: torch.Tensor, src_address: int, nbytes: int):
    """Device-to-device copy of library-owned memory into a torch tensor."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    if nbytes == 0:
        return dst
    assert dst.is_cuda and dst.is_contiguous() and dst.numel() * dst.element_size() >= nbytes
    torch.cuda.current_stream().synchronize()
    st = _hip.hipMemcpy(C.c_void_p(dst.data_ptr()), C.c_void_p(src_address), nbytes, 3)
    if st != 0:
        raise RuntimeError(f"hipMemcpy failed: {st}")
    return dst


def lfem_assemble(mesh, pattern, what: int, coef_a=None, coef_c=None, vals_m=None, vals_a=None,
                  vals_mc=None, scatter: int = LFEM_SCATTER_AUTO, stream=None):
    st = _L.lfem_assemble(mesh, pattern, int(what), _ptr(coef_a, torch.float64, "coef_a"),
                          _ptr(coef_c, torch.float64, "coef_c"),
                          _ptr(vals_m, torch.float64, "vals_m"),
                          _ptr(vals_a, torch.float64, "vals_a"),
                          _ptr(vals_mc, torch.float64, "vals_mc"), int(scatter), _stream(stream))
    _lib.check(st, "lfem_assemble")


def lfem_assemble_mass(mesh, pattern, vals, stream=None):
    _lib.check(_L.lfem_assemble_mass(mesh, pattern, _ptr(vals, torch.float64, "vals"),
                                     _stream(stream)), "lfem_assemble_mass")


def lfem_assemble_stiffness(mesh, pattern, coef, vals, stream=None):
    _lib.check(_L.lfem_assemble_stiffness(mesh, pattern, _ptr(coef, torch.float64, "coef"),
                                          _ptr(vals, torch.float64, "vals"), _stream(stream)),
               "lfem_assemble_stiffness")


def lfem_assemble_weighted(mesh, pattern, coef, vals, stream=None):
    _lib.check(_L.lfem_assemble_weighted(mesh, pattern, _ptr(coef, torch.float64, "coef"),
                                         _ptr(vals, torch.float64, "vals"), _stream(stream)),
               "lfem_assemble_weighted")


def lfem_pattern_autotune(mesh, pattern, what: int, stream=None) -> int:
    v = C.c_int()
    _lib.check(_L.lfem_pattern_autotune(mesh, pattern, int(what), _stream(stream), C.byref(v)),
               "lfem_pattern_autotune")
    return v.value


def lfem_set_debug(on: bool) -> bool:
    """Turn the library's debug bounds checks on or off; returns the previous
    setting."""
    return bool(_L.lfem_set_debug(1 if on else 0))


def lfem_pattern_autotune_ex(mesh, pattern, what: int, flags: int = 0, stream=None):
    """Returns (variant, block_cap)."""
    v, cap = C.c_int(), C.c_int()
    _lib.check(_L.lfem_pattern_autotune_ex(mesh, pattern, int(what), int(flags), _stream(stream), C.byref(v),
                                           C.byref(cap)), "lfem_pattern_autotune_ex")
    return v.value, cap.value


def lfem_tune_cache_clear():
    _L.lfem_tune_cache_clear()


def lfem_pattern_schedule(mesh, pattern, variant: int, block_cap: int = 0, stream=None):
    _lib.check(_L.lfem_pattern_schedule(mesh, pattern, int(variant), int(block_cap), _stream(stream)),
               "lfem_pattern_schedule")


def lfem_batch_create(meshes, patterns, what: int, autotune: int = 0, stream=None):
    n = len(meshes)
    ms = (C.c_void_p * n)(*[m.value for m in meshes])
    ps = (C.c_void_p * n)(*[p.value for p in patterns])
    out = C.c_void_p()
    _lib.check(_L.lfem_batch_create(n, ms, ps, int(what), int(autotune), _stream(stream),
                                    C.byref(out)), "lfem_batch_create")
    return out


def lfem_batch_create_ex(meshes, patterns, what: int, coef_a=None, coef_c=None, autotune: int = 0,
                         stream=None):
    """coef_a / coef_c: None or a list (one entry per mesh) of float64 device
    tensors (N_i,) or None; the batch keeps their pointers, so the caller keeps
    the tensors alive for the batch's lifetime."""
    n = len(meshes)
    ms = (C.c_void_p * n)(*[m.value for m in meshes])
    ps = (C.c_void_p * n)(*[p.value for p in patterns])

    def arr(cs, name):
        if cs is None:
            return None
        if len(cs) != n:
            raise ValueError(f"{name} needs one entry per mesh")
        return (C.c_void_p * n)(*[(_ptr(c, torch.float64, name).value if c is not None else None)
                                  for c in cs])

    out = C.c_void_p()
    _lib.check(_L.lfem_batch_create_ex(n, ms, ps, int(what), arr(coef_a, "coef_a"), arr(coef_c, "coef_c"),
                                       int(autotune), _stream(stream), C.byref(out)), "lfem_batch_create_ex")
    return out


class BatchOutputs:
    """The output pointer array of a batch, marshalled once: a flat list of
    float64 device tensors (mesh-major, ordered M, A, MC within a mesh) and
    the C array of their addresses.  Keeps the tensors referenced; pass it to
    lfem_assemble_batch in place of the list to skip the per-call marshalling
    (a repeated time step writes the same outputs)."""

    def __init__(self, vals):
        self.vals = list(vals)
        self.array = (C.c_void_p * len(self.vals))(*[_ptr(v, torch.float64, "vals").value for v in self.vals])


def lfem_assemble_batch(batch, vals, stream=None):
    """vals: flat list of float64 device tensors, mesh-major, ordered M, A, MC
    within a mesh, or a BatchOutputs built from such a list."""
    arr = vals.array if isinstance(vals, BatchOutputs) else BatchOutputs(vals).array
    _lib.check(_L.lfem_assemble_batch(batch, arr, _stream(stream)), "lfem_assemble_batch")


def prepare_assemble(mesh, pattern, what: int, coef_a=None, coef_c=None, vals_m=None, vals_a=None,
                     vals_mc=None, scatter: int = LFEM_SCATTER_AUTO, stream=None):
    """lfem_assemble with its arguments marshalled once: returns a callable
    that issues the same call (same tensors, stream and scatter) each time it
    is called.  The tensors stay referenced by the callable."""
    keep = (coef_a, coef_c, vals_m, vals_a, vals_mc)
    args = (mesh, pattern, int(what), _ptr(coef_a, torch.float64, "coef_a"), _ptr(coef_c, torch.float64, "coef_c"),
            _ptr(vals_m, torch.float64, "vals_m"), _ptr(vals_a, torch.float64, "vals_a"),
            _ptr(vals_mc, torch.float64, "vals_mc"), int(scatter), _stream(stream))
    fn = _L.lfem_assemble

    def call():
        _lib.check(fn(*args), "lfem_assemble")

    call.keep = keep
    return call


def lfem_shape_grad(mesh, u, v, alpha, w, z, beta, grad, stream=None):
    st = _L.lfem_shape_grad(mesh, _ptr(u, torch.float64, "u"), _ptr(v, torch.float64, "v"),
                            float(alpha), _ptr(w, torch.float64, "w"),
                            _ptr(z, torch.float64, "z"), float(beta),
                            _ptr(grad, torch.float64, "grad"), _stream(stream))
    _lib.check(st, "lfem_shape_grad")


def lfem_shape_grad_noalloc(mesh, u, v, alpha, w, z, beta, grad, stream=None):
    st = _L.lfem_shape_grad_noalloc(mesh, _ptr(u, torch.float64, "u"), _ptr(v, torch.float64, "v"),
                                    float(alpha), _ptr(w, torch.float64, "w"),
                                    _ptr(z, torch.float64, "z"), float(beta),
                                    _ptr(grad, torch.float64, "grad"), _stream(stream))
    _lib.check(st, "lfem_shape_grad_noalloc")


def lfem_energy(mesh, u, v, alpha, w, z, beta, J_out, stream=None):
    st = _L.lfem_energy(mesh, _ptr(u, torch.float64, "u"), _ptr(v, torch.float64, "v"),
                        float(alpha), _ptr(w, torch.float64, "w"), _ptr(z, torch.float64, "z"),
                        float(beta), _ptr(J_out, torch.float64, "J_out"), _stream(stream))
    _lib.check(st, "lfem_energy")


def lfem_assemble_load(mesh, coef_f, b, stream=None):
    st = _L.lfem_assemble_load(mesh, _ptr(coef_f, torch.float64, "coef_f"), _ptr(b, torch.float64, "b"),
                               _stream(stream))
    _lib.check(st, "lfem_assemble_load")


def lfem_spmv(pattern, vals, x, alpha, y, nvec: int = 1, stream=None):
    st = _L.lfem_spmv(pattern, _ptr(vals, torch.float64, "vals"), _ptr(x, torch.float64, "x"), float(alpha),
                      _ptr(y, torch.float64, "y"), int(nvec), _stream(stream))
    _lib.check(st, "lfem_spmv")


def lfem_dziuk_system(mesh, pattern, tau, x, vals_m, vals_a, vals_s, rhs, stream=None):
    st = _L.lfem_dziuk_system(mesh, pattern, float(tau), _ptr(x, torch.float64, "x"),
                              _ptr(vals_m, torch.float64, "vals_m"), _ptr(vals_a, torch.float64, "vals_a"),
                              _ptr(vals_s, torch.float64, "vals_s"), _ptr(rhs, torch.float64, "rhs"),
                              _stream(stream))
    _lib.check(st, "lfem_dziuk_system")


def lfem_kll_system(mesh, pattern, tau, delta0, nu, H, hist, vals_m, vals_a, vals_s, f, rhs, stream=None):
    st = _L.lfem_kll_system(mesh, pattern, float(tau), float(delta0), _ptr(nu, torch.float64, "nu"),
                            _ptr(H, torch.float64, "H"), _ptr(hist, torch.float64, "hist"),
                            _ptr(vals_m, torch.float64, "vals_m"), _ptr(vals_a, torch.float64, "vals_a"),
                            _ptr(vals_s, torch.float64, "vals_s"), _ptr(f, torch.float64, "f"),
                            _ptr(rhs, torch.float64, "rhs"), _stream(stream))
    _lib.check(st, "lfem_kll_system")


def lfem_assemble_kll(mesh, nu, H, f, stream=None):
    st = _L.lfem_assemble_kll(mesh, _ptr(nu, torch.float64, "nu"), _ptr(H, torch.float64, "H"),
                              _ptr(f, torch.float64, "f"), _stream(stream))
    _lib.check(st, "lfem_assemble_kll")


def lfem_reference_table(dim: int, order: int, quad_points: int = 0) -> dict:
    """Host query of the library's quadrature rule and nodal basis for an
    element type: dict of numpy arrays w (Q,), xi (Q, dim), phi (Q, k),
    dphi (Q, k, dim).  Touches no device."""
    import numpy as np
    q, k = C.c_int(), C.c_int()
    _lib.check(_L.lfem_reference_table(dim, order, quad_points, C.byref(q), C.byref(k), None, None, None, None),
               "lfem_reference_table")
    out = {"w": np.zeros(q.value), "xi": np.zeros((q.value, dim)), "phi": np.zeros((q.value, k.value)),
           "dphi": np.zeros((q.value, k.value, dim))}
    ptrs = [C.c_void_p(out[key].ctypes.data) for key in ("w", "xi", "phi", "dphi")]
    _lib.check(_L.lfem_reference_table(dim, order, quad_points, C.byref(q), C.byref(k), *ptrs),
               "lfem_reference_table")
    return out


def lfem_status_get(mesh) -> int:
    n = C.c_int64()
    _lib.check(_L.lfem_status_get(mesh, C.byref(n)), "lfem_status_get")
    return n.value


def lfem_status_reset(mesh, stream=None):
    _lib.check(_L.lfem_status_reset(mesh, _stream(stream)), "lfem_status_reset")


def lfem_last_error() -> str:
    return _L.lfem_last_error().decode(errors="replace")


def lfem_version() -> str:
    return _L.lfem_version().decode()


def lfem_mesh_destroy(mesh):
    _L.lfem_mesh_destroy(mesh)


def lfem_pattern_destroy(pattern):
    _L.lfem_pattern_destroy(pattern)


def lfem_batch_destroy(batch):
    _L.lfem_batch_destroy(batch)


from .mesh import DeviceMesh, ShapeEnergy, assemble  # noqa: E402  (convenience wrappers)

__all__ += ["DeviceMesh", "ShapeEnergy", "assemble"]
