"""Convenience wrappers over the C ABI: a mesh handle that keeps its device
tensors alive, and the shape-energy autograd Function.  Argument marshalling
only; the arithmetic runs in liblfem.so."""

from __future__ import annotations

import numpy as np
import torch

from . import (LFEM_A, LFEM_BULK, LFEM_M, LFEM_MC, LFEM_SCATTER_AUTO, LFEM_SURFACE,
               copy_from_device, lfem_assemble, lfem_assemble_kll, lfem_assemble_load,
               lfem_dziuk_system, lfem_energy, lfem_kll_system, lfem_mesh_create, lfem_mesh_destroy,
               lfem_mesh_set_coords, lfem_pattern_build,
               lfem_pattern_destroy, lfem_pattern_get, lfem_shape_grad, lfem_spmv, lfem_status_get)


class DeviceMesh:
    """A mesh resident in device memory plus its library handles.

    ``coords`` float64 (n_amb, N) and ``conn`` int32 (k, T) tensors are kept
    referenced for the lifetime of the handle (the library does not copy
    them)."""

    def __init__(self, domain, dim, order, coords, conn, quad_points=0, device="cuda",
                 stream=None):
        self.domain = domain if isinstance(domain, int) else (
            LFEM_SURFACE if domain == "surface" else LFEM_BULK)
        self.dim, self.order = int(dim), int(order)
        self.coords = torch.as_tensor(np.ascontiguousarray(coords), dtype=torch.float64,
                                      device=device).contiguous()
        self.conn = torch.as_tensor(np.ascontiguousarray(conn), dtype=torch.int32,
                                    device=device).contiguous()
        self.handle = lfem_mesh_create(self.domain, self.dim, self.order, self.coords,
                                       self.conn, quad_points, stream)
        self.pattern = None
        self.nnz = None

    @classmethod
    def from_dict(cls, m, device="cuda", stream=None):
        return cls(m["domain"], m["dim"], m["order"], m["coords"], m["conn"],
                   m.get("quad", 0), device, stream)

    @property
    def N(self):
        return self.coords.shape[1]

    @property
    def T(self):
        return self.conn.shape[1]

    def build_pattern(self, stream=None):
        if self.pattern is None:
            self.pattern = lfem_pattern_build(self.handle, stream)
            _, self.nnz, _, _ = lfem_pattern_get(self.pattern)
        return self.pattern

    def pattern_tensors(self):
        """(row_ptr int32 (N+1,), col_idx int32 (nnz,)) copied out of the pattern
        once and kept (the pattern is fixed for the handle's lifetime)."""
        self.build_pattern()
        if getattr(self, "_pattern_t", None) is None:
            n, nnz, rp, ci = lfem_pattern_get(self.pattern)
            row_ptr = torch.empty(n + 1, dtype=torch.int32, device=self.coords.device)
            col_idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.coords.device)
            copy_from_device(row_ptr, rp, (n + 1) * 4)
            copy_from_device(col_idx, ci, nnz * 4)
            self._pattern_t = (row_ptr, col_idx[:nnz])
        return self._pattern_t

    def sparse_csr(self, vals):
        """A torch.sparse_csr_tensor (N, N) over the pattern's index tensors
        (shared between the matrices of this mesh) with the given (nnz,) values."""
        rp, ci = self.pattern_tensors()
        return torch.sparse_csr_tensor(rp, ci, vals, size=(self.N, self.N), dtype=torch.float64,
                                       device=vals.device)

    def matvec(self, vals, x, alpha=1.0, out=None, stream=None):
        """y = alpha * V x for an assembled matrix with values `vals` (nnz,) and
        x of shape (N,) or (n, N) (component-major); rows summed in column order."""
        self.build_pattern(stream)
        x = x.contiguous()
        y = out if out is not None else torch.empty_like(x)
        nvec = 1 if x.dim() == 1 else x.shape[0]
        lfem_spmv(self.pattern, vals, x, alpha, y, nvec, stream)
        return y

    def set_coords(self, coords):
        coords = coords.contiguous()
        lfem_mesh_set_coords(self.handle, coords)
        self.coords = coords

    def assemble(self, what, coef_a=None, coef_c=None, scatter=LFEM_SCATTER_AUTO, out=None,
                 stream=None):
        """Returns a dict {"M", "A", "MC"} of float64 value tensors (nnz,)."""
        self.build_pattern(stream)
        out = dict(out or {})
        dev = self.coords.device
        for bit, key in ((LFEM_M, "M"), (LFEM_A, "A"), (LFEM_MC, "MC")):
            if what & bit and key not in out:
                out[key] = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        lfem_assemble(self.handle, self.pattern, what, coef_a, coef_c, out.get("M"),
                      out.get("A"), out.get("MC"), scatter, stream)
        return out

    def load(self, f=None, out=None, stream=None):
        """Load vector b_j = sum_E sum_q w mu f_h phi_j as a float64 (N,) tensor;
        f: nodal values (N,) or None for f = 1."""
        b = out if out is not None else torch.empty(self.N, dtype=torch.float64, device=self.coords.device)
        lfem_assemble_load(self.handle, f, b, stream)
        return b

    def kll(self, nu, H=None, out=None, stream=None):
        """Non-linear terms f = (f_1; f_2) of the mean-curvature-flow example as a
        float64 (n_amb + 1, N) tensor; nu: (n_amb, N) nodal vector field, H: (N,)
        or None for H = 1."""
        n = self.coords.shape[0]
        f = out if out is not None else torch.empty(n + 1, self.N, dtype=torch.float64,
                                                    device=self.coords.device)
        lfem_assemble_kll(self.handle, nu, H, f, stream)
        return f

    def dziuk_system(self, tau, x=None, out=None, stream=None):
        """Per-step system of Dziuk's mean-curvature-flow scheme at the current
        coordinates: dict with "M", "A", "S" = M + tau A (nnz,) and "rhs" = M x
        as an (n_amb, N) tensor (x: (n_amb, N) or None for the coordinates)."""
        self.build_pattern(stream)
        out = dict(out or {})
        dev = self.coords.device
        for key in ("M", "A", "S"):
            if key not in out:
                out[key] = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        if "rhs" not in out:
            out["rhs"] = torch.empty(self.coords.shape[0], self.N, dtype=torch.float64, device=dev)
        lfem_dziuk_system(self.handle, self.pattern, tau, x, out["M"], out["A"], out["S"], out["rhs"], stream)
        return out

    def kll_system(self, tau, delta0, nu, H, hist=None, out=None, stream=None):
        """Per-step system of the BDF mean-curvature-flow algorithm (coupled
        in u = (nu; H)) at the current coordinates (the extrapolated surface):
        dict with "M", "A", "S" = delta0 M + tau A (nnz,), "f" the non-linear
        terms and "rhs" = tau f - M hist, both (n_amb + 1, N).  nu: (n_amb, N)
        and H: (N,) the extrapolated normal and mean curvature; hist:
        (n_amb + 1, N) = sum_{j>=1} delta_j u^{n-j}, or None for zero."""
        self.build_pattern(stream)
        out = dict(out or {})
        dev = self.coords.device
        for key in ("M", "A", "S"):
            if key not in out:
                out[key] = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        for key in ("f", "rhs"):
            if key not in out:
                out[key] = torch.empty(self.coords.shape[0] + 1, self.N, dtype=torch.float64, device=dev)
        lfem_kll_system(self.handle, self.pattern, tau, delta0, nu, H, hist, out["M"], out["A"], out["S"],
                        out["f"], out["rhs"], stream)
        return out

    def degenerate_count(self):
        return lfem_status_get(self.handle)

    def close(self):
        if getattr(self, "pattern", None) is not None:
            lfem_pattern_destroy(self.pattern)
            self.pattern = None
        if getattr(self, "handle", None) is not None:
            lfem_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _AtCoords:
    """Point a DeviceMesh at other coordinates for the duration of a block and
    restore its own afterwards (the handle never keeps a pointer into a tensor
    the caller may free)."""

    def __init__(self, mesh, x):
        self.mesh, self.x = mesh, x

    def __enter__(self):
        self.saved = self.mesh.coords
        self.mesh.set_coords(self.x)
        return self.mesh

    def __exit__(self, *exc):
        self.mesh.set_coords(self.saved)
        return False


class ShapeEnergy(torch.autograd.Function):
    """J(x) = alpha u^T A(x) v + beta w^T M(x) z as a differentiable function of
    the node coordinates x (n_amb, N) and of the nodal vectors u, v, w, z.

    Forward: lfem_energy (matrix-free).  Backward: dJ/dx by lfem_shape_grad;
    dJ/du = alpha A v, dJ/dv = alpha A u, dJ/dw = beta M z, dJ/dz = beta M w
    (A and M symmetric) by assembling A(x), M(x) and lfem_spmv, only for the
    inputs that require a gradient.  The mesh's own coordinates are restored
    after each call."""

    @staticmethod
    def forward(ctx, x, mesh, u, v, w=None, z=None, alpha=1.0, beta=1.0):
        x = x.detach().contiguous()
        J = torch.empty(1, dtype=torch.float64, device=x.device)
        with _AtCoords(mesh, x):
            lfem_energy(mesh.handle, u, v, alpha, w, z, beta, J)
        ctx.mesh = mesh
        ctx.args = (alpha, beta)
        ctx.save_for_backward(x, u, v, w, z)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        x, u, v, w, z = ctx.saved_tensors
        alpha, beta = ctx.args
        mesh = ctx.mesh
        need = ctx.needs_input_grad
        gx = gu = gv = gw = gz = None
        with _AtCoords(mesh, x):
            if need[0]:
                g = torch.empty_like(x)
                lfem_shape_grad(mesh.handle, u, v, alpha, w, z, beta, g)
                gx = g * gJ
            want_a = u is not None and v is not None and (need[2] or need[3])
            want_m = w is not None and z is not None and (need[4] or need[5])
            if want_a or want_m:
                what = (LFEM_A if want_a else 0) | (LFEM_M if want_m else 0)
                mats = mesh.assemble(what)
                if want_a:
                    if need[2]:
                        gu = mesh.matvec(mats["A"], v.detach(), alpha) * gJ
                    if need[3]:
                        gv = mesh.matvec(mats["A"], u.detach(), alpha) * gJ
                if want_m:
                    if need[4]:
                        gw = mesh.matvec(mats["M"], z.detach(), beta) * gJ
                    if need[5]:
                        gz = mesh.matvec(mats["M"], w.detach(), beta) * gJ
        return (gx, None, gu, gv, gw, gz, None, None)


_KINDS = {"mass": LFEM_M, "m": LFEM_M, "stiffness": LFEM_A, "a": LFEM_A, "weighted": LFEM_MC, "mc": LFEM_MC}


def assemble(mesh, kind, coef=None, scatter=LFEM_SCATTER_AUTO, stream=None):
    """One matrix of a DeviceMesh as a torch.sparse_csr_tensor (N, N), float64:
    kind "mass" (M), "stiffness" (A, with the nodal coefficient `coef` inside
    when given) or "weighted" (M_c, `coef` required).  The index tensors are
    the mesh's pattern, shared by every matrix assembled on it."""
    bit = _KINDS[kind.lower()]
    if bit == LFEM_MC and coef is None:
        raise ValueError("the weighted mass needs a nodal coefficient")
    out = mesh.assemble(bit, coef_a=coef if bit == LFEM_A else None,
                        coef_c=coef if bit == LFEM_MC else None, scatter=scatter, stream=stream)
    key = {LFEM_M: "M", LFEM_A: "A", LFEM_MC: "MC"}[bit]
    return mesh.sparse_csr(out[key])
