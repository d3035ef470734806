"""MI355X (gfx950) matrix-free high-order linear elasticity: PA apply + GMG-PCG.

Thin Python layer over the C ABI in ``include/paelast.h`` (``capi``): it only
marshals arguments (torch tensors for device memory, torch streams).  All
arithmetic runs in the HIP library; if it is not built, import still works but
every call raises.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import capi
from .capi import (PA_ADD, PA_F32, PA_F64, PA_GEOM_AFFINE, PA_GEOM_QP_DATA, PA_GEOM_TRILINEAR, PA_MAT_ANISO, PA_MAT_ELEM_ISO, PA_MAT_QP_ISO, PA_SOLVE_F32_IR, PA_SOLVE_F32_PREC, PA_SOLVE_F64, PA_STOP_PREC, PA_STOP_TRUE,
                   PA_UNCONSTRAINED, PaError)

__all__ = ["Operator", "Hierarchy", "mesh_struct", "capi", "PA_F64", "PA_F32", "PA_UNCONSTRAINED", "PA_ADD",
           "PA_MAT_ELEM_ISO", "PA_MAT_QP_ISO", "PA_MAT_ANISO", "PA_GEOM_AFFINE", "PA_GEOM_QP_DATA",
           "PA_GEOM_TRILINEAR",
           "PA_SOLVE_F64", "PA_SOLVE_F32_IR", "PA_SOLVE_F32_PREC", "PA_STOP_PREC", "PA_STOP_TRUE", "PaError", "solve_opts"]


def _torch():
    import torch
    return torch


def mesh_struct(mesh):
    """pa_mesh_t from a box description (n, L, A, x0, grade, clamped_faces attributes).

    Returns (struct, keepalive) -- keep the second item alive while the struct is used.
    """
    m = capi.pa_mesh_t()
    keep = []
    for a in range(3):
        m.n[a] = int(mesh.n[a])
        m.L[a] = float(mesh.L[a])
        m.x0[a] = float(mesh.x0[a])
        g = None if mesh.grade is None else mesh.grade[a]
        if g is not None:
            arr = np.ascontiguousarray(g, dtype=np.float64)
            keep.append(arr)
            m.grade[a] = arr.ctypes.data_as(C.POINTER(C.c_double))
        else:
            m.grade[a] = C.POINTER(C.c_double)()
    A = np.asarray(mesh.A, dtype=np.float64).reshape(9)
    for i in range(9):
        m.A[i] = float(A[i])
    m.clamped_faces = int(mesh.clamped_faces)
    return m, keep


def _dptr(t) -> int:
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def solve_opts(**kw) -> capi.pa_solve_opts_t:
    o = capi.pa_solve_opts_t()
    capi.pa_solve_opts_default(C.byref(o))
    keep = None
    for k, v in kw.items():
        if k == "lambda_max":
            keep = np.ascontiguousarray(v, dtype=np.float64)
            o.lambda_max = keep.ctypes.data_as(C.POINTER(C.c_double))
        else:
            setattr(o, k, v)
    o._keep = keep
    return o


class Operator:
    """The PA elasticity operator of a box mesh (owns a pa_op_t)."""

    def __init__(self, mesh, p: int, lam, mu, q: Optional[int] = None, dtype: int = PA_F64, stream=None,
                 device: str = "cuda"):
        NE = int(mesh.n[0] * mesh.n[1] * mesh.n[2])
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (NE,)))
        mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (NE,)))
        self.mesh, self.p, self.q = mesh, int(p), int(q if q is not None else p + 2)
        self.dtype = dtype
        self.stream = stream
        ms, keep = mesh_struct(mesh)
        h = C.c_void_p()
        capi.check(capi.pa_elast_setup(C.byref(ms), self.p, self.q, lam.ctypes.data_as(C.POINTER(C.c_double)),
                                       mu.ctypes.data_as(C.POINTER(C.c_double)), dtype,
                                       C.c_void_p(_stream_handle(stream)), C.byref(h)))
        self._attach(h)

    def _attach(self, h):
        self.handle = h
        n = C.c_int64()
        capi.check(capi.pa_elast_ndofs(h, C.byref(n)))
        self.N = int(n.value)
        self._hier = None

    @classmethod
    def with_material(cls, mesh, p: int, kind: int, data, q: Optional[int] = None, dtype: int = PA_F64,
                      stream=None):
        """pa_elast_setup_material: kind PA_MAT_QP_ISO with data [NE, q^3, 2] (lambda, mu per
        Gauss-Legendre point, point qx + q (qy + q qz)), or PA_MAT_ANISO with data [NE, 21]
        (upper triangle of the Voigt stiffness, row by row)."""
        self = cls.__new__(cls)
        self.mesh, self.p, self.q = mesh, int(p), int(q if q is not None else p + 2)
        self.dtype = dtype
        self.stream = stream
        d = np.ascontiguousarray(np.asarray(data, dtype=np.float64))
        NE = int(mesh.n[0] * mesh.n[1] * mesh.n[2])
        want = NE * (2 * self.q ** 3 if kind == PA_MAT_QP_ISO else 21)
        if d.size != want:
            raise ValueError(f"material data must hold {want} values, got {d.size}")
        ms, keep = mesh_struct(mesh)
        h = C.c_void_p()
        capi.check(capi.pa_elast_setup_material(C.byref(ms), self.p, self.q, int(kind),
                                                d.ctypes.data_as(C.POINTER(C.c_double)), dtype,
                                                C.c_void_p(_stream_handle(stream)), C.byref(h)))
        self._attach(h)
        return self

    @classmethod
    def unstructured(cls, hm, lam, mu, q: Optional[int] = None, dtype: int = PA_F64, stream=None):
        """pa_elast_setup_unstructured from a mesh description with the fields vertices
        [NV, 3], elem_vertices [NE, 8], p, elem_nodes [NE, (p+1)^3], num_nodes and clamped
        [num_nodes] (e.g. synthetic.HexMesh)."""
        self = cls.__new__(cls)
        self.mesh, self.p = hm, int(hm.p)
        self.q = int(q if q is not None else self.p + 2)
        self.dtype = dtype
        self.stream = stream
        V = np.ascontiguousarray(np.asarray(hm.vertices, dtype=np.float64))
        ev = np.ascontiguousarray(np.asarray(hm.elem_vertices, dtype=np.int32))
        en = np.ascontiguousarray(np.asarray(hm.elem_nodes, dtype=np.int32))
        NE, nn = ev.shape[0], int(hm.num_nodes)
        D = self.p + 1
        if V.ndim != 2 or V.shape[1] != 3 or ev.shape != (NE, 8) or en.shape != (NE, D ** 3):
            raise ValueError("vertices [NV,3], elem_vertices [NE,8] and elem_nodes [NE,(p+1)^3] expected")
        cl = None if hm.clamped is None else np.ascontiguousarray(np.asarray(hm.clamped, dtype=np.uint8))
        if cl is not None and cl.shape != (nn,):
            raise ValueError(f"clamped must be [{nn}]")
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (NE,)))
        mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (NE,)))
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
        h = C.c_void_p()
        capi.check(capi.pa_elast_setup_unstructured(
            V.shape[0], V.ctypes.data_as(dp), NE, ev.ctypes.data_as(ip), nn, en.ctypes.data_as(ip),
            None if cl is None else cl.ctypes.data_as(C.POINTER(C.c_uint8)), self.p, self.q,
            lam.ctypes.data_as(dp), mu.ctypes.data_as(dp), dtype, C.c_void_p(_stream_handle(stream)), C.byref(h)))
        self._attach(h)
        return self

    @classmethod
    def with_geometry(cls, mesh, p: int, vertices, lam, mu, kind: int = PA_GEOM_TRILINEAR, q: Optional[int] = None,
                      dtype: int = PA_F64, stream=None):
        """pa_elast_setup_geometry: trilinear hexahedra through vertices [(n0+1)(n1+1)(n2+1), 3]
        (vertex (i,j,k) at i + (n0+1)(j + (n1+1)k)); kind PA_GEOM_QP_DATA stores J^{-1} and
        w det J per quadrature point, PA_GEOM_TRILINEAR recomputes them in the apply."""
        self = cls.__new__(cls)
        self.mesh, self.p, self.q = mesh, int(p), int(q if q is not None else p + 2)
        self.dtype = dtype
        self.stream = stream
        NE = int(mesh.n[0] * mesh.n[1] * mesh.n[2])
        v = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64))
        nv = (int(mesh.n[0]) + 1) * (int(mesh.n[1]) + 1) * (int(mesh.n[2]) + 1)
        if v.shape != (nv, 3):
            raise ValueError(f"vertices must be [{nv}, 3], got {v.shape}")
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (NE,)))
        mu = np.ascontiguousarray(np.broadcast_to(np.asarray(mu, dtype=np.float64), (NE,)))
        dp = C.POINTER(C.c_double)
        ms, keep = mesh_struct(mesh)
        h = C.c_void_p()
        capi.check(capi.pa_elast_setup_geometry(C.byref(ms), v.ctypes.data_as(dp), int(kind), self.p, self.q,
                                                lam.ctypes.data_as(dp), mu.ctypes.data_as(dp), dtype,
                                                C.c_void_p(_stream_handle(stream)), C.byref(h)))
        self._attach(h)
        return self

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.dtype == PA_F64 else torch.float32

    def empty(self):
        torch = _torch()
        return torch.empty(self.N, dtype=self.torch_dtype, device="cuda")

    def apply(self, x, y=None, flags: int = 0):
        if y is None:
            y = self.empty()
        assert x.dtype == self.torch_dtype and y.dtype == self.torch_dtype
        assert x.numel() == self.N and y.numel() == self.N and x.is_contiguous() and y.is_contiguous()
        capi.check(capi.pa_elast_apply_ex(self.handle, C.c_void_p(_dptr(x)), C.c_void_p(_dptr(y)), int(flags)))
        return y

    def apply_noalloc(self, x, y=None, flags: int = 0):
        """pa_elast_apply_noalloc: the same apply with the library's static scratch array."""
        if y is None:
            y = self.empty()
        assert x.dtype == self.torch_dtype and y.dtype == self.torch_dtype
        assert x.numel() == self.N and y.numel() == self.N and x.is_contiguous() and y.is_contiguous()
        capi.check(capi.pa_elast_apply_noalloc(self.handle, C.c_void_p(_dptr(x)), C.c_void_p(_dptr(y)), int(flags)))
        return y

    def apply_variant(self, x, y=None, variant: int = 0, flags: int = 0):
        """pa_elast_apply_variant: the unfused ablation forms of the same operator."""
        if y is None:
            y = self.empty()
        assert x.dtype == self.torch_dtype and y.dtype == self.torch_dtype
        assert x.numel() == self.N and y.numel() == self.N and x.is_contiguous() and y.is_contiguous()
        capi.check(capi.pa_elast_apply_variant(self.handle, C.c_void_p(_dptr(x)), C.c_void_p(_dptr(y)), int(flags),
                                               int(variant)))
        return y

    def diagonal(self, flags: int = 0):
        d = self.empty()
        capi.check(capi.pa_elast_diagonal(self.handle, C.c_void_p(_dptr(d)), int(flags)))
        return d

    def rhs(self, f=(0.0, 0.0, 0.0), traction_face: int = -1, t=(0.0, 0.0, 0.0)):
        torch = _torch()
        b = torch.empty(self.N, dtype=torch.float64, device="cuda")
        fa = (C.c_double * 3)(*f)
        ta = (C.c_double * 3)(*t)
        capi.check(capi.pa_elast_rhs(self.handle, fa, int(traction_face), ta, C.c_void_p(_dptr(b))))
        return b

    def hierarchy(self, **opts):
        return Hierarchy(self, **opts)

    def solve(self, b, x=None, rtol: float = 1e-8, **opts):
        """gmg_pcg_solve: hierarchy cached on the operator."""
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        o = solve_opts(**opts)
        info = capi.pa_solve_info_t()
        rc = capi.gmg_pcg_solve(self.handle, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x)), float(rtol), C.byref(o),
                                C.byref(info))
        if rc not in (capi.PA_OK, capi.PA_ENOCONV):
            capi.check(rc)
        return x, info, rc

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            capi.pa_elast_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hierarchy:
    """A GMG hierarchy (owns a pa_gmg_t) built on an Operator."""

    def __init__(self, op: Operator, **opts):
        self.op = op
        self.opts = solve_opts(**opts)
        h = C.c_void_p()
        capi.check(capi.gmg_setup(op.handle, C.byref(self.opts), C.byref(h)))
        self.handle = h
        self.num_levels = capi.gmg_num_levels(h)

    def level_info(self, level: int):
        n = (C.c_int32 * 3)()
        p, dt = C.c_int(), C.c_int()
        nd = C.c_int64()
        lm = C.c_double()
        capi.check(capi.gmg_level_info(self.handle, level, n, C.byref(p), C.byref(nd), C.byref(dt), C.byref(lm)))
        return dict(n=tuple(n), p=p.value, N=nd.value, dtype=dt.value, lambda_max=lm.value)

    def _vec(self, level: int):
        torch = _torch()
        info = self.level_info(level)
        return torch.zeros(info["N"], dtype=torch.float64 if info["dtype"] == PA_F64 else torch.float32,
                           device="cuda")

    def level_apply(self, level: int, x, y=None, flags: int = 0):
        h = C.c_void_p()
        capi.check(capi.gmg_level_op(self.handle, level, C.byref(h)))
        if y is None:
            y = _torch().empty_like(x)
        capi.check(capi.pa_elast_apply_ex(h, C.c_void_p(_dptr(x)), C.c_void_p(_dptr(y)), int(flags)))
        return y

    def level_diagonal(self, level: int, flags: int = 0):
        h = C.c_void_p()
        capi.check(capi.gmg_level_op(self.handle, level, C.byref(h)))
        d = self._vec(level)
        capi.check(capi.pa_elast_diagonal(h, C.c_void_p(_dptr(d)), int(flags)))
        return d

    def prolong(self, level: int, xc):
        xf = self._vec(level)
        capi.check(capi.gmg_prolong(self.handle, level, C.c_void_p(_dptr(xc)), C.c_void_p(_dptr(xf))))
        return xf

    def restrict(self, level: int, rf):
        rc = self._vec(level + 1)
        capi.check(capi.gmg_restrict(self.handle, level, C.c_void_p(_dptr(rf)), C.c_void_p(_dptr(rc))))
        return rc

    def smooth(self, level: int, b, x=None):
        if x is None:
            x = self._vec(level)
            capi.check(capi.gmg_smooth(self.handle, level, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x)), 1))
        else:
            capi.check(capi.gmg_smooth(self.handle, level, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x)), 0))
        return x

    def coarse_solve(self, b):
        x = self._vec(self.num_levels - 1)
        capi.check(capi.gmg_coarse_solve(self.handle, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x))))
        return x

    def vcycle(self, r):
        z = self._vec(0)
        capi.check(capi.gmg_vcycle(self.handle, C.c_void_p(_dptr(r)), C.c_void_p(_dptr(z))))
        return z

    def pcg(self, b, x=None, rtol: float = 1e-8):
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        info = capi.pa_solve_info_t()
        rc = capi.gmg_pcg_run(self.handle, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x)), float(rtol), C.byref(info))
        if rc not in (capi.PA_OK, capi.PA_ENOCONV):
            capi.check(rc)
        return x, info, rc

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            capi.gmg_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
