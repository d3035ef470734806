"""ctypes declarations of the paelast C ABI (include/paelast.h), same names.

Argument marshalling only: every computation runs in the HIP library.  The
library must have been built (``python -m paper_2601_08374_amd.build``); loading
fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# PAELAST_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PAELAST_LIB") or os.path.join(_PKG, "lib", "libpaelast.so")

PA_OK = 0
PA_EINVAL = -1
PA_ENOMEM = -2
PA_EUNSUPPORTED = -3
PA_EHIP = -4
PA_ENOCONV = -5
PA_EBREAKDOWN = -6

PA_F64 = 0
PA_F32 = 1
PA_UNCONSTRAINED = 1
PA_ADD = 2
PA_NOALLOC_SCRATCH_BYTES = 64 << 20
PA_VARIANT_FUSED = 0
PA_VARIANT_UNFUSED_DENSE = 1
PA_VARIANT_UNFUSED_SF = 2
PA_VARIANT_UNFUSED_SF_VOIGT = 3
PA_VARIANT_FUSED_UNSTAGED = 4
PA_VARIANT_FUSED_QUADRATURE = 5
PA_MAT_ELEM_ISO = 0
PA_MAT_QP_ISO = 1
PA_MAT_ANISO = 2
PA_GEOM_AFFINE = 0
PA_GEOM_QP_DATA = 1
PA_GEOM_TRILINEAR = 2
PA_SOLVE_F64 = 0
PA_SOLVE_F32_IR = 1
PA_SOLVE_F32_PREC = 2
PA_STOP_PREC = 0
PA_STOP_TRUE = 1

ERROR_NAMES = {0: "PA_OK", -1: "PA_EINVAL", -2: "PA_ENOMEM", -3: "PA_EUNSUPPORTED", -4: "PA_EHIP",
               -5: "PA_ENOCONV", -6: "PA_EBREAKDOWN"}


class pa_mesh_t(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3), ("A", C.c_double * 9), ("x0", C.c_double * 3),
                ("grade", C.POINTER(C.c_double) * 3), ("clamped_faces", C.c_uint32)]


class pa_solve_opts_t(C.Structure):
    _fields_ = [("mode", C.c_int), ("stop", C.c_int), ("p_levels", C.c_int), ("h_levels", C.c_int),
                ("cheb_degree", C.c_int), ("power_iters", C.c_int), ("cheb_lo_frac", C.c_double),
                ("cheb_safety", C.c_double), ("max_iter", C.c_int), ("inner_rtol", C.c_double),
                ("inner_max_iter", C.c_int), ("max_outer", C.c_int), ("seed", C.c_uint64),
                ("coarse_max_dofs", C.c_int), ("lambda_max", C.POINTER(C.c_double))]


class pa_solve_info_t(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer_iters", C.c_int), ("rel_res_true", C.c_double),
                ("rel_res_prec", C.c_double), ("t_setup", C.c_double), ("t_solve", C.c_double),
                ("num_levels", C.c_int)]


_vp = C.c_void_p
_i = C.c_int
_d = C.c_double
_dp = C.POINTER(C.c_double)

# name -> (restype, argtypes); the list of exported entry points of include/paelast.h
SIGNATURES = {
    "pa_solve_opts_default": (None, [C.POINTER(pa_solve_opts_t)]),
    "pa_elast_setup": (_i, [C.POINTER(pa_mesh_t), _i, _i, _dp, _dp, _i, _vp, C.POINTER(_vp)]),
    "pa_elast_setup_material": (_i, [C.POINTER(pa_mesh_t), _i, _i, _i, _dp, _i, _vp, C.POINTER(_vp)]),
    "pa_elast_setup_geometry": (_i, [C.POINTER(pa_mesh_t), _dp, _i, _i, _i, _dp, _dp, _i, _vp, C.POINTER(_vp)]),
    "pa_elast_setup_unstructured": (_i, [C.c_int64, _dp, C.c_int64, C.POINTER(C.c_int32), C.c_int64,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_uint8), _i, _i, _dp, _dp, _i, _vp,
                                         C.POINTER(_vp)]),
    "pa_elast_destroy": (None, [_vp]),
    "pa_elast_set_stream": (_i, [_vp, _vp]),
    "pa_elast_ndofs": (_i, [_vp, C.POINTER(C.c_int64)]),
    "pa_bytes_required": (C.c_int64, [C.POINTER(pa_mesh_t), _i, _i, _i]),
    "pa_elast_apply": (_i, [_vp, _vp, _vp]),
    "pa_elast_apply_ex": (_i, [_vp, _vp, _vp, _i]),
    "pa_elast_apply_noalloc": (_i, [_vp, _vp, _vp, _i]),
    "pa_elast_apply_variant": (_i, [_vp, _vp, _vp, _i, _i]),
    "pa_elast_diagonal": (_i, [_vp, _vp, _i]),
    "pa_elast_rhs": (_i, [_vp, _dp, _i, _dp, _vp]),
    "gmg_setup": (_i, [_vp, C.POINTER(pa_solve_opts_t), C.POINTER(_vp)]),
    "gmg_destroy": (None, [_vp]),
    "gmg_num_levels": (_i, [_vp]),
    "gmg_level_info": (_i, [_vp, _i, C.POINTER(C.c_int32), C.POINTER(_i), C.POINTER(C.c_int64), C.POINTER(_i),
                            _dp]),
    "gmg_level_op": (_i, [_vp, _i, C.POINTER(_vp)]),
    "gmg_prolong": (_i, [_vp, _i, _vp, _vp]),
    "gmg_restrict": (_i, [_vp, _i, _vp, _vp]),
    "gmg_smooth": (_i, [_vp, _i, _vp, _vp, _i]),
    "gmg_coarse_solve": (_i, [_vp, _vp, _vp]),
    "gmg_vcycle": (_i, [_vp, _vp, _vp]),
    "gmg_pcg_run": (_i, [_vp, _vp, _vp, _d, C.POINTER(pa_solve_info_t)]),
    "gmg_pcg_solve": (_i, [_vp, _vp, _vp, _d, C.POINTER(pa_solve_opts_t), C.POINTER(pa_solve_info_t)]),
    "gmg_pcg_begin": (_i, [_vp, _vp, _vp, _d, C.POINTER(_vp)]),
    "gmg_pcg_step": (_i, [_vp, _i]),
    "gmg_pcg_poll": (_i, [_vp, C.POINTER(_i), C.POINTER(_i)]),
    "gmg_pcg_end": (_i, [_vp, C.POINTER(pa_solve_info_t)]),
    "pa_probe_fma": (_i, [_vp, _i, _i, _i, _vp]),
    "pa_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"paelast HIP library not built: {path} is missing "
                           "(run python -m paper_2601_08374_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int):
    if code != PA_OK:
        raise PaError(code, load().pa_last_error().decode())
    return code


def __getattr__(name):
    # module-level access to the C entry points: capi.pa_elast_apply(...)
    if name in SIGNATURES:
        return getattr(load(), name)
    raise AttributeError(name)
