"""Host-side checks of the C ABI (no GPU needed): every declared symbol is exported,
argument validation returns the documented codes before touching the device,
and the HBM byte model used for admission behaves sensibly."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synthetic as syn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2601_08374_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("library not built")
    return capi, capi.load()


def _declared():
    txt = open(os.path.join(ROOT, "include", "paelast.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"if", "sizeof"})


def test_every_declared_symbol_is_exported():
    capi, lib = _lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(capi.SIGNATURES), set(names) ^ set(capi.SIGNATURES)


def _setup(mesh, p, q, lam, mu, dtype=0):
    capi, lib = _lib()
    from paper_2601_08374_amd import mesh_struct
    ms, keep = mesh_struct(mesh)
    h = C.c_void_p()
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    rc = lib.pa_elast_setup(C.byref(ms), p, q, lam.ctypes.data_as(C.POINTER(C.c_double)),
                            mu.ctypes.data_as(C.POINTER(C.c_double)), dtype, None, C.byref(h))
    return rc, lib.pa_last_error().decode()


@pytest.mark.parametrize("case", ["p0", "p9", "q_low", "q_high", "mu_neg", "lam_bad", "dtype", "det_neg", "n_zero",
                                  "grade_dec", "clamp_bits"])
def test_setup_argument_validation(case):
    mesh = syn.BoxMesh(n=(2, 2, 2))
    ones = np.ones(8)
    p, q, lam, mu, dt = 2, 4, ones, ones, 0
    expect = -1
    if case == "p0":
        p, q = 0, 2
    elif case == "p9":
        p, q, expect = 9, 11, -3
    elif case == "q_low":
        q = 2
    elif case == "q_high":
        q = 6
    elif case == "mu_neg":
        mu = -ones
    elif case == "lam_bad":
        lam = -ones   # lambda + 2 mu / 3 < 0
    elif case == "dtype":
        dt = 7
    elif case == "det_neg":
        mesh = syn.BoxMesh(n=(2, 2, 2), A=np.diag([1.0, -1.0, 1.0]))
    elif case == "n_zero":
        mesh = syn.BoxMesh(n=(2, 0, 2))
    elif case == "grade_dec":
        mesh = syn.BoxMesh(n=(2, 2, 2), grade=[np.array([0.0, 0.7, 0.5]), None, None])
    elif case == "clamp_bits":
        mesh = syn.BoxMesh(n=(2, 2, 2), clamped_faces=1 << 7)
    rc, msg = _setup(mesh, p, q, lam, mu, dt)
    assert rc == expect, (rc, msg)
    assert msg


def test_null_arguments():
    capi, lib = _lib()
    assert lib.pa_elast_apply(None, None, None) == -1
    assert lib.pa_elast_apply_ex(None, None, None, 0) == -1
    assert lib.pa_elast_diagonal(None, None, 0) == -1
    assert lib.gmg_setup(None, None, None) == -1
    assert lib.gmg_pcg_run(None, None, None, 1e-8, None) == -1
    assert lib.gmg_num_levels(None) == 0
    lib.pa_elast_destroy(None)
    lib.gmg_destroy(None)


def test_bytes_required_model():
    capi, lib = _lib()
    from paper_2601_08374_amd import mesh_struct
    small, keep = mesh_struct(syn.BoxMesh(n=(4, 4, 4), clamped_faces=1))
    big, keep2 = mesh_struct(syn.BoxMesh(n=(32, 32, 32), clamped_faces=1))
    a = lib.pa_bytes_required(C.byref(small), 2, 0, 0)
    b = lib.pa_bytes_required(C.byref(small), 2, 0, 1)
    c = lib.pa_bytes_required(C.byref(big), 8, 0, 1)
    d = lib.pa_bytes_required(C.byref(big), 8, 1, 1)
    assert 0 < a < b < c
    N = 3 * (32 * 8 + 1) ** 3
    assert 6 * 8 * N < c < 40 * 8 * N          # a handful of FP64 vectors per level
    assert d < c                               # FP32 hierarchy is smaller even with FP64 outer vectors
    assert lib.pa_bytes_required(C.byref(small), 9, 0, 1) < 0


def test_p1_operator_bytes_follow_the_kernel_switch():
    """p = 1 operators of at most 32768 elements run the sum-factorized kernel and carry its
    per-element skeleton buffer (3 components x 8 element-boundary nodes); larger ones the
    linear-element kernel's tile buffer (8 x 8 column tiles, z chunks as short as keep every
    tile wavefront resident: 2048 wavefronts in double precision, 4096 in single, face arrays
    of 2(tz+1)9 + 2(tz+1)9 + 2 81 words per component).  Host-side accounting only (no GPU
    call)."""
    capi, lib = _lib()
    from paper_2601_08374_amd import mesh_struct

    def operator_bytes(n, dtype):
        ms, keep = mesh_struct(syn.BoxMesh(n=n))
        return lib.pa_bytes_required(C.byref(ms), 1, dtype, 0)

    def tile_words(n, slots):
        nxy = ((n[0] + 7) // 8) * ((n[1] + 7) // 8)
        tz = 1
        while tz < n[2] and nxy * ((n[2] + tz - 1) // tz) > slots:
            tz += 1
        tiles = nxy * ((n[2] + tz - 1) // tz)
        return tiles * 3 * (2 * (tz + 1) * 9 * 2 + 2 * 81)

    for dtype, w in ((0, 8), (1, 4)):
        for n in ((32, 32, 32), (4, 4, 4), (40, 30, 27)):
            NE = n[0] * n[1] * n[2]
            assert NE <= 32768
            assert operator_bytes(n, dtype) == NE * 12 * w + 24 * NE * w + 4096, n
        for n in ((40, 40, 40), (130, 130, 9), (120, 120, 96), (400, 400, 5)):
            NE = n[0] * n[1] * n[2]
            assert NE > 32768
            slots = 2048 if dtype == 0 else 4096
            assert operator_bytes(n, dtype) == NE * 12 * w + tile_words(n, slots) * w + 4096, (n, dtype)
    # the two slot counts give different chunks on the sheared box of the benchmark
    assert tile_words((120, 120, 96), 2048) != tile_words((120, 120, 96), 4096)


def test_binding_constants_match_the_header():
    """Every integer constant include/paelast.h defines has the same value in the ctypes
    binding (host-side check, no GPU)."""
    from paper_2601_08374_amd import capi
    hdr = open(os.path.join(ROOT, "include", "paelast.h")).read()
    defs = {}
    for name, val in re.findall(r"^#define\s+(PA_\w+)\s+\(?(-?\d+)u?\)?", hdr, flags=re.M):
        defs[name] = int(val)
    assert "PA_VARIANT_FUSED_QUADRATURE" in defs and len(defs) >= 25
    for name, val in defs.items():
        if name == "PA_NOALLOC_SCRATCH_BYTES":
            continue   # (64u << 20): not a plain integer literal
        assert hasattr(capi, name), name
        assert getattr(capi, name) == val, (name, getattr(capi, name), val)


def test_solve_opts_defaults():
    capi, lib = _lib()
    o = capi.pa_solve_opts_t()
    lib.pa_solve_opts_default(C.byref(o))
    assert o.cheb_degree == 2 and o.power_iters == 10 and o.max_iter == 5000
    assert abs(o.cheb_lo_frac - 0.1) < 1e-15 and abs(o.cheb_safety - 1.2) < 1e-15
    assert abs(o.inner_rtol - 3e-3) < 1e-18 and o.inner_max_iter == 50 and o.max_outer == 20
