"""Benchmarks beside the operator sweep.

Solver: the 8:1:1 cantilever (80x8x8 hexahedra, clamped at x=0, unit downward
traction on x=8, E=1, nu=0.3) at p in {4,6,8}: plain FP64 GMG-PCG, the FP32 apply /
FP32 V-cycle inside FP64 iterative refinement, and FP64 PCG preconditioned by the
FP32 V-cycle, all to a true relative residual of 1e-8, with p-hierarchy down to 1
and 2 h-levels, Chebyshev(3)-Jacobi smoothing; at p = 8 also with the material
given per quadrature point.

Apply: the cumulative ablation (unfused variants vs the fused kernel), the fused
apply with the three material data forms, the fused apply on trilinear
(non-affine) hexahedra with stored vs recomputed geometry, and the fused apply on the
same geometry given as an unstructured mesh, on the sheared box."""
from __future__ import annotations

import time

import numpy as np


def _solve(pa, torch, mesh, p, lam, mu, mode, reps=3, qp_data=None):
    NE = mesh.num_elements
    if qp_data is None:
        op = pa.Operator(mesh, p, np.full(NE, lam), np.full(NE, mu))
    else:
        op = pa.Operator.with_material(mesh, p, pa.PA_MAT_QP_ISO, qp_data)
    b = op.rhs((0.0, 0.0, 0.0), 1, (0.0, 0.0, -1.0))
    best = None
    for _ in range(reps):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = op.hierarchy(mode=mode, stop=pa.PA_STOP_TRUE, cheb_degree=3, h_levels=2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info, rc = H.pcg(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        H.close()
        rec = {"rc": rc, "setup_s": t1 - t0, "solve_s": t2 - t1, "iters": info.iters, "outer": info.outer_iters,
               "rel_res_true": info.rel_res_true, "levels": info.num_levels, "N": op.N}
        if best is None or rec["solve_s"] < best[0]["solve_s"]:
            best = (rec, x)
    rec, x = best
    rec["solver_gdofs_L1"] = rec["iters"] * op.N / rec["solve_s"] / 1e9
    return rec, x, op


def cantilever_solves(torch, dev, ps=(4, 6, 8)):
    import synthetic as syn
    import paper_2601_08374_amd as pa
    mesh = syn.cantilever_mesh(80, 8, 8)
    lam, mu = (float(v) for v in syn.lame_from_young_poisson(1.0, 0.3))
    out = {"workload": "cantilever 80x8x8, clamped x=0, traction (0,0,-1) on x=8, E=1, nu=0.3, rtol 1e-8 "
                       "(true residual), p-levels to 1 + 2 h-levels, Chebyshev(3)-Jacobi"}
    for p in ps:
        r64, x64, op = _solve(pa, torch, mesh, p, lam, mu, pa.PA_SOLVE_F64)
        out[f"p{p}"] = {"f64": r64}
        Ax = op.apply(x64)
        for mode, name in ((pa.PA_SOLVE_F32_IR, "f32_ir"), (pa.PA_SOLVE_F32_PREC, "f32_prec")):
            r32, x32, _ = _solve(pa, torch, mesh, p, lam, mu, mode)
            # error against the FP64 solution, in the energy norm of the FP64 operator
            e = x32 - x64
            Ae = op.apply(e)
            r32["err_vs_f64_energy"] = float(torch.sqrt((e @ Ae) / (x64 @ Ax)))
            r32["err_vs_f64_l2"] = float(torch.linalg.norm(e) / torch.linalg.norm(x64))
            r32["time_vs_f64"] = r32["solve_s"] / r64["solve_s"]
            out[f"p{p}"][name] = r32
            del x32, e, Ae
        del x64, Ax, op
        torch.cuda.empty_cache()
    # the same cantilever with the material at every quadrature point (the paper's PA data
    # form): the finest level keeps the per-point data, coarser levels its element means
    pq = ps[-1]
    NE = mesh.num_elements
    lq, mq = syn.quadrature_point_lame(np.full(NE, lam), np.full(NE, mu), pq + 2, seed=11, spread=0.4)
    data = np.stack([lq, mq], axis=-1)
    qrec = {"workload": f"p={pq}, per-point lambda, mu = the E=1, nu=0.3 values x (1 + 0.4 u), u ~ U[-1,1] "
                        "independently per point (seed 11); otherwise as above"}
    for mode, name in ((pa.PA_SOLVE_F64, "f64"), (pa.PA_SOLVE_F32_PREC, "f32_prec")):
        r, x, op = _solve(pa, torch, mesh, pq, lam, mu, mode, qp_data=data)
        r["time_vs_element_data"] = r["solve_s"] / out[f"p{pq}"][name]["solve_s"]
        qrec[name] = r
        del x, op
        torch.cuda.empty_cache()
    out[f"p{pq}_qpoint"] = qrec
    return out


PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X vector FP64 / FP32
PEAK_HBM_GBS = 8000.0                        # MI355X HBM3E

# Pointwise FLOPs per quadrature point beyond the isotropic stress of the paper's count:
# per-point Lame data (2 products), the anisotropic C eps_V (6 strains, 36 products + 30
# sums, 6 scalings, less the ~15 of the isotropic stress), the recomputed trilinear
# Jacobian (2 x 3 column FMAs, 9 cofactors of 3, det J of 5, 1/det J and its scaling).
EXTRA_POINT_FLOPS = {"qpoint_iso": 2, "anisotropic": 60, "trilinear": 46}


def flops_per_element(p: int, q: int | None = None) -> int:
    """Per-element FLOPs of the optimized operator, the paper's count (Sec. 5.4.1 table):
    30 D^3 Q + 36 D^2 Q^2 + 36 D Q^3 + 113 Q^3 + 12 D^3, D = p+1, Q = p+2."""
    D = p + 1
    Q = p + 2 if q is None else q
    return 30 * D ** 3 * Q + 36 * D ** 2 * Q ** 2 + 36 * D * Q ** 3 + 113 * Q ** 3 + 12 * D ** 3


def algorithmic_bytes(N: int, NE: int, word: int) -> int:
    """Read x once, write y once, 12 words of per-element PA data."""
    return 2 * word * N + 12 * word * NE


def _rates(N, NE, p, word, dname, t, extra_words=0, extra_bytes=0, extra_flops_pt=0):
    """Time per apply and its rates against the FP VALU and HBM peaks.  Algorithmic bytes:
    x and y once, the 12-word element data, the form's extra words per element and extra
    bytes; FLOPs: the paper's count plus the form's extra pointwise FLOPs."""
    Q = p + 2
    fl = (flops_per_element(p) + extra_flops_pt * Q ** 3) * NE
    by = algorithmic_bytes(N, NE, word) + extra_words * word * NE + extra_bytes
    return {"us": round(t * 1e6, 1), "gdofs": round(N / t / 1e9, 3), "tflops": round(fl / t / 1e12, 3),
            "frac_alu": round(fl / t / 1e12 / PEAK_TFLOPS[dname], 4), "gbs": round(by / t / 1e9, 1),
            "frac_hbm": round(by / t / 1e9 / PEAK_HBM_GBS, 4), "algorithmic_bytes": int(by),
            "flops": int(fl)}


def _time_apply(torch, dev, op, reps):
    """Mean HIP-event time of reps applies (after one warm-up) on the current stream."""
    import synthetic as syn
    tdt = torch.float64 if op.dtype == 0 else torch.float32
    x = torch.tensor(syn.uniform_vector(op.N, 0), dtype=tdt, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    op.apply(x, y)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        op.apply(x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def apply_material(torch, dev, ps=(1, 2, 4, 8), reps=10):
    """The fused apply with the three material data forms on the sheared box (q = p+2):
    per-element Lame parameters, per-quadrature-point Lame parameters and a per-element
    anisotropic Voigt stiffness; HIP-event time per apply, FP64 and FP32, with rates
    against the VALU and HBM peaks."""
    import synthetic as syn
    import paper_2601_08374_amd as pa
    out = {"workload": "sheared box (~4.2M dofs), q=p+2; two materials (element), +-30% per point "
                       f"(quadrature point), random SPD Voigt stiffness (anisotropic); mean of {reps} "
                       "applies after one warm-up, HIP events",
           "extra_point_flops": {k: v for k, v in EXTRA_POINT_FLOPS.items() if k != "trilinear"}}
    for p in ps:
        mesh = syn.sheared_box_mesh(p)
        NE, q = mesh.num_elements, p + 2
        lam, mu = syn.two_material_lame(NE, seed=1)
        lq, mq = syn.quadrature_point_lame(lam, mu, q, seed=4)
        qp = np.stack([lq, mq], axis=-1)
        del lq, mq
        C = syn.random_spd_stiffness(NE, seed=5)
        c21 = np.ascontiguousarray(C[:, np.triu_indices(6)[0], np.triu_indices(6)[1]])
        rec = {}
        for dtype, dname in ((pa.PA_F64, "f64"), (pa.PA_F32, "f32")):
            word = 8 if dtype == pa.PA_F64 else 4
            forms = (("element_iso", lambda: pa.Operator(mesh, p, lam, mu, dtype=dtype), 0, 0),
                     ("qpoint_iso", lambda: pa.Operator.with_material(mesh, p, pa.PA_MAT_QP_ISO, qp, dtype=dtype),
                      2 * q ** 3, EXTRA_POINT_FLOPS["qpoint_iso"]),
                     ("anisotropic", lambda: pa.Operator.with_material(mesh, p, pa.PA_MAT_ANISO, c21, dtype=dtype),
                      21, EXTRA_POINT_FLOPS["anisotropic"]))
            for form, make, xw, xf in forms:
                op = make()
                t = _time_apply(torch, dev, op, reps)
                rec[f"{form}_{dname}"] = _rates(op.N, NE, p, word, dname, t, extra_words=xw, extra_flops_pt=xf)
                op.close()
        out[f"p{p}"] = rec
        del qp, C, c21
        torch.cuda.empty_cache()
    return out


def apply_geometry(torch, dev, ps=(1, 2, 4, 8), reps=10):
    """The fused apply on the sheared box with its interior vertices moved (trilinear
    hexahedra): geometry stored per quadrature point (J^{-1}, w det J) vs recomputed per
    point from 21 map coefficients per element, next to the affine box; HIP-event time
    per apply, FP64 and FP32, and rates against the peaks."""
    import synthetic as syn
    import paper_2601_08374_amd as pa
    out = {"workload": "sheared box (~4.2M dofs), q=p+2, two materials; interior vertices moved by up to "
                       f"0.2 of the spacing (seed 17); mean of {reps} applies after one warm-up, HIP events",
           "extra_point_flops": {"trilinear": EXTRA_POINT_FLOPS["trilinear"]}}
    for p in ps:
        mesh = syn.sheared_box_mesh(p)
        NE, q = mesh.num_elements, p + 2
        lam, mu = syn.two_material_lame(NE, seed=1)
        verts = syn.perturbed_vertices(mesh, amp=0.2, seed=17)
        rec = {}
        for dtype, dname in ((pa.PA_F64, "f64"), (pa.PA_F32, "f32")):
            word = 8 if dtype == pa.PA_F64 else 4
            forms = (("affine", lambda: pa.Operator(mesh, p, lam, mu, dtype=dtype), 0, 0),
                     ("qp_data", lambda: pa.Operator.with_geometry(mesh, p, verts, lam, mu,
                                                                   kind=pa.PA_GEOM_QP_DATA, dtype=dtype),
                      10 * q ** 3, 0),
                     ("trilinear", lambda: pa.Operator.with_geometry(mesh, p, verts, lam, mu,
                                                                     kind=pa.PA_GEOM_TRILINEAR, dtype=dtype),
                      21, EXTRA_POINT_FLOPS["trilinear"]))
            for form, make, xw, xf in forms:
                op = make()
                t = _time_apply(torch, dev, op, reps)
                rec[f"{form}_{dname}"] = _rates(op.N, NE, p, word, dname, t, extra_words=xw, extra_flops_pt=xf)
                op.close()
        out[f"p{p}"] = rec
        torch.cuda.empty_cache()
    return out


def apply_unstructured(torch, dev, ps=(1, 2, 4, 8), reps=10):
    """The fused apply on the distorted sheared box given as an unstructured mesh
    (explicit element-to-node map, every element in a random orientation), in box order
    and with elements and nodes shuffled at random (no locality), next to the structured
    trilinear operator on the same geometry; HIP-event time per apply, rates against the
    peaks (algorithmic bytes add the map, 4 (p+1)^3 bytes per element)."""
    import synthetic as syn
    import paper_2601_08374_amd as pa
    out = {"workload": "sheared box (~4.2M dofs), q=p+2, two materials, interior vertices moved by up to 0.2 "
                       "of the spacing; unstructured: random orientation per element, box order ('ordered') or "
                       f"random element and node order ('shuffled'); mean of {reps} applies after one warm-up"}
    for p in ps:
        mesh = syn.sheared_box_mesh(p)
        NE = mesh.num_elements
        lam, mu = syn.two_material_lame(NE, seed=1)
        verts = syn.perturbed_vertices(mesh, amp=0.2, seed=17)
        rec = {}
        hm, _, order = syn.box_as_unstructured(mesh, verts, p, seed=1, permute=False, renumber=False)
        hs, _, order_s = syn.box_as_unstructured(mesh, verts, p, seed=2, permute=True, renumber=False,
                                                 shuffle_nodes=True)
        mapb = 4 * (p + 1) ** 3 * NE
        for dtype, dname in ((pa.PA_F64, "f64"), (pa.PA_F32, "f32")):
            word = 8 if dtype == pa.PA_F64 else 4
            xf = EXTRA_POINT_FLOPS["trilinear"]
            forms = (("structured_trilinear", lambda: pa.Operator.with_geometry(
                          mesh, p, verts, lam, mu, kind=pa.PA_GEOM_TRILINEAR, dtype=dtype), 0),
                     ("unstructured_ordered", lambda: pa.Operator.unstructured(hm, lam[order], mu[order],
                                                                               dtype=dtype), mapb),
                     ("unstructured_shuffled", lambda: pa.Operator.unstructured(hs, lam[order_s], mu[order_s],
                                                                                dtype=dtype), mapb))
            for form, make, xb in forms:
                op = make()
                t = _time_apply(torch, dev, op, reps)
                rec[f"{form}_{dname}"] = _rates(op.N, NE, p, word, dname, t, extra_words=21, extra_bytes=xb,
                                                extra_flops_pt=xf)
                op.close()
        out[f"p{p}"] = rec
        del hm, hs
        torch.cuda.empty_cache()
    return out


def apply_ablation(torch, dev, ps=(1, 2, 4, 8), reps=5):
    """Cumulative ablation of the apply on the sheared box (FP64, q = p+2), in the order of the
    paper's ablation table: unfused dense baseline -> + sum factorization -> + Voigt stress ->
    + fusion into one kernel (quadrature-point data staged per element) -> + the slice-wise
    organisation (registers and LDS tiles; pointwise stage at the q^3 Gauss points) -> + the
    regrouped sums of the production apply (p = 1 closed form, p >= 2 collocation at the
    Gauss-Lobatto nodes).  HIP-event time per apply, with rates
    against the FP64 VALU and HBM peaks on the fused operator's FLOP and byte counts."""
    import synthetic as syn
    import paper_2601_08374_amd as pa
    names = [("unfused_dense", pa.capi.PA_VARIANT_UNFUSED_DENSE), ("unfused_sf", pa.capi.PA_VARIANT_UNFUSED_SF),
             ("unfused_sf_voigt", pa.capi.PA_VARIANT_UNFUSED_SF_VOIGT),
             ("fused_unstaged", pa.capi.PA_VARIANT_FUSED_UNSTAGED),
             ("fused_quadrature", pa.capi.PA_VARIANT_FUSED_QUADRATURE), ("fused", pa.capi.PA_VARIANT_FUSED)]
    out = {"workload": "sheared box (~4.2M dofs), FP64, q=p+2, two materials; mean of "
                       f"{reps} applies after one warm-up, HIP events"}
    stream = torch.cuda.current_stream()
    for p in ps:
        mesh = syn.sheared_box_mesh(p)
        lam, mu = syn.two_material_lame(mesh.num_elements, seed=1)
        op = pa.Operator(mesh, p, lam, mu, q=p + 2, dtype=pa.PA_F64)
        x = torch.tensor(syn.uniform_vector(op.N, 0), dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        rec, prev = {}, None
        for name, v in names:
            op.apply_variant(x, y, variant=v)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                op.apply_variant(x, y, variant=v)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            # rates on the fused operator's algorithmic FLOPs and bytes (the dense variant
            # executes O(p^6) FLOPs per element, the unfused ones move QVec arrays besides)
            r = _rates(op.N, mesh.num_elements, p, 8, "f64", t)
            if prev is not None:
                r["marginal_speedup"] = round(prev / t, 2)
            rec[name] = r
            prev = t
        rec["overall_speedup"] = round(rec["unfused_dense"]["us"] / rec["fused"]["us"], 1)
        out[f"p{p}"] = rec
        op.close()
        del x, y
        torch.cuda.empty_cache()
    return out
