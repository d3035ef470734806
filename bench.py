#!/usr/bin/env python3
"""Benchmark of the matrix-free PA elasticity apply (and, optionally, GMG-PCG solves).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--serve N]

Workload (one GPU): the operator-apply sweep on the globally sheared box --
(120/p,120/p,96/p) affine parallelepipeds (shear 0.2), ~4.2M dofs, q = p+2,
two materials per element (E = 1 and 100, nu = 0.3, seed 1), x ~ U[-1,1]
(seed 0).  One step applies the FP64 operator once at every p of the sweep
(p = 1, 2, 4, 6, 8); inputs are resident in HBM and every apply uses a
different buffer pair from a rotating set of >= 1 GB so that x and y stream
from HBM rather than the 256 MB last-level cache.

Printed: one short JSON line (the last line of stdout) with value = aggregate
FP64 apply throughput over the step (total dofs / wall time, GDoF/s), the
roofline of the dominant kernel (HIP-event timing of its launches inside the
timed region; p = 1 against the HBM roof, p >= 2 against the FP64 VALU roof in
the paper's FLOPs, with the FLOPs the regrouped kernels actually issue beside
them), the FP64 CPU oracle timed on a bounded sample, the per-p
FP64/FP32 apply sweep for p = 1..8 and brief solve and serving figures.  The
full results (sweep rates, ablation, material/geometry/unstructured forms,
solves, serving) go to the --detail file.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_F64_TFLOPS = 78.6     # MI355X vector FP64
PEAK_F32_TFLOPS = 157.3    # MI355X vector FP32
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E
# Degrees whose apply is bound by memory traffic: the p = 1 kernel evaluates the element's
# quadrature sums in closed form (about a tenth of the paper's FLOP count per element,
# about 5 FLOPs per algorithmic byte, below the ridge point of 9.8)
HBM_BOUND_PS = (1,)
STEP_PS = (1, 2, 4, 6, 8)

# HBM bytes per FP64 apply (apply kernel + skeleton kernel) from two rocprofv3
# --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Each counter is
# scaled by what it reads for a 256 MiB device-to-device copy: FETCH_SIZE reads
# 131088 KiB (factor 2.0), WRITE_SIZE 262144 KiB (factor 1.0).  Keyed by the
# source hash of the kernels they were taken on, so an edited kernel reports
# null until it is measured again.
MEASURED_TRAFFIC = {
    ("974d3442566f24cd", 1, "f64"): 298462418,
    ("974d3442566f24cd", 2, "f64"): 316217191,
    ("974d3442566f24cd", 4, "f64"): 199612569,
    ("974d3442566f24cd", 8, "f64"): 138049802,
}

# FP64 FLOPs the fused kernel issues per apply, from rocprofv3 SQ counters of the same
# runs: 64 lanes x (2 SQ_INSTS_VALU_FMA_F64 + ADD_F64 + MUL_F64) per wave x SQ_WAVES (idle
# lanes included).  The kernels regroup the paper's sums (closed form at p = 1, collocation
# at the Gauss-Lobatto nodes above), so they issue fewer FLOPs than F(p) counts.
MEASURED_ISSUED_FLOPS = {
    ("974d3442566f24cd", 1, "f64"): 64 * (2 * 1630 + 2174 + 1321) * 2028,
    ("974d3442566f24cd", 2, "f64"): 64 * (2 * 549 + 18 + 76) * 24686,
    ("974d3442566f24cd", 4, "f64"): 64 * (2 * 801 + 420 + 126) * 8640,
    ("974d3442566f24cd", 8, "f64"): 64 * (2 * 2301 + 828 + 226) * 4050,
}


def log(msg: str):
    """Progress line on stderr (the summary JSON is the last stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


from paper_2601_08374_amd.benchmarks import algorithmic_bytes, flops_per_element  # noqa: E402


KERNEL_SOURCES = ("internal.h", "apply_kernel.h", "apply_p1.hip")


def kernel_source_hash() -> str:
    """sha256 of the sources of the apply kernels (general kernel, linear-element kernel)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2601_08374_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def apply_kernel_names(p: int) -> str:
    """The two kernels of one FP64 apply at degree p (q = p + 2)."""
    if p == 1:
        return "pa_apply_lin_kernel<Q=3,double> + pa_lin_skeleton_kernel<double>"
    return f"pa_apply_kernel<P={p},Q={p + 1},double,collocated> + pa_skeleton_kernel<P={p},double>"


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ps, reps: int = 3):
    """Time the FP64 oracle apply (element-matrix GEMM + scatter) on the host cores.

    Sample: the first 1/8 of the sheared box of each p (n // 2 elements per axis, same
    element size, two materials, x ~ U[-1,1]).  Per p: element-matrix formation timed
    once, then one warm-up apply and the median of `reps` applies with the default thread
    pools, then the median of `reps` applies with every thread pool limited to one thread.
    `cores` is the number of threads the timed applies kept busy (process CPU time over
    wall time), `host_cores` the cores the process may run on."""
    import numpy as np
    import synthetic as syn
    from oracle import elasticity
    from threadpoolctl import threadpool_limits

    host_cores = len(os.sched_getaffinity(0))
    res = {}
    tot_dofs = tot_t = tot_t1 = 0.0
    cpu_s = wall_s = 0.0
    for p in ps:
        sub = _sub_box(syn.sheared_box_mesh(p), 2)
        lam, mu = syn.two_material_lame(sub.num_elements, seed=1)
        t0 = time.perf_counter()
        op = elasticity.Operator(sub, p, p + 2, lam, mu)
        t_setup = time.perf_counter() - t0
        x = syn.uniform_vector(op.N, 0)
        op.apply(x)                                   # warm-up
        ts = []
        for _ in range(reps):
            c0, t0 = time.process_time(), time.perf_counter()
            op.apply(x)
            ts.append(time.perf_counter() - t0)
            cpu_s += time.process_time() - c0
            wall_s += ts[-1]
        t = float(np.median(ts))
        with threadpool_limits(limits=1):
            t1s = []
            for _ in range(reps):
                t0 = time.perf_counter()
                op.apply(x)
                t1s.append(time.perf_counter() - t0)
        t1 = float(np.median(t1s))
        res[p] = {"gdofs": op.N / t / 1e9, "gdofs_1thread": op.N / t1 / 1e9, "t_apply_s": t,
                  "t_apply_1thread_s": t1, "t_setup_s": t_setup, "N": op.N, "n": list(sub.n)}
        tot_dofs += op.N
        tot_t += t
        tot_t1 += t1
        del op
    return {"value": tot_dofs / tot_t / 1e9, "unit": "GDoF/s", "cores": max(1, round(cpu_s / wall_s)),
            "host_cores": host_cores, "cpu_model": cpu_model(), "kind": "oracle",
            "value_1thread": tot_dofs / tot_t1 / 1e9,
            "sample": "FP64 oracle apply (batched element-matrix GEMM + scatter) on the first 1/8 of the "
                      f"sheared box at each p in {list(ps)} (n//2 elements per axis, ~0.5M dofs each); one "
                      f"warm-up, median of {reps}; also with thread pools limited to 1; element-matrix "
                      "formation timed separately",
            "per_p": res}


def _sub_box(mesh, f: int = 4):
    """The first 1/f^3 of a box (n // f elements per axis, same element size): the bounded
    sample the oracle of a general form is timed on."""
    import synthetic as syn
    n = tuple(max(1, k // f) for k in mesh.n)
    L = tuple(mesh.L[a] * n[a] / mesh.n[a] for a in range(3))
    return syn.BoxMesh(n=n, L=L, A=mesh.A, x0=mesh.x0)


def _oracle_rate(build, N: int):
    """GDoF/s of one FP64 oracle apply (setup excluded) of a sample with N dofs."""
    import synthetic as syn
    op = build()
    x = syn.uniform_vector(N, 0)
    t0 = time.perf_counter()
    op.apply(x)
    t = time.perf_counter() - t0
    return {"gdofs": N / t / 1e9, "t_apply_s": round(t, 4), "N": N}


def cpu_baseline_forms(section: str, ps=(1, 2, 4, 8)):
    """The FP64 oracle of one general form (material data, trilinear geometry, unstructured
    mesh) timed on the host cores, at each p on the first 1/64 of the sheared box: the
    same inputs as the GPU section of that name, restricted to the sample."""
    import synthetic as syn
    from oracle import geometry, material
    notes = {"material": "material (strain-displacement form)",
             "geometry": "trilinear-geometry (quadrature sum with per-point Jacobians)",
             "unstructured": "unstructured-mesh (quadrature sum, explicit map)"}
    out = {"kind": "oracle", "cores": len(os.sched_getaffinity(0)), "unit": "GDoF/s",
           "sample": f"one FP64 {notes[section]} oracle apply at each p on the first 1/64 of the sheared "
                     "box (n // 4 elements per axis, same element size), setup excluded"}
    for p in ps:
        mesh = syn.sheared_box_mesh(p)
        NE, q = mesh.num_elements, p + 2
        lam, mu = syn.two_material_lame(NE, seed=1)
        sub = _sub_box(mesh)
        ns = sub.num_elements
        if section == "material":
            C = syn.random_spd_stiffness(NE, seed=5)[:ns]
            Cs = material.isotropic_voigt(*syn.quadrature_point_lame(lam[:ns], mu[:ns], q, seed=4))
            out[f"p{p}"] = {"qpoint_iso": _oracle_rate(lambda: material.GeneralOperator(sub, p, q, Cs),
                                                       sub.num_dofs(p)),
                            "anisotropic": _oracle_rate(lambda: material.GeneralOperator(sub, p, q, C),
                                                        sub.num_dofs(p))}
        elif section == "geometry":
            sv = syn.perturbed_vertices(sub, amp=0.2, seed=17)
            out[f"p{p}"] = _oracle_rate(lambda: geometry.TrilinearOperator(sub, p, q, sv, lam[:ns], mu[:ns]),
                                        sub.num_dofs(p))
        else:
            sv = syn.perturbed_vertices(sub, amp=0.2, seed=17)
            hsub, _, osub = syn.box_as_unstructured(sub, sv, p, seed=1, permute=False, renumber=False)
            out[f"p{p}"] = _oracle_rate(lambda: geometry.UnstructuredOperator(hsub, q, lam[osub], mu[osub]),
                                        hsub.num_dofs)
    return out


def measured_ceilings(torch, dev, reps: int = 5):
    """Attainable rates measured on the device: vector FMA throughput in FP64 and FP32
    (pa_probe_fma, 8 independent chains per lane) and a plain 1 GiB device-to-device copy
    (torch; 2 GiB moved per copy).  HIP events on the current stream."""
    import ctypes as C
    from paper_2601_08374_amd import capi
    stream = torch.cuda.current_stream()
    out = {}

    def timed(fn):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    blocks, iters = 256 * 32, 2048
    for dname, dtype, tdt in (("f64", 0, torch.float64), ("f32", 1, torch.float32)):
        buf = torch.empty(blocks * 256, dtype=tdt, device=dev)
        t = timed(lambda: capi.check(capi.pa_probe_fma(C.c_void_p(buf.data_ptr()), dtype, blocks, iters,
                                                       C.c_void_p(stream.cuda_stream))))
        out[f"fma_{dname}_tflops"] = round(4096 * blocks * iters / t / 1e12, 2)
        del buf
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    t = timed(lambda: b.copy_(a))
    out["copy_gbs"] = round(2 * 8 * n / t / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def _r(v, nd=3):
    return None if v is None else round(float(v), nd)


def _sig(v, n=3):
    """v to n significant digits."""
    return None if v is None else float(f"{float(v):.{n}g}")


def compact_summary(res: dict) -> dict:
    """The one-line result (well under 2 KB): the contract fields, the roofline of the
    dominant kernel, the CPU baseline, and per-p FP64/FP32 apply GDoF/s; solve and serving
    figures in brief.  Everything else stays in the detail file."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
            "scaling", "vs_baseline", "dtype", "data")
    out = {k: res[k] for k in keys if k in res}
    cfg = res["config"]
    dofs = {str(p): n for p, n in cfg["dofs"].items()}
    out["config"] = {"workload": cfg["workload"][:180], "parallelism": cfg["parallelism"],
                     "dofs": next(iter(dofs.values())) if len(set(dofs.values())) == 1 else dofs}
    rf = res["roofline"]
    out["roofline"] = {k: rf[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                          "flops_per_launch", "issued_flops_per_launch", "frac_issued",
                                          "algorithmic_bytes_per_launch", "launch_us",
                                          "measured_peak", "frac_measured") if k in rf}
    out["step_per_p_gdofs"] = {str(p): _r(v, 1) for p, v in res["step_per_p_gdofs"].items()}
    cb = res.get("cpu_baseline")
    if cb:
        out["cpu_baseline"] = {"value": _sig(cb["value"]), "unit": cb["unit"], "cores": cb["cores"],
                               "host_cores": cb["host_cores"], "cpu_model": cb["cpu_model"].strip()[:48],
                               "kind": cb["kind"], "value_1thread": _sig(cb["value_1thread"]),
                               "sample": "oracle FP64 apply on the first 1/8 of each step box, median of 3",
                               "per_p": {str(p): _sig(v["gdofs"]) for p, v in cb["per_p"].items()}}
    sw = res.get("sweep")
    if sw:
        out["sweep_gdofs"] = {d: {str(p): _r(sw[p][d]["gdofs"], 1) for p in sw} for d in ("f64", "f32")}
        out["sweep_frac_f64"] = {str(p): _r(sw[p]["f64"]["frac_hbm" if p in HBM_BOUND_PS else "frac_alu_peak"], 3)
                                 for p in sw}
        out["sweep_roof"] = "p1 hbm bytes, p2-8 fp64 valu paper flops"
    sv = res.get("solve")
    if sv:
        out["solve_ms"] = {k[1:]: {m: _r(v[m]["solve_s"] * 1e3, 1) for m in ("f64", "f32_prec", "f32_ir") if m in v}
                           for k, v in sv.items() if k.startswith("p") and k[1:].isdigit()}
    se = res.get("serve")
    if se:
        out["serve"] = {m: {"solves_per_s": _r(se[m]["solves_per_s"], 2), "p50_s": _r(se[m]["p50_latency_s"], 3),
                            "p99_s": _r(se[m]["p99_latency_s"], 3)} for m in ("f64", "f32_ir", "f32_prec") if m in se}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rotate-gb", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every timing of the oracle on the host")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the cantilever GMG-PCG solves")
    ap.add_argument("--no-ablation", action="store_true", help="skip the unfused apply variants")
    ap.add_argument("--no-material", action="store_true", help="skip the general material data forms")
    ap.add_argument("--no-geometry", action="store_true", help="skip the non-affine geometry forms")
    ap.add_argument("--no-unstructured", action="store_true", help="skip the unstructured-mesh apply")
    ap.add_argument("--serve", type=int, default=512,
                    help="requests in the serving stream (0 skips it)")
    ap.add_argument("--profile-apply", type=int, default=0, metavar="P",
                    help="profiling mode: only run --reps applies of the degree-P sheared-box operator "
                         "(then three 256 MiB copies that calibrate the traffic counters) and exit")
    ap.add_argument("--profile-solve", type=int, default=0, metavar="P",
                    help="profiling mode: build the degree-P cantilever hierarchy, run one GMG-PCG solve "
                         "(--solve-mode) to rtol 1e-8 and exit")
    ap.add_argument("--profile-setup", action="store_true",
                    help="profiling mode: build the FP64 GMG hierarchy (Chebyshev(3), automatic h-levels) of "
                         "three serving-sized boxes --reps times each, print the setup times and exit")
    ap.add_argument("--solve-mode", choices=("f64", "f32_ir", "f32_prec"), default="f64")
    ap.add_argument("--dtype", choices=("f64", "f32"), default="f64")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--detail", default=os.path.join(tempfile.gettempdir(), "paelast_bench_detail.json"),
                    help="file for the full results (the stdout line is a summary); empty: none")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU implementation: --gpus must be 1 (the partition of the mesh "
                                   "over several GPUs is not implemented)", "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import synthetic as syn
    import paper_2601_08374_amd as pa

    pa.capi.load()   # fails loudly when the HIP library is missing
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 3
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def make(p, dtype):
        mesh = syn.sheared_box_mesh(p)
        lam, mu = syn.two_material_lame(mesh.num_elements, seed=1)
        op = pa.Operator(mesh, p, lam, mu, q=p + 2, dtype=dtype)
        tdt = torch.float64 if dtype == pa.PA_F64 else torch.float32
        x0 = torch.tensor(syn.uniform_vector(op.N, 0), dtype=tdt, device=dev)
        word = 8 if dtype == pa.PA_F64 else 4
        K = max(1, int(np.ceil(args.rotate_gb * 1e9 / (2 * word * op.N))))
        xs = [x0.clone() for _ in range(K)]
        ys = [torch.empty_like(x0) for _ in range(K)]
        return dict(op=op, xs=xs, ys=ys, N=op.N, NE=mesh.num_elements, word=word, p=p, dtype=dtype)

    if args.profile_apply:
        s = make(args.profile_apply, pa.PA_F64 if args.dtype == "f64" else pa.PA_F32)
        K = len(s["xs"])
        for i in range(args.reps):
            s["op"].apply(s["xs"][i % K], s["ys"][i % K])
        a = torch.empty(32 << 20, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_apply": args.profile_apply, "dtype": args.dtype, "reps": args.reps,
                          "N": s["N"], "NE": s["NE"], "calibration_copy_bytes": a.numel() * 8}), flush=True)
        return 0

    if args.profile_solve:
        p = args.profile_solve
        mesh = syn.cantilever_mesh(80, 8, 8)
        lam, mu = (float(v) for v in syn.lame_from_young_poisson(1.0, 0.3))
        op = pa.Operator(mesh, p, np.full(mesh.num_elements, lam), np.full(mesh.num_elements, mu))
        b = op.rhs((0.0, 0.0, 0.0), 1, (0.0, 0.0, -1.0))
        mode = {"f64": pa.PA_SOLVE_F64, "f32_ir": pa.PA_SOLVE_F32_IR, "f32_prec": pa.PA_SOLVE_F32_PREC}[args.solve_mode]
        H = op.hierarchy(mode=mode, stop=pa.PA_STOP_TRUE, cheb_degree=3, h_levels=2)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info, rc = H.pcg(b, x, rtol=1e-8)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        print(json.dumps({"profile_solve": p, "mode": args.solve_mode, "rc": rc, "iters": info.iters,
                          "outer": info.outer_iters, "rel_res_true": info.rel_res_true, "solve_s": t,
                          "N": op.N}), flush=True)
        return 0

    if args.profile_setup:
        out = []
        for n, p in (((9, 9, 9), 2), ((17, 25, 30), 4), ((32, 32, 32), 8)):
            mesh = syn.BoxMesh(n=n, L=tuple(v / 32 for v in n), clamped_faces=1)
            NE = mesh.num_elements
            lam, mu = (float(v) for v in syn.lame_from_young_poisson(10.0, 0.3))
            op = pa.Operator(mesh, p, np.full(NE, lam), np.full(NE, mu))
            ts = []
            for _ in range(args.reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                H = op.hierarchy(mode=pa.PA_SOLVE_F64, stop=pa.PA_STOP_TRUE, cheb_degree=3)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                nc = H.level_info(H.num_levels - 1)["N"]
                H.close()
            op.close()
            out.append({"n": n, "p": p, "N": op.N, "coarse_N": nc, "setup_ms_min": round(1e3 * min(ts), 2),
                        "setup_ms_median": round(1e3 * float(np.median(ts)), 2)})
        print(json.dumps({"profile_setup": out, "reps": args.reps}), flush=True)
        return 0

    # ---------------- timed step: FP64 apply at every p of the sweep
    setups = {p: make(p, pa.PA_F64) for p in STEP_PS}
    ctr = {p: 0 for p in STEP_PS}

    def step(events=None):
        for p in STEP_PS:
            s = setups[p]
            i = ctr[p] % len(s["xs"])
            ctr[p] += 1
            if events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                s["op"].apply(s["xs"][i], s["ys"][i])
                e1.record(stream)
                events[p].append((e0, e1))
            else:
                s["op"].apply(s["xs"][i], s["ys"][i])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = {p: [] for p in STEP_PS}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(events)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_p_ms = {p: float(np.mean([a.elapsed_time(b) for a, b in events[p]])) for p in STEP_PS}
    log(f"timed step done: {args.steps} steps in {wall:.3f} s")
    total_dofs = args.steps * sum(setups[p]["N"] for p in STEP_PS)
    value = total_dofs / wall / 1e9

    # dominant kernel of the step and its roofline
    pdom = max(STEP_PS, key=lambda p: per_p_ms[p])
    sd = setups[pdom]
    t_launch = per_p_ms[pdom] * 1e-3
    flops = flops_per_element(pdom) * sd["NE"]
    abytes = algorithmic_bytes(sd["N"], sd["NE"], 8)
    src_hash = kernel_source_hash()
    tr = MEASURED_TRAFFIC.get((src_hash, pdom, "f64"))
    roofline = {"traffic": tr, "kernel": apply_kernel_names(pdom), "flops_per_launch": flops,
                "algorithmic_bytes_per_launch": abytes, "launch_us": round(t_launch * 1e6, 2),
                "source_hash": src_hash}
    if pdom in HBM_BOUND_PS:
        achieved = abytes / t_launch / 1e9
        roofline.update({"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(achieved / PEAK_HBM_GBS, 4)})
    else:
        achieved = flops / t_launch / 1e12
        roofline.update({"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_F64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_F64_TFLOPS, 4),
                         "hbm_gbs": round(abytes / t_launch / 1e9, 1)})

    issued = MEASURED_ISSUED_FLOPS.get((src_hash, pdom, "f64"))
    roofline["issued_flops_per_launch"] = issued
    roofline["frac_issued"] = None if issued is None else round(issued / t_launch / 1e12 / PEAK_F64_TFLOPS, 4)

    log("measured ceilings (FMA probe, copy)")
    ceilings = measured_ceilings(torch, dev)
    ceil = ceilings["copy_gbs"] if pdom in HBM_BOUND_PS else ceilings["fma_f64_tflops"]
    roofline["measured_peak"] = ceil
    roofline["frac_measured"] = round(achieved / ceil, 4)

    result = {
        "metric": "PA apply GDoF/s at p=1..8 (FP64 vs FP32); GMG-PCG solves/s + p99 latency",
        "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "FP64 apply at p=1,2,4,6,8 on the sheared box (shear 0.2), (120/p,120/p,96/p) "
                               "elements, ~4.2M dofs, q=p+2, E in {1,100} nu=0.3 seed 1, x~U[-1,1] seed 0, "
                               "cold buffers",
                   "dofs": {p: setups[p]["N"] for p in STEP_PS}, "parallelism": "single GPU"},
        "step_per_p_gdofs": {p: round(setups[p]["N"] / (per_p_ms[p] * 1e-3) / 1e9, 3) for p in STEP_PS},
        "roofline": roofline,
        "ceilings": ceilings,
    }
    for p in STEP_PS:
        for k in ("xs", "ys"):
            setups[p][k] = None
    del setups
    torch.cuda.empty_cache()

    # ---------------- per-p sweep FP64 / FP32, p = 1..8 (outside the timed step)
    if not args.no_sweep:
        sweep = {}
        for p in range(1, 9):
            log(f"sweep p={p}")
            sweep[p] = {}
            for dtype, name, peak in ((pa.PA_F64, "f64", PEAK_F64_TFLOPS), (pa.PA_F32, "f32", PEAK_F32_TFLOPS)):
                s = make(p, dtype)
                K = len(s["xs"])
                for i in range(3):
                    s["op"].apply(s["xs"][i % K], s["ys"][i % K])
                reps = max(20, 2 * K)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for i in range(reps):
                    s["op"].apply(s["xs"][i % K], s["ys"][i % K])
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) * 1e-3 / reps
                # hot: one buffer pair, resident in the last-level cache
                e0.record(stream)
                for i in range(reps):
                    s["op"].apply(s["xs"][0], s["ys"][0])
                e1.record(stream)
                torch.cuda.synchronize()
                th = e0.elapsed_time(e1) * 1e-3 / reps
                fl = flops_per_element(p) * s["NE"]
                by = algorithmic_bytes(s["N"], s["NE"], s["word"])
                sweep[p][name] = {"bound": "hbm" if p in HBM_BOUND_PS else "alu",
                                  "gdofs": round(s["N"] / t / 1e9, 3), "gdofs_hot": round(s["N"] / th / 1e9, 3),
                                  "us": round(t * 1e6, 2), "tflops": round(fl / t / 1e12, 3),
                                  "frac_alu_peak": round(fl / t / 1e12 / peak, 4),
                                  "frac_alu_measured": round(fl / t / 1e12 / ceilings[f"fma_{name}_tflops"], 4),
                                  "gbs": round(by / t / 1e9, 1), "frac_hbm": round(by / t / 1e9 / PEAK_HBM_GBS, 4),
                                  "N": s["N"]}
                del s
                torch.cuda.empty_cache()
        result["sweep"] = sweep

    if not args.no_ablation:
        log("apply ablation")
        from paper_2601_08374_amd import benchmarks
        result["ablation"] = benchmarks.apply_ablation(torch, dev)
    if not args.no_material:
        log("apply with general material data")
        from paper_2601_08374_amd import benchmarks
        result["material"] = benchmarks.apply_material(torch, dev)
    if not args.no_geometry:
        log("apply on non-affine geometry")
        from paper_2601_08374_amd import benchmarks
        result["geometry"] = benchmarks.apply_geometry(torch, dev)
    if not args.no_unstructured:
        log("apply on unstructured meshes")
        from paper_2601_08374_amd import benchmarks
        result["unstructured"] = benchmarks.apply_unstructured(torch, dev)
    if not args.no_solve:
        log("cantilever solves")
        from paper_2601_08374_amd import benchmarks
        result["solve"] = benchmarks.cantilever_solves(torch, dev)
    if args.serve:
        log(f"serving stream of {args.serve} requests")
        from paper_2601_08374_amd import serve
        result["serve"] = serve.bench_stream(args.serve)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(STEP_PS)
        for section in ("material", "geometry", "unstructured"):
            if section in result:
                log(f"cpu baseline (oracle), {section}")
                result[section]["cpu_oracle"] = cpu_baseline_forms(section)
    detail = args.detail
    if detail:
        try:
            os.makedirs(os.path.dirname(os.path.abspath(detail)), exist_ok=True)
            with open(detail, "w") as fh:
                json.dump(result, fh, indent=1)
            log(f"full results written to {detail}")
        except OSError as exc:
            log(f"could not write {detail}: {exc}")
    line = json.dumps(compact_summary(result), separators=(",", ":"))
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
