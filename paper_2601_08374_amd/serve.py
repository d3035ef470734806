"""Continuous-batching request loop for elasticity solves on one GPU.

Requests (box meshes of different sizes and orders) arrive over time.  The
scheduler admits them in arrival order while a slot is free and the HBM budget
covers the request's operator + hierarchy (``pa_bytes_required``), keeps every
admitted solve's operators and Krylov state on the device, and advances all of
them through the step API (``gmg_pcg_step`` / ``gmg_pcg_poll``) so that solves
admitted at different times overlap on the device, each on its own stream.
Completed solves free their memory and slot immediately, which admits the next
waiting request.  Admission is strictly FIFO (a request that does not fit
blocks later ones), so no request starves.

The scheduler is pure host logic over an injected executor; ``GpuExecutor``
is the real one (all arithmetic in the HIP library), tests use a fake.
"""
from __future__ import annotations

import collections
import ctypes as C
import dataclasses
import time
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Record:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    status: int = 0
    iters: int = 0
    outer: int = 0
    rel_res: float = float("nan")
    ndofs: int = 0
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """FIFO admission by slot and memory budget; round-robin stepping of active solves."""

    def __init__(self, executor, slots: int = 8, budget_bytes: int = 64 << 30, iters_per_step: int = 2,
                 clock=time.perf_counter, idle_sleep: float = 0.0):
        self.ex = executor
        self.slots = slots
        self.budget = budget_bytes
        self.k = iters_per_step
        self.clock = clock
        self.idle_sleep = idle_sleep
        self.max_used = 0
        self.max_active = 0

    def run(self, requests, time_scale: float = 1.0):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        records = {r.rid: Record(r.rid, r.arrival * time_scale) for r in requests}
        active = []
        used = 0
        free_slots = list(range(self.slots))
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            # admission, in arrival order
            while pending and pending[0].arrival * time_scale <= now and free_slots:
                req = pending[0]
                rec = records[req.rid]
                try:
                    need = int(self.ex.bytes_required(req))
                except Exception as e:          # invalid request: reject, do not block the queue
                    pending.popleft()
                    rec.error, rec.status, rec.finished = str(e), -1, self.clock() - t0
                    continue
                if need < 0 or need > self.budget:
                    pending.popleft()
                    rec.error, rec.status, rec.finished = f"needs {need} bytes > budget", -2, self.clock() - t0
                    continue
                if used + need > self.budget:
                    break                       # wait for memory; later requests may not overtake
                pending.popleft()
                slot = free_slots.pop(0)
                try:
                    h = self.ex.start(req, slot)
                except Exception as e:
                    free_slots.append(slot)
                    rec.error, rec.status, rec.finished = str(e), -3, self.clock() - t0
                    continue
                used += need
                self.max_used = max(self.max_used, used)
                rec.admitted = self.clock() - t0
                rec.ndofs = getattr(h, "ndofs", 0)
                active.append((req, h, need, slot))
            self.max_active = max(self.max_active, len(active))
            progressed = False
            for (req, h, need, slot) in active:
                self.ex.step(h, self.k)
            still = []
            for (req, h, need, slot) in active:
                done, status = self.ex.poll(h)
                if not done:
                    still.append((req, h, need, slot))
                    continue
                progressed = True
                rec = records[req.rid]
                info = self.ex.finish(h)
                rec.finished = self.clock() - t0
                rec.status = status
                rec.iters, rec.outer, rec.rel_res = info.get("iters", 0), info.get("outer", 0), info.get("rel_res", 0)
                self.ex.release(h)
                used -= need
                free_slots.append(slot)
            active = still
            if not progressed and self.idle_sleep:
                time.sleep(self.idle_sleep)
        return [records[r.rid] for r in requests]


def summarize(records, makespan: Optional[float] = None):
    ok = [r for r in records if r.status == 0 and r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    if makespan is None:
        makespan = max((r.finished for r in records), default=0.0) - min((r.arrival for r in records), default=0.0)
    return {"solves": len(ok), "failed": len(records) - len(ok), "makespan_s": makespan,
            "solves_per_s": len(ok) / makespan if makespan > 0 else None,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_iters": float(np.mean([r.iters for r in ok])) if ok else None,
            "max_rel_res": float(max((r.rel_res for r in ok), default=0.0))}


class _Handle:
    __slots__ = ("op", "H", "b", "x", "solve", "ndofs", "stream", "req")


class GpuExecutor:
    """Runs each request on its own HIP stream through the C step API."""

    def __init__(self, mode: int = 0, rtol: float = 1e-8, cheb_degree: int = 3, slots: int = 8,
                 element_size: float = 1.0 / 32):
        import torch

        import paper_2601_08374_amd as pa
        self.torch, self.pa, self.cap = torch, pa, pa.capi
        self.mode, self.rtol, self.k = mode, rtol, cheb_degree
        self.h = element_size
        self.streams = [torch.cuda.Stream() for _ in range(slots)]

    def mesh_of(self, req):
        import synthetic as syn
        n = tuple(int(v) for v in req.n)
        return syn.BoxMesh(n=n, L=tuple(v * self.h for v in n), clamped_faces=1)

    def bytes_required(self, req):
        mesh = self.mesh_of(req)
        ms, keep = self.pa.mesh_struct(mesh)
        dt = self.pa.PA_F32 if self.mode == self.pa.PA_SOLVE_F32_IR else self.pa.PA_F64
        nb = self.cap.load().pa_bytes_required(C.byref(ms), int(req.p), dt, 1)
        if nb < 0:
            raise ValueError(self.cap.load().pa_last_error().decode())
        # plus the caller-owned FP64 b and x
        return nb + 2 * 8 * mesh.num_dofs(int(req.p))

    def start(self, req, slot):
        import synthetic as syn
        torch, pa, cap = self.torch, self.pa, self.cap
        h = _Handle()
        h.req = req
        h.stream = self.streams[slot % len(self.streams)]
        mesh = self.mesh_of(req)
        NE = mesh.num_elements
        lam, mu = syn.lame_from_young_poisson(req.E, req.nu)
        with torch.cuda.stream(h.stream):
            h.op = pa.Operator(mesh, int(req.p), np.full(NE, float(lam)), np.full(NE, float(mu)),
                               stream=h.stream)
            h.H = pa.Hierarchy(h.op, mode=self.mode, stop=pa.PA_STOP_TRUE, cheb_degree=self.k)
            h.b = h.op.rhs(tuple(req.f))
            h.x = torch.zeros_like(h.b)
            s = C.c_void_p()
            cap.check(cap.gmg_pcg_begin(h.H.handle, C.c_void_p(h.b.data_ptr()), C.c_void_p(h.x.data_ptr()),
                                        float(self.rtol), C.byref(s)))
        h.solve = s
        h.ndofs = h.op.N
        return h

    def step(self, h, n):
        self.cap.check(self.cap.gmg_pcg_step(h.solve, int(n)))

    def poll(self, h):
        d, st = C.c_int(), C.c_int()
        self.cap.check(self.cap.gmg_pcg_poll(h.solve, C.byref(d), C.byref(st)))
        return bool(d.value), int(st.value)

    def finish(self, h):
        info = self.cap.pa_solve_info_t()
        self.cap.gmg_pcg_end(h.solve, C.byref(info))
        h.solve = None
        return {"iters": info.iters, "outer": info.outer_iters, "rel_res": info.rel_res_true}

    def release(self, h):
        h.stream.synchronize()
        h.H.close()
        h.op.close()
        h.b = h.x = None


class KeepingExecutor(GpuExecutor):
    """GpuExecutor that keeps each solution on the host (for tests)."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.solutions = {}

    def finish(self, h):
        out = super().finish(h)
        self.solutions[h.req.rid] = h.x.cpu().numpy()
        return out


def bench_stream(num: int = 64, seed: int = 5, slots: int = 8, budget_gb: float = 64.0, n_hi: int = 32,
                 rate: Optional[float] = None):
    """Serving benchmark: closed-loop capacity on a strided sample of the stream, then Poisson
    arrivals at 0.8x it, for FP32+refinement, FP64 PCG with the FP32 V-cycle, and plain FP64."""
    import synthetic as syn
    import paper_2601_08374_amd as pa
    out = {"requests": num, "slots": slots, "budget_gb": budget_gb, "rtol": 1e-8, "n_range": [4, n_hi],
           "p_choices": [2, 4, 6, 8]}
    for mode, name in ((pa.PA_SOLVE_F32_IR, "f32_ir"), (pa.PA_SOLVE_F32_PREC, "f32_prec"), (pa.PA_SOLVE_F64, "f64")):
        ex = GpuExecutor(mode=mode, slots=slots)
        reqs = syn.serving_stream(num, rate=1.0, seed=seed, n_hi=n_hi)
        sched = Scheduler(ex, slots=slots, budget_bytes=int(budget_gb * (1 << 30)))
        r0 = rate
        if r0 is None:
            # every k-th request (64 of them at most): the sizes of the whole stream, whose early
            # requests happen to be smaller than its mean
            sample = reqs[:: max(1, num // 64)][:64]
            closed = [dataclasses.replace(r, arrival=0.0) for r in sample]
            t0 = time.perf_counter()
            recs = sched.run(closed)
            cap_rate = len(sample) / (time.perf_counter() - t0)
            r0 = 0.8 * cap_rate
            out[f"{name}_closed_loop_solves_per_s"] = cap_rate
        reqs = syn.serving_stream(num, rate=r0, seed=seed, n_hi=n_hi)
        t0 = time.perf_counter()
        recs = sched.run(reqs)
        makespan = time.perf_counter() - t0
        s = summarize(recs, makespan)
        s["arrival_rate"] = r0
        s["max_active"] = sched.max_active
        out[name] = s
    return out
