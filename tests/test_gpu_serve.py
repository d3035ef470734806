"""Continuous batching on the GPU: every served result is bitwise the same request solved
alone, and meets the FP64 true residual evaluated by the oracle."""
import dataclasses

import numpy as np
import pytest

import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


_ORACLE = {}
EPS64 = float(np.finfo(np.float64).eps)


def _oracle_system(ex, req):
    """The oracle's operator and load vector of a served request (box, clamped x = 0, its
    E, nu and constant body force), built once per request."""
    if req.rid not in _ORACLE:
        from oracle import elasticity
        mesh = ex.mesh_of(req)
        lam, mu = syn.lame_from_young_poisson(req.E, req.nu)
        op = elasticity.Operator(mesh, req.p, req.p + 2, float(lam), float(mu))
        b = elasticity.body_force_vector(mesh, req.p, req.p + 2, np.asarray(req.f))
        b[op.ess] = 0.0
        _ORACLE[req.rid] = (op, b)
    return _ORACLE[req.rid]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_alone_equals_mix(mode):
    """A stream of boxes of p in {2, 4, 6, 8} and 4..8 elements per axis, served with four
    slots: each result is bitwise the result of the same request served alone (every
    reduction of setup and solve has a fixed order, and iterations enqueued after a solve
    met its stopping test do nothing), and each served solution's true residual, evaluated
    by the oracle's own FP64 apply, meets rtol 1e-8 within the rounding scale of that
    evaluation (eps times the magnitudes of its terms, |b| + sum_e |K^e| |x|)."""
    from paper_2601_08374_amd.serve import KeepingExecutor, Scheduler, summarize
    reqs = syn.serving_stream(12, rate=2000.0, seed=3, n_lo=4, n_hi=8, ps=(2, 4, 6, 8))
    assert {r.p for r in reqs} == {2, 4, 6, 8}
    alone_ex = KeepingExecutor(mode=mode, slots=1)
    for r in reqs:
        Scheduler(alone_ex, slots=1).run([dataclasses.replace(r, arrival=0.0)])
    mix_ex = KeepingExecutor(mode=mode, slots=4)
    sched = Scheduler(mix_ex, slots=4, budget_bytes=8 << 30)
    recs = sched.run(reqs)
    assert sched.max_active > 1                 # solves were in flight together
    assert all(r.status == 0 for r in recs), [(r.rid, r.status, r.error) for r in recs]
    for req, r in zip(reqs, recs):
        assert r.rel_res <= 1e-8 * (1 + 1e-12)
        a, m = alone_ex.solutions[r.rid], mix_ex.solutions[r.rid]
        assert np.array_equal(a, m), (r.rid, np.abs(a - m).max())
        op, b = _oracle_system(mix_ex, req)
        nb = np.linalg.norm(b)
        res = np.linalg.norm(b - op.apply(m, constrained=True)) / nb
        scale = EPS64 * np.linalg.norm(np.abs(b) + op.abs_apply(np.abs(m), constrained=True)) / nb
        print(f"  request {r.rid}: n={req.n} p={req.p} iters {r.iters} GPU res {r.rel_res:.2e} "
              f"oracle res {res:.2e} (rounding {scale:.1e})", flush=True)
        assert res <= 1e-8 + scale, (r.rid, res, scale)
        assert abs(res - r.rel_res) <= 2 * scale, (r.rid, res, r.rel_res, scale)
    s = summarize(recs)
    print("mode", mode, s, flush=True)


def test_budget_limited_admission_on_gpu():
    from paper_2601_08374_amd.serve import GpuExecutor, Scheduler
    reqs = syn.serving_stream(6, rate=1e6, seed=4, n_lo=6, n_hi=6, ps=(2,))   # equal sizes
    ex = GpuExecutor(mode=0, slots=4)
    need = max(ex.bytes_required(r) for r in reqs)
    sched = Scheduler(ex, slots=4, budget_bytes=int(1.5 * need))   # room for one solve at a time
    recs = sched.run(reqs)
    assert all(r.status == 0 for r in recs)
    assert sched.max_active == 1
    assert sched.max_used <= 1.5 * need
