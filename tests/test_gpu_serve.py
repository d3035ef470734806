"""Continuous batching on the GPU: every served result equals the same request solved
alone (within the solve tolerance), and both meet the FP64 true residual."""
import dataclasses

import numpy as np
import pytest

import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_alone_equals_mix(mode):
    from paper_2601_08374_amd.serve import KeepingExecutor, Scheduler, summarize
    reqs = syn.serving_stream(10, rate=2000.0, seed=3, n_lo=4, n_hi=9, ps=(2, 4))
    alone_ex = KeepingExecutor(mode=mode, slots=1)
    for r in reqs:
        Scheduler(alone_ex, slots=1).run([dataclasses.replace(r, arrival=0.0)])
    mix_ex = KeepingExecutor(mode=mode, slots=4)
    sched = Scheduler(mix_ex, slots=4, budget_bytes=8 << 30)
    recs = sched.run(reqs)
    assert sched.max_active > 1                 # solves were in flight together
    assert all(r.status == 0 for r in recs), [(r.rid, r.status, r.error) for r in recs]
    for r in recs:
        assert r.rel_res <= 1e-8 * 1.0001
        a, m = alone_ex.solutions[r.rid], mix_ex.solutions[r.rid]
        diff = np.linalg.norm(a - m) / np.linalg.norm(a)
        assert diff <= 1e-6, (r.rid, diff)
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
