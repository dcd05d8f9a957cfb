"""Serving with continuous batching: runs admitted into a resident pool as
memory frees up, stepped together, retired when done.  Each result must be
bit-identical to the same run stepped alone."""

import numpy as np
import pytest

from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import serve as SV
from paper_1704_01202_amd import workloads as W
from tests.test_gpu_parity import ctx, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_served_runs_match_runs_alone(ctx):
    trace = W.config_c5_trace(seed=7, n_requests=7, rate=400.0, size_lo=2e3, size_hi=2e4,
                              cells_lo=2, cells_hi=12, steps_lo=4, steps_hi=11)
    # a small pool: the runs cannot all be resident at once
    pool = SV.Pool(ctx, budget_bytes=12 << 20, max_cells=256, max_runs=8)
    states = {}

    def keep(pool, r, rec):
        states[r.req.rid] = pool.state(r)

    recs, waited = SV.serve(pool, trace, k=3, on_done=keep)
    assert pool.status() == 0
    assert len(recs) == len(trace)
    say("peak resident runs %d, longest queue %d" % (pool.peak_active, waited))
    assert pool.peak_active >= 2, "no two runs were resident together"
    assert waited >= 1, "no request waited for memory"
    assert pool.ealloc.used() == 0 and pool.ialloc.used() == 0
    for q in trace:
        bat = RT.Batch(ctx, [(q.spec, q.parts)])
        for s in range(q.nsteps):
            bat.step(s)
        torch.cuda.synchronize()
        a, g = bat.state(0), states[q.rid]
        for f in ("e_start", "i_start", "ew", "iz", "ik", "evx", "evy", "evz", "ivx", "ivy",
                  "ivz", "ex", "ix"):
            assert np.array_equal(getattr(a, f), getattr(g, f)), (q.rid, f)
        assert np.array_equal(bat.run_counters()[0], recs[q.rid]["counters"]), q.rid
        say("request %d (%d cells, %d steps) identical alone and served" %
            (q.rid, q.spec.ncells, q.nsteps))
