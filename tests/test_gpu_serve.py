"""Serving with continuous batching: runs admitted into a resident pool as
memory frees up, stepped together, retired when done.  Each result must be
bit-identical to the same run stepped alone on the GPU and to the oracle, and
a run's device status must be its own."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import binding as B
from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import serve as SV
from paper_1704_01202_amd import workloads as W
from tests import cases
from tests.test_gpu_parity import compare, ctx, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _oracle_run(tables, q):
    sim = O.Sim(tables, q.spec)
    sim.bin(q.parts)
    for s in range(q.nsteps):
        sim.step(s)
    return sim


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
        assert recs[q.rid]["status"] == 0, q.rid
        bat = RT.Batch(ctx, [(q.spec, q.parts)])
        for s in range(q.nsteps):
            bat.step(s)
        torch.cuda.synchronize()
        a, g = bat.state(0), states[q.rid]
        for f in ("e_start", "i_start", "ew", "iz", "ik", "evx", "evy", "evz", "ivx", "ivy",
                  "ivz", "ex", "ix"):
            assert np.array_equal(getattr(a, f), getattr(g, f)), (q.rid, f)
        assert np.array_equal(bat.run_counters()[0], recs[q.rid]["counters"]), q.rid
        # and the oracle, run by run
        sim = _oracle_run(ctx.tables, q)
        compare(g, sim.state(), "served request %d" % q.rid)
        oc = sim.counters()[0]   # last step only; the run totals are checked above
        assert oc.shape[0] == q.spec.ncells
        say("request %d (%d cells, %d steps) identical alone, served and in the oracle" %
            (q.rid, q.spec.ncells, q.nsteps))


def test_served_run_status_is_its_own(ctx):
    # slabs without spare slots (capacity rule (0, 0)): a hot run whose
    # ionizations need new electron slots overflows, a cold run beside it
    # does not; only the hot run's record carries XP_ST_CAPACITY, and the cold
    # run's result is the oracle's
    hot_spec, hot_parts = cases.one_run(2, 32, 30, 3000.0, 1.0, seed=79, e_weight=3)
    cold_spec, cold_parts = cases.one_run(3, 20, 20, 5.0, 0.1, seed=80, e_weight=3)
    cold = W.Request(rid=1, arrival=0.0, spec=cold_spec, parts=cold_parts, nsteps=3)
    hot = W.Request(rid=0, arrival=0.0, spec=hot_spec, parts=hot_parts, nsteps=3)
    late = W.Request(rid=2, arrival=0.0, spec=cold_spec, parts=cold_parts, nsteps=2)
    # the oracle: the hot run ionizes in its first step, the cold one never
    # needs a new slot
    sim_hot = _oracle_run(ctx.tables, hot)
    assert sim_hot.state().ew.size > hot_parts.ne
    sim_cold = O.Sim(ctx.tables, cold_spec)
    sim_cold.bin(cold_parts)
    for s in range(cold.nsteps):
        sim_cold.step(s)
        assert sim_cold.counters()[0][:, O.COUNTERS.index("E_NEW")].sum() == 0
    pool = SV.Pool(ctx, budget_bytes=12 << 20, max_cells=64, max_runs=4, capacity=(0, 0))
    states = {}

    def keep(pool, r, rec):
        states[r.req.rid] = pool.state(r)

    recs, _ = SV.serve(pool, [hot, cold, late], k=1, on_done=keep)
    assert pool.status() & B.XP_ST_CAPACITY
    assert recs[0]["status"] & B.XP_ST_CAPACITY
    assert recs[1]["status"] == 0 and recs[2]["status"] == 0
    compare(states[1], sim_cold.state(), "cold run beside an overflowing one")
    sim_late = _oracle_run(ctx.tables, late)
    compare(states[2], sim_late.state(), "run admitted after the overflow")
