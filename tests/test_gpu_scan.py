"""Batched scans on the GPU: one batch of independent runs with per-run device
step counters, steps captured in a HIP graph, knobs picked by timing.  Every
run must come out bit-identical to the same run stepped alone and to the CPU
oracle, after every replay."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import scan as SC
from paper_1704_01202_amd import workloads as W
from tests.test_gpu_parity import compare, ctx, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def small_scan(nruns=6):
    # sizes 2e3 .. 3e4 particles: runs below and above the LDS limits
    return W.config_c4_runs(seed=4, nruns=nruns, nsteps=9, size_lo=2e3, size_hi=3e4)


def test_scan_graph_replays_match_eager_alone_and_oracle(ctx):
    runs = small_scan()
    sc = SC.Scan(ctx, runs)
    ref = RT.Batch(ctx, runs)
    sims = []
    for spec, parts in runs:
        sim = O.Sim(ctx.tables, spec)
        sim.bin(parts)
        sims.append(sim)
    # two eager steps give the stats the capture plans with
    for s in range(2):
        sc.eager_step()
        ref.step(s)
        for sim in sims:
            sim.step(s)
    sc.capture(3)
    step = 2
    for rep in range(3):
        sc.replay()
        for _ in range(3):
            ref.step(step)
            for sim in sims:
                sim.step(step)
            step += 1
        torch.cuda.synchronize()
        assert sc.status() == 0 and ref.status() == 0
        # eager work and a synchronisation between replays
        _ = sc.bat.diagnostics()
        for r in range(len(runs)):
            g = sc.bat.state(r)
            e = ref.state(r)
            for f in ("e_start", "i_start", "ew", "iz", "ik", "evx", "evy", "evz", "ivx", "ex"):
                assert np.array_equal(getattr(g, f), getattr(e, f)), (rep, r, f)
            compare(g, sims[r].state(), "scan replay %d run %d" % (rep, r))
        say("replay %d ok at step %d" % (rep, step))
    assert sc.bat.stats()[2] >= 1, "no run took the global-memory path"
    # the same runs stepped alone
    _, _, alone = SC.sequential(ctx, runs, step, keep=True)
    for r, bat in enumerate(alone):
        g, a = sc.bat.state(r), bat.state(0)
        for f in ("e_start", "ew", "iz", "ik", "evx", "ivz"):
            assert np.array_equal(getattr(g, f), getattr(a, f)), (r, f)


def test_autotune_changes_speed_not_results(ctx):
    runs = small_scan(4)
    sc = SC.Scan(ctx, runs)
    cands = [{"schedule": 1, "quantile": 0.9, "big_grid": 0},
             {"schedule": 2, "quantile": 1.0, "big_grid": 1024},
             {"schedule": 0, "quantile": 0.99, "big_grid": 8192}]
    best, ms = sc.autotune(cands, reps=2)
    assert best in cands and ms > 0
    n = sc.steps_done
    ref = RT.Batch(ctx, runs)
    for s in range(n):
        ref.step(s)
    torch.cuda.synchronize()
    for r in range(len(runs)):
        g, e = sc.bat.state(r), ref.state(r)
        for f in ("e_start", "ew", "iz", "ik", "evx", "evy", "evz", "ivx"):
            assert np.array_equal(getattr(g, f), getattr(e, f)), (r, f)
