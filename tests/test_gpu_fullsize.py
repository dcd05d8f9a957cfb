"""Parity at full size, in the launch configuration the benchmarks time.

* The whole 512 x 512-cell target (33.5 M particles) stepped by the library
  exactly as bench.py steps it (default schedule, LDS plans from the
  statistics the host has seen) against the oracle on every cell, over the
  whole 200-step run: run counters after every step, the full particle state
  at checkpoints.
* The whole 1024 x 256 density ramp for 10 steps.
* All 256 runs of the batched scan at full size in one batch (the largest is
  one cell of about 2 million particles on the global-memory path) for 3
  steps, and its 16 smallest runs for their whole 500 steps.
* The 512 x 512 target with Nanbu's law and the reduced transport.
"""

import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import workloads as W
from tests.test_gpu_parity import compare, ctx, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def host_threads():
    env = os.environ.get("OMP_NUM_THREADS", "")
    n = int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def _c2_checkpoints(n):
    return {0, 24, 49, 99, 149, n - 1}


def test_c2_full_size_parity(ctx):
    spec, parts = W.config_c2()
    nsteps = spec.nsteps
    say("C2 full: %d cells, %d electrons, %d ions, %d steps" % (spec.ncells, parts.ne, parts.ni, nsteps))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(7, 16))
    th = host_threads()
    total = np.zeros(len(O.COUNTERS), dtype=np.int64)
    for s in range(nsteps):
        bat.step(s)
        sim.step(s, O.ALL, th)
        torch.cuda.synchronize()
        assert bat.status() == 0, s
        cnt, _ = sim.counters()
        total += cnt.sum(axis=0).astype(np.int64)
        # the run's accumulated counters equal the oracle's per-step sums
        assert np.array_equal(bat.run_counters()[0].astype(np.int64), total), s
        if s in _c2_checkpoints(nsteps):
            w, nb = compare(bat.state(), sim.state(), "C2 full step %d" % s)
            say("C2 full step %d ok: %d electrons (differing words %d)" % (s, int(bat.d_e_cnt.sum()), nb))
        elif s % 10 == 9:
            say("C2 full step %d: counters ok" % s)


def test_c3_full_grid_parity(ctx):
    spec, parts = W.config_c3()
    say("C3 full: %d cells, %d electrons, %d ions" % (spec.ncells, parts.ne, parts.ni))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(7, 16))
    th = host_threads()
    total = np.zeros(len(O.COUNTERS), dtype=np.int64)
    for s in range(10):
        bat.step(s)
        sim.step(s, O.ALL, th)
        torch.cuda.synchronize()
        assert bat.status() == 0, s
        cnt, _ = sim.counters()
        total += cnt.sum(axis=0).astype(np.int64)
        assert np.array_equal(bat.run_counters()[0].astype(np.int64), total), s
        if s in (0, 4, 9):
            _, nb = compare(bat.state(), sim.state(), "C3 full step %d" % s)
            say("C3 full step %d ok (differing words %d)" % (s, nb))


def _step_all(sims, s, pool):
    # single-cell runs: one oracle thread per run, the runs spread over a pool
    list(pool.map(lambda sim: sim.step(s, O.ALL, 1), sims))


def test_c4_all_runs_parity(ctx):
    from concurrent.futures import ThreadPoolExecutor
    runs = W.config_c4_runs()
    sizes = np.array([p.ne + p.ni for _, p in runs])
    say("C4 all %d runs: %d particles, largest %d" % (len(runs), int(sizes.sum()), int(sizes.max())))
    bat = RT.Batch(ctx, runs, capacity=(12, 16))
    sims = []
    for spec, parts in runs:
        sim = O.Sim(ctx.tables, spec)
        sim.bin(parts)
        sims.append(sim)
    with ThreadPoolExecutor(host_threads()) as pool:
        for s in range(3):
            bat.step(s)
            _step_all(sims, s, pool)
            torch.cuda.synchronize()
            assert bat.status() == 0
            gst = bat.states()
            for k, sim in enumerate(sims):
                compare(gst[k], sim.state(), "C4 run %d step %d" % (k, s))
            say("C4 all runs step %d ok" % s)
    assert bat.stats()[2] >= 1, "no run took the global-memory path"


def test_c4_smallest_runs_full_length(ctx):
    from concurrent.futures import ThreadPoolExecutor
    runs = W.config_c4_runs()
    sizes = np.array([p.ne + p.ni for _, p in runs])
    pick = [int(r) for r in np.argsort(sizes)[:16]]
    sample = [runs[r] for r in pick]
    nsteps = sample[0][0].nsteps
    say("C4 smallest runs %s, %d steps" % (pick, nsteps))
    bat = RT.Batch(ctx, sample, capacity=(12, 16))
    sims = []
    for spec, parts in sample:
        sim = O.Sim(ctx.tables, spec)
        sim.bin(parts)
        sims.append(sim)
    totals = np.zeros((len(sims), len(O.COUNTERS)), dtype=np.int64)
    with ThreadPoolExecutor(host_threads()) as pool:
        for s in range(nsteps):
            bat.step(s)
            _step_all(sims, s, pool)
            for k, sim in enumerate(sims):
                totals[k] += sim.counters()[0].sum(axis=0)
            if s % 100 == 99 or s == nsteps - 1:
                torch.cuda.synchronize()
                assert bat.status() == 0
                assert np.array_equal(bat.run_counters().astype(np.int64), totals), s
                gst = bat.states()
                for k, sim in enumerate(sims):
                    compare(gst[k], sim.state(), "C4 run %d step %d" % (pick[k], s))
                say("C4 smallest runs step %d ok" % s)


def test_c2_full_size_variants_parity(ctx):
    # the 512 x 512 target with Nanbu's scattering law and the reduced
    # radiation transport after every step, as bench.py --nanbu --transport
    # steps it: state, photon events, field and transmission against the oracle
    spec, parts = W.config_c2()
    f0 = np.tile(np.asarray(spec.photon_n, dtype=np.float64), (spec.ncells, 1))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    sim.set_cell_field(f0)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(7, 16), cell_nhv=f0)
    th = host_threads()
    flags = O.ALL | O.NANBU
    for s in range(2):
        bat.step(s, flags)
        sim.step(s, flags, th)
        tg = bat.transport()
        to = sim.transport()
        torch.cuda.synchronize()
        assert bat.status() == 0
        compare(bat.state(), sim.state(), "C2 full nanbu+transport step %d" % s)
        assert np.array_equal(bat.absorbed()[:, :1], sim.absorbed()[:, :1]), s
        assert np.array_equal(bat.cell_field(), sim.cell_field()), s
        assert np.array_equal(tg.cpu().numpy()[0, :1], to), s
        say("C2 full nanbu+transport step %d ok, transmission %.6f" % (s, to[0]))
