"""Parity at full size, in the launch configuration the benchmarks time.

* The whole 512 x 512-cell target (33.5 M particles) stepped by the library
  exactly as bench.py steps it (default schedule, LDS plans from the previous
  step's statistics) against the oracle on every cell, for a few steps.
* A sample of the 256-run batched scan at full size, including its largest
  run (one cell with about 2 million particles on the global-memory path),
  stepped together in one batch against each run's oracle.
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


def test_c2_full_size_parity(ctx):
    spec, parts = W.config_c2()
    say("C2 full: %d cells, %d electrons, %d ions" % (spec.ncells, parts.ne, parts.ni))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(7, 16))
    th = host_threads()
    total = np.zeros(24, dtype=np.int64)
    for s in range(3):
        bat.step(s)
        sim.step(s, O.ALL, th)
        torch.cuda.synchronize()
        assert bat.status() == 0
        w, nb = compare(bat.state(), sim.state(), "C2 full step %d" % s)
        cnt, _ = sim.counters()
        total += cnt[:, :24].sum(axis=0).astype(np.int64)
        # the run's accumulated counters equal the oracle's per-step sums
        assert np.array_equal(bat.run_counters()[0][:24].astype(np.int64), total), s
        say("C2 full step %d ok (differing words %d)" % (s, nb))


def test_c4_full_size_sample_parity(ctx):
    runs = W.config_c4_runs()
    sizes = np.array([p.ne + p.ni for _, p in runs])
    order = np.argsort(sizes)
    pick = sorted(set([int(order[-1]), int(order[0]), int(order[len(order) // 2]), 7, 100, 201]))
    sample = [runs[r] for r in pick]
    say("C4 sample runs %s, particles %s" % (pick, [int(sizes[r]) for r in pick]))
    bat = RT.Batch(ctx, sample, capacity=(10, 16))
    sims = []
    for spec, parts in sample:
        sim = O.Sim(ctx.tables, spec)
        sim.bin(parts)
        sims.append(sim)
    th = host_threads()
    for s in range(2):
        bat.step(s)
        for sim in sims:
            sim.step(s, O.ALL, th)
        torch.cuda.synchronize()
        assert bat.status() == 0
        for k, sim in enumerate(sims):
            compare(bat.state(k), sim.state(), "C4 run %d step %d" % (pick[k], s))
        say("C4 sample step %d ok" % s)
    assert bat.stats()[2] >= 1, "no run took the global-memory path"


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
