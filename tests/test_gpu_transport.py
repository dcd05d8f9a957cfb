"""The reduced radiation transport on the GPU against the oracle: after every
step the photon events per cell and bin, the rebuilt per-cell field and the
run transmissions must be identical, with the particle state as in the other
parity tests.  LDS schedules, the global-memory path, several bins, empty
cells and a 1D run."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import binding as B
from paper_1704_01202_amd import runtime as RT
from tests import cases
from tests.test_gpu_parity import compare, ctx, say  # noqa: F401

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(ctx, spec, parts, steps, flags, schedule=0, big="auto", capacity=(7, 16), label=""):
    nb = len(spec.photon_hv)
    f0 = np.tile(np.asarray(spec.photon_n, dtype=np.float64), (spec.nx * spec.ny, 1))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    sim.set_cell_field(f0)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=capacity, cell_records=True, cell_nhv=f0,
                   big=big)
    events = 0
    for s in range(steps):
        bat.step(s, flags, schedule=schedule)
        sim.step(s, flags)
        tg = bat.transport()
        to = sim.transport()
        torch.cuda.synchronize()
        assert bat.status() == 0, "%s step %d status %d" % (label, s, bat.status())
        compare(bat.state(), sim.state(), "%s step %d" % (label, s))
        ga, oa = bat.absorbed()[:, :nb], sim.absorbed()[:, :nb]
        assert np.array_equal(ga, oa), "%s step %d photon events" % (label, s)
        events += int(oa.sum())
        gf, of = bat.cell_field(), sim.cell_field()
        assert np.array_equal(gf, of), "%s step %d field (max rel %.2e)" % (
            label, s, np.max(np.abs(gf - of) / np.maximum(np.abs(of), 1e-300)))
        assert np.array_equal(tg.cpu().numpy()[0, :nb], to), "%s step %d transmission" % (label, s)
        say("%s step %d ok: %d photon events, transmission %s" % (label, s, int(oa.sum()), to))
    assert events > 0
    return bat, sim


def _slab(seed, nx=24, ny=6, ni_hi=60, ne_hi=60, bins=((1650.0, 1850.0), (6e29, 9e29))):
    rng = np.random.default_rng(seed)
    ni = rng.integers(0, ni_hi, nx * ny)
    ne = rng.integers(0, ne_hi, nx * ny)
    ni[3] = 0          # a vacuum cell inside a row
    spec, parts = cases.one_run(nx, ne, ni, 40.0, 0.2, seed=seed, ny=ny, lnl=3.0,
                                photon_hv=bins[0], photon_n=bins[1])
    parts.ik[:] = rng.integers(0, 2, parts.ni)
    return spec, parts


def test_transport_matches_oracle(ctx):
    spec, parts = _slab(71)
    _run(ctx, spec, parts, 5, O.ALL, label="transport/wave")
    for sched in (2, 5):
        spec, parts = _slab(72, ni_hi=12, ne_hi=12)
        _run(ctx, spec, parts, 4, O.ALL | O.THERM, schedule=sched, capacity=(5, 4),
             label="transport/%d" % sched)
    # a 1D run of 300 cells (rows longer than a wave)
    spec, parts = _slab(73, nx=300, ny=1, ni_hi=20, ne_hi=20, bins=((1850.0,), (2e30,)))
    _run(ctx, spec, parts, 4, O.ALL, label="transport/1d")


def test_transport_global_path(ctx):
    spec, parts = _slab(74, nx=12, ny=4)
    _run(ctx, spec, parts, 4, O.ALL, schedule=3, big="all", capacity=(3, 16),
         label="transport/global")
    # oversized cells beside LDS cells
    ne = np.array([60, 3000, 2600, 45, 0, 30])
    ni = np.array([50, 1500, 600, 40, 20, 0])
    spec, parts = cases.one_run(ne.size, ne, ni, 30.0, 0.1, seed=75, e_weight=1, dt=0.05e-15,
                                photon_hv=(1850.0,), photon_n=(4e30,))
    bat, _ = _run(ctx, spec, parts, 3, O.ALL, label="transport/oversized")
    assert bat.stats()[2] == 2


def test_transport_several_runs(ctx):
    # runs of different shapes and bins in one batch: each run's rows start at
    # its own first cell, each run's transmission is its own
    specs = []
    a = _slab(76, nx=12, ny=5, bins=((1650.0, 1850.0), (6e29, 9e29)))
    b = _slab(77, nx=70, ny=1, ni_hi=30, ne_hi=30, bins=((1800.0,), (2e30,)))
    c = _slab(78, nx=9, ny=3, ni_hi=40, ne_hi=40, bins=((1900.0,), (1e30,)))
    runs = [a, b, c]
    nbmax = max(len(s.photon_hv) for s, _ in runs)
    fields = []
    for spec, _ in runs:
        f = np.zeros((spec.nx * spec.ny, nbmax))
        f[:, :len(spec.photon_n)] = spec.photon_n
        fields.append(f)
    bat = RT.Batch(ctx, runs, capacity=(7, 16), cell_records=True, cell_nhv=np.concatenate(fields))
    sims = []
    for (spec, parts), f in zip(runs, fields):
        sim = O.Sim(ctx.tables, spec)
        sim.bin(parts)
        sim.set_cell_field(f[:, :len(spec.photon_n)])
        sims.append(sim)
    for s in range(4):
        bat.step(s, O.ALL)
        tg = bat.transport().cpu().numpy()
        for r, ((spec, _), sim) in enumerate(zip(runs, sims)):
            sim.step(s, O.ALL)
            to = sim.transport()
            nb = len(spec.photon_hv)
            compare(bat.state(r), sim.state(), "runs/%d step %d" % (r, s))
            assert np.array_equal(bat.absorbed(r)[:, :nb], sim.absorbed()[:, :nb]), (r, s)
            assert np.array_equal(bat.cell_field(r), sim.cell_field()), (r, s)
            assert np.array_equal(tg[r, :nb], to), (r, s)
            assert np.all(tg[r, nb:] == 0.0)
        say("several runs step %d ok: %s" % (s, tg[:, :2].tolist()))


def test_transport_long_run(ctx):
    # 60 steps of a 1D slab of 64 cells under an intense beam: the field,
    # the events and the transmission stay identical while the target opens up
    spec, parts = _slab(79, nx=64, ny=1, ni_hi=40, ne_hi=40, bins=((1850.0,), (3e30,)))
    # slabs for full ionization: Al3+ can give up 10 electrons
    bat, sim = _run(ctx, spec, parts, 60, O.ALL, capacity=(10, 16), label="transport/long")
    assert bat.status() == 0


def test_transport_graph_replays(ctx):
    # steps and transports captured in a HIP graph (per-run device step
    # counter) against the same batch stepped eagerly and the oracle; eager
    # work and synchronisation between the replays
    spec, parts = _slab(80, nx=40, ny=3, bins=((1650.0, 1850.0), (6e29, 9e29)))
    nb = len(spec.photon_hv)
    f0 = np.tile(np.asarray(spec.photon_n, dtype=np.float64), (spec.nx * spec.ny, 1))
    flags = O.ALL | O.NANBU
    gb = RT.Batch(ctx, [(spec, parts)], capacity=(10, 16), cell_nhv=f0)
    eb = RT.Batch(ctx, [(spec, parts)], capacity=(10, 16), cell_nhv=f0)
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    sim.set_cell_field(f0)
    d_step = torch.zeros(1, dtype=torch.int32, device=ctx.device)
    for s in range(2):
        gb.step(0, flags, d_step=d_step)
        gb.transport()
        d_step.add_(1)
        eb.step(s, flags)
        eb.transport()
        sim.step(s, flags)
        sim.transport()
    torch.cuda.synchronize()
    hint = int(gb.plan_hint())
    k = 2
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        for _ in range(k):
            gb.step(0, flags, d_step=d_step, e_hint=hint, record_stats=False)
            gb.transport()
            d_step.add_(1)
    torch.cuda.current_stream().wait_stream(side)
    step = 2
    for rep in range(3):
        g.replay()
        for _ in range(k):
            eb.step(step, flags)
            te = eb.transport()
            sim.step(step, flags)
            to = sim.transport()
            step += 1
        torch.cuda.synchronize()
        assert gb.status() == 0 and eb.status() == 0
        _ = gb.diagnostics()
        gs, es = gb.state(), eb.state()
        for f in ("e_start", "ew", "iz", "ik", "evx", "evy", "evz", "ivx", "ex"):
            assert np.array_equal(getattr(gs, f), getattr(es, f)), (rep, f)
        assert np.array_equal(gb.cell_field(), eb.cell_field()), rep
        assert np.array_equal(gb.d_trans.cpu().numpy(), te.cpu().numpy()), rep
        compare(gs, sim.state(), "transport replay %d" % rep)
        assert np.array_equal(gb.cell_field(), sim.cell_field()), rep
        assert np.array_equal(gb.d_trans.cpu().numpy()[0, :nb], to), rep
        say("transport replay %d ok at step %d" % (rep, step))


def test_transport_long_rows_and_many_rows(ctx):
    # rows longer than one 512-cell fetch: 1301 cells are three fetches, the
    # last one ragged and not a multiple of 8, so the carried product crosses
    # two fetch boundaries and the padded tail (tau = 1) is walked
    spec, parts = _slab(91, nx=1301, ny=2, ni_hi=8, ne_hi=8, bins=((1850.0,), (3e30,)))
    _run(ctx, spec, parts, 3, O.ALL, capacity=(10, 16), label="transport/1301x2")
    # more rows than one fetch of the row sum (1100 rows of two cells)
    spec, parts = _slab(92, nx=2, ny=1100, ni_hi=8, ne_hi=8, bins=((1650.0, 1850.0), (6e29, 3e30)))
    _run(ctx, spec, parts, 3, O.ALL, capacity=(10, 16), label="transport/2x1100")


def test_transport_rejects_inconsistent_run_grid(ctx):
    # a run table whose grid does not cover its cell range: every row of that
    # run is left as it was and XP_ST_RUN_TABLE is raised for the batch and the
    # run; the consistent run beside it is transported as usual
    a = _slab(93, nx=10, ny=3, ni_hi=20, ne_hi=20, bins=((1850.0,), (3e30,)))
    b = _slab(94, nx=8, ny=2, ni_hi=20, ne_hi=20, bins=((1850.0,), (3e30,)))
    f = np.full((a[0].nx * a[0].ny + b[0].nx * b[0].ny, 1), 3e30)
    bat = RT.Batch(ctx, [a, b], capacity=(7, 16), cell_records=True, cell_nhv=f)
    bat.step(0, O.ALL)
    torch.cuda.synchronize()
    # corrupt run 0's nx on the device (its cell count stays 30)
    off = B.XpRun.nx.offset
    raw = bat.d_runs.cpu().numpy().copy()
    raw[off:off + 4] = np.frombuffer(np.int32(7).tobytes(), dtype=np.uint8)
    bat.d_runs.copy_(torch.from_numpy(raw).to(ctx.device))
    before = bat.d_cell_nhv.cpu().numpy().copy()
    bat.transport()
    torch.cuda.synchronize()
    after = bat.d_cell_nhv.cpu().numpy()
    n0 = a[0].nx * a[0].ny
    assert np.array_equal(after[:n0], before[:n0])
    assert not np.array_equal(after[n0:], before[n0:])
    assert bat.status() & B.XP_ST_RUN_TABLE
    rs = bat.run_status()
    assert rs[0] & B.XP_ST_RUN_TABLE and not rs[1] & B.XP_ST_RUN_TABLE
    assert bat.d_trans.cpu().numpy()[0, 0] == 0.0 and bat.d_trans.cpu().numpy()[1, 0] > 0.0
