"""GPU parity of the two photon-field variants of S5 (Sec. III) against the
oracle: the photon budget with partial photoionization (XP_PHOTO_FRAC) and
the return of K-alpha photons to the field (XP_KA_FIELD), on the LDS
schedules, the global-memory path and with the reduced transport.  Same bar
as the other parity tests: state, counters, photon events and returned
photons per cell identical, velocities bit-identical."""

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import workloads as W
from tests import cases
from tests.test_gpu_parity import compare, ctx, say  # noqa: F401

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair(c, spec, parts, steps, flags, field=None, schedule=0, big="auto", capacity=(7, 16),
          transport=False, label=""):
    nb = len(spec.photon_hv)
    sim = O.Sim(c.tables, spec)
    sim.bin(parts)
    if field is not None:
        sim.set_cell_field(field)
    bat = RT.Batch(c, [(spec, parts)], capacity=capacity, cell_records=True, cell_nhv=field,
                   big=big, kalpha_return=True)
    tot = np.zeros(len(O.COUNTERS), dtype=np.int64)
    for s in range(steps):
        bat.step(s, flags, schedule=schedule)
        sim.step(s, flags)
        torch.cuda.synchronize()
        assert bat.status() == 0, "%s step %d status %d" % (label, s, bat.status())
        compare(bat.state(), sim.state(), "%s step %d" % (label, s))
        gc, gl, gm = bat.cell_records_of()
        oc, ol = sim.counters()
        assert np.array_equal(gc, oc), "%s step %d counters" % (label, s)
        assert np.allclose(gl, ol, rtol=1e-12, atol=1e-9), "%s step %d ledger" % (label, s)
        gk, ok = bat.kalpha_field(), sim.kalpha_field()
        assert np.array_equal(gk, ok), "%s step %d returned K-alpha photons" % (label, s)
        if field is not None:
            assert np.array_equal(bat.absorbed()[:, :nb], sim.absorbed()[:, :nb]), (label, s)
        if transport:
            tg = bat.transport()
            to = sim.transport()
            torch.cuda.synchronize()
            assert np.array_equal(bat.cell_field(), sim.cell_field()), "%s step %d field" % (label, s)
            assert np.array_equal(tg.cpu().numpy()[0, :nb], to), "%s step %d transmission" % (label, s)
        tot += oc.sum(axis=0)
        say("%s step %d ok" % (label, s))
    return {k: int(tot[O.COUNTERS.index(k)]) for k in
            ("PHOTO_STARVED", "PHOTO_PARTIAL", "KALPHA", "KA_FIELD", "PHOTO_1S")}


def _budget(nx, m, ni=6, ne=3, seed=7, n_hv=1e32):
    spec, parts = cases.one_run(nx, ne, ni, 5.0, 0.1, seed=seed, z0=3, photon_hv=(1850.0,),
                                photon_n=(n_hv,))
    return dataclasses.replace(spec, w0=n_hv * spec.volume / m), parts


def test_photo_budget(ctx):
    # every shell of every ion certain to fire, budgets of 2.5 and 2.3
    # macro-photons (the partial event in every cell), per-cell fields from 0
    # to 40 macro-photons; wave, block, two-wave and lane-group schedules and
    # the global-memory path
    flags = O.PHOTO | O.DECAY | O.PHOTO_FRAC
    for sched, big in ((0, "auto"), (1, "auto"), (2, "auto"), (5, "auto"), (3, "all")):
        spec, parts = _budget(8, 2.5)
        t = _pair(ctx, spec, parts, 2, flags, schedule=sched, big=big, label="budget/%d" % sched)
        assert t["PHOTO_STARVED"] > 0 and t["PHOTO_PARTIAL"] > 0
        spec, parts = _budget(64, 2.3, ni=4, seed=11)
        _pair(ctx, spec, parts, 1, flags, schedule=sched, big=big, label="budget23/%d" % sched)
        ms = np.array([0.0, 0.4, 1.0, 1.7, 4.0, 40.0])
        spec, parts = _budget(ms.size, 1.0, ni=5, seed=13, n_hv=1e33)
        _pair(ctx, spec, parts, 2, flags, field=(ms * 1e33)[:, None], schedule=sched, big=big,
              label="budget-field/%d" % sched)


def test_photo_budget_large_cells(ctx):
    # cells of 300-3000 ions: the walk over many ions and chunks of the
    # global path, and the same cells through LDS where they fit
    ni = np.array([300, 1500, 3000, 40])
    ne = np.array([20, 40, 60, 10])
    spec, parts = cases.one_run(ni.size, ne, ni, 5.0, 0.1, seed=17, z0=3, e_weight=1,
                                photon_hv=(1650.0, 1850.0), photon_n=(1e32, 2e32))
    spec = dataclasses.replace(spec, w0=1e32 * spec.volume / 7.5)
    for sched, big in ((0, "auto"), (3, "all")):
        t = _pair(ctx, spec, parts, 2, O.PHOTO | O.DECAY | O.PHOTO_FRAC, schedule=sched, big=big,
                  capacity=(4, 16), label="budget-large/%d" % sched)
        assert t["PHOTO_STARVED"] > 0


def test_kalpha_return(ctx):
    # radiative decays only (gamma_a = 0): charge states 3 (K-alpha below
    # every bin), 5 and 8 (returned to the 1500 and 1700 eV bins); then a
    # slab with the transport, where the returned photons join the beam
    tb = dataclasses.replace(ctx.tables, gamma_a=np.zeros_like(ctx.tables.gamma_a))
    c2 = RT.Context(tb)
    hv, nhv = (1500.0, 1700.0, 1850.0), (1e28, 2e28, 3e28)
    for sched, big in ((0, "auto"), (1, "auto"), (5, "auto"), (3, "all")):
        spec, parts = cases.one_run(12, 4, 40, 5.0, 0.1, seed=8, z0=3, k0=1, dt_rad=2e-14,
                                    photon_hv=hv, photon_n=nhv)
        parts.iz[:] = np.random.default_rng(8).choice([3, 5, 8], parts.ni)
        t = _pair(c2, spec, parts, 2, O.DECAY | O.KA_FIELD, schedule=sched, big=big,
                  label="kalpha/%d" % sched)
        assert 0 < t["KA_FIELD"] < t["KALPHA"]
    nx, ny = 40, 3
    spec, parts = cases.one_run(nx, 20, 40, 30.0, 0.1, seed=9, ny=ny, z0=5, k0=1, dt_rad=2e-15,
                                photon_hv=hv, photon_n=(1e29, 2e29, 3e29))
    parts.iz[:] = np.random.default_rng(9).choice([5, 6, 8], parts.ni)
    field = np.tile(np.array([1e29, 2e29, 3e29]), (nx * ny, 1))
    t = _pair(c2, spec, parts, 4, O.ALL | O.KA_FIELD, field=field, transport=True,
              label="kalpha/transport")
    assert t["KA_FIELD"] > 0


def test_photon_field_variants_together(ctx):
    # both variants with the whole step: C1 for 20 steps, a reduced C2, and a
    # slab whose weak 1650 eV bin holds less than one macro-photon per cell
    flags = O.ALL | O.PHOTO_FRAC | O.KA_FIELD
    spec, parts = W.config_c1()
    _pair(ctx, spec, parts, 20, flags, capacity=(3, 16), label="C1/field")
    spec, parts = W.config_c2(nx=6, ny=6)
    _pair(ctx, spec, parts, 6, flags, label="C2r/field")
    rng = np.random.default_rng(19)
    nx, ny = 48, 4
    ni = rng.integers(5, 50, nx * ny)
    ne = rng.integers(5, 50, nx * ny)
    spec, parts = cases.one_run(nx, ne, ni, 40.0, 0.2, seed=19, ny=ny, lnl=3.0, dt_rad=1e-15,
                                photon_hv=(1650.0, 1850.0), photon_n=(1e25, 3e30))
    parts.ik[:] = rng.integers(0, 2, parts.ni)
    field = np.tile(np.array([1e25, 3e30]), (nx * ny, 1))
    for sched, big in ((0, "auto"), (3, "all")):
        _pair(ctx, spec, parts, 6, flags, field=field, schedule=sched, big=big, transport=True,
              capacity=(10, 16), label="slab/field/%d" % sched)
