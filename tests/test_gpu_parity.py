"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar (integer work bit-exact; floating point as stated):
* elementary functions, Philox, sqrt and division of the device: bit-identical
  to the oracle's / IEEE;
* binning: identical cell contents and order;
* steps: per cell identical counts, weights, charge states, K vacancies and
  event counters; velocities identical to 1e-12 relative (the contract makes
  them bit-identical; the tolerance only absorbs a tie decided differently);
* schedule invariance: one wave per cell and one block per cell give the same
  bits.
"""

import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1704_01202_amd import binding as B  # noqa: E402
from paper_1704_01202_amd import runtime as RT  # noqa: E402
from paper_1704_01202_amd import workloads as W  # noqa: E402
from tests import cases  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tab = W.make_tables()
    return RT.Context(tab)


def compare(gs, os_, label, vtol=1e-12, strict=True):
    """gs: GPU CompactState, os_: oracle State.

    Integers must be identical.  Velocities must agree element by element to
    vtol relative, with an absolute floor of vtol times 1e-3 of the array's rms
    speed for components near 0; with strict (the default) every word must be
    identical, since both sides evaluate the same IEEE operation sequence.
    """
    assert np.array_equal(gs.e_start, os_.e_start), label + " electron counts"
    assert np.array_equal(gs.i_start, os_.i_start), label + " ion counts"
    assert np.array_equal(gs.ew, os_.ew), label + " weights"
    assert np.array_equal(gs.iz, os_.iz), label + " Z"
    assert np.array_equal(gs.ik, os_.ik), label + " k"
    assert np.array_equal(gs.ex, os_.ex), label + " electron x"
    worst = 0.0
    nbits = 0
    for a, b in ((gs.evx, os_.evx), (gs.evy, os_.evy), (gs.evz, os_.evz),
                 (gs.ivx, os_.ivx), (gs.ivy, os_.ivy), (gs.ivz, os_.ivz)):
        if a.size == 0:
            continue
        floor = 1e-3 * max(float(np.sqrt(np.mean(b * b))), 1e-300)
        rel = np.abs(a - b) / np.maximum(np.abs(b), floor)
        worst = max(worst, float(rel.max()))
        nbits += int((a.view(np.uint64) != b.view(np.uint64)).sum())
    assert worst <= vtol, "%s velocities differ: max rel %.3e" % (label, worst)
    if strict:
        assert nbits == 0, "%s: %d velocity words differ (max rel %.3e)" % (label, nbits, worst)
    return worst, nbits


def canonical_sum(leaves):
    """Pairwise sum, leaves padded with +0 to a power of two, level by level, + 0.0."""
    p = 1
    while p < len(leaves):
        p <<= 1
    v = list(leaves) + [0.0] * (p - len(leaves))
    while len(v) > 1:
        v = [v[2 * i] + v[2 * i + 1] for i in range(len(v) // 2)]
    return v[0] + 0.0


def run_pair(ctx, spec, parts, steps, flags=O.ALL, schedule=0, capacity=(7, 16),
             check_every=1, label="", big="auto"):
    tab = ctx.tables
    sim = O.Sim(tab, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=capacity, cell_records=True, big=big)
    compare(bat.state(), sim.state(), label + " after binning")
    for s in range(steps):
        bat.step(s, flags, schedule=schedule)
        sim.step(s, flags)
        if (s + 1) % check_every == 0 or s == steps - 1:
            torch.cuda.synchronize()
            assert bat.status() == 0, "status %d at step %d" % (bat.status(), s)
            w, nb = compare(bat.state(), sim.state(), "%s step %d" % (label, s))
            gc, gl, gm = bat.cell_records_of()
            oc, ol = sim.counters()
            assert np.array_equal(gc, oc), "%s step %d counters" % (label, s)
            om = sim.moments()
            assert np.array_equal(gm[:, :29], om[:, :29]), "%s step %d moments" % (label, s)
            assert np.allclose(gl, ol, rtol=1e-12, atol=1e-9), "%s step %d ledger" % (label, s)
            say("%s step %d ok (max rel %.1e, differing words %d)" % (label, s, w, nb))
    return bat, sim


def test_device_building_blocks(ctx):
    rng = np.random.default_rng(101)
    dev = ctx.device
    n = 200000
    xs = np.concatenate([np.exp(rng.uniform(-700, 700, n // 2)), rng.uniform(0.5, 2, n // 2)])
    dx = torch.from_numpy(xs).to(dev)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    for which, fn in ((0, O.log), (2, O.cbrt)):
        B.xp_selftest(ctx.h, which, n, dx.data_ptr(), None, out.data_ptr(), None, RT._stream())
        g = out.cpu().numpy()
        ref = np.array([fn(v) for v in xs[:20000]])
        assert np.array_equal(g[:20000], ref), "selftest %d" % which
        say("selftest %d ok" % which)
    xe = rng.uniform(-700, 700, 20000)
    dxe = torch.from_numpy(xe).to(dev)
    B.xp_selftest(ctx.h, 1, xe.size, dxe.data_ptr(), None, out.data_ptr(), None, RT._stream())
    assert np.array_equal(out.cpu().numpy()[:xe.size], np.array([O.exp(v) for v in xe]))
    # sqrt and division are IEEE correctly rounded on both sides
    B.xp_selftest(ctx.h, 5, n, dx.data_ptr(), None, out.data_ptr(), None, RT._stream())
    assert np.array_equal(out.cpu().numpy(), np.sqrt(xs))
    # canonical tree sums (one wave, a block of 256, groups of 16 lanes) on
    # values of mixed sign and magnitude, where the order of the additions
    # shows in the bits
    for which, r, rows in ((7, 64, 400), (8, 256, 120), (9, 64, 400)):
        v = rng.choice([-1.0, 1.0], rows * r) * 10.0 ** rng.uniform(-18, 18, rows * r)
        dv = torch.from_numpy(v).to(dev)
        o = torch.empty(rows, dtype=torch.float64, device=dev)
        B.xp_selftest(ctx.h, which, v.size, dv.data_ptr(), None, o.data_ptr(), None, RT._stream())
        got = o.cpu().numpy()
        want, seq_differs = [], 0
        for j in range(rows):
            leaves = [float(t) for t in v[j * r: j * r + (j * 37) % r + 1]]
            want.append(canonical_sum(leaves))
            acc = 0.0
            for t in leaves:
                acc += t
            seq_differs += acc != want[-1]
        assert seq_differs > rows // 10, "the values do not tell summation orders apart"
        assert np.array_equal(got, np.array(want)), "tree self-test %d" % which
        say("tree self-test %d ok (%d of %d rows differ from the sequential sum)" % (which, seq_differs, rows))
    pairs = np.exp(rng.uniform(-300, 300, 2 * n))
    dp = torch.from_numpy(pairs).to(dev)
    B.xp_selftest(ctx.h, 6, n, dp.data_ptr(), None, out.data_ptr(), None, RT._stream())
    assert np.array_equal(out.cpu().numpy(), pairs[0::2] / pairs[1::2])
    # sincos
    ks = rng.integers(0, 1 << 52, 20000, dtype=np.int64).astype(np.uint64)
    du = torch.from_numpy(ks.view(np.int64)).to(dev)
    o2 = torch.empty(2 * ks.size, dtype=torch.float64, device=dev)
    B.xp_selftest(ctx.h, 3, ks.size, None, du.data_ptr(), o2.data_ptr(), None, RT._stream())
    g = o2.cpu().numpy().reshape(-1, 2)
    ref = np.array([O.sincos2pi(int(k)) for k in ks])
    assert np.array_equal(g, ref)
    # Philox
    words = rng.integers(0, 1 << 32, (50000, 6), dtype=np.uint64).astype(np.uint32)
    dw = torch.from_numpy(words.view(np.int64).reshape(-1)).to(dev)
    ow = torch.empty(4 * 50000, dtype=torch.int32, device=dev)
    B.xp_selftest(ctx.h, 4, 50000, None, dw.data_ptr(), None, ow.data_ptr(), RT._stream())
    gw = ow.cpu().numpy().view(np.uint32).reshape(-1, 4)
    assert np.array_equal(gw, O.philox(words[:, :4], words[:, 4:]))
    say("building blocks ok")


def test_bin_matches_oracle_2d(ctx):
    spec, parts = W.config_c2(nx=24, ny=20)
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)])
    compare(bat.state(), sim.state(), "bin 2d")
    g = bat.state()
    assert np.array_equal(g.ey, sim.state().ey)


def test_c1_parity(ctx):
    spec, parts = W.config_c1()
    steps = int(os.environ.get("XPIC_C1_STEPS", "100"))
    run_pair(ctx, spec, parts, steps, check_every=10, capacity=(3, 16), label="C1")


def test_c2_reduced_parity(ctx):
    spec, parts = W.config_c2(nx=16, ny=12)
    run_pair(ctx, spec, parts, 40, check_every=8, label="C2r")


def test_c3_strip_parity(ctx):
    spec, parts = W.config_c3(nx=96, ny=4)
    run_pair(ctx, spec, parts, 20, check_every=5, capacity=(1, 16), label="C3s")


def test_schedule_invariance(ctx):
    # one wave per cell, one block per cell, and 2, 4, 8 cells per wave give
    # the same bits (the uneven strip exercises the small-cell groups)
    for spec, parts in (W.config_c2(nx=8, ny=8), W.config_c3(nx=64, ny=2)):
        outs = []
        for sched in (1, 2, 4, 5, 6):
            bat = RT.Batch(ctx, [(spec, parts)])
            for s in range(12):
                bat.step(s, O.ALL, schedule=sched)
            torch.cuda.synchronize()
            assert bat.status() == 0
            outs.append(bat.state())
        for k in range(1, len(outs)):
            for f in ("evx", "evy", "evz", "ew", "iz", "ik", "ivx", "e_start", "ex"):
                assert np.array_equal(getattr(outs[0], f), getattr(outs[k], f)), (k, f)
        say("schedules agree on %d cells" % spec.ncells)


@pytest.mark.parametrize("sched", [4, 5, 6])
def test_group_schedules_match_oracle(ctx, sched):
    # slabs of at most 32 electron and 16 ion slots, so that even groups of
    # 8 lanes take every cell (the oracle keeps these cells within 32
    # electrons over the 10 steps)
    rng = np.random.default_rng(5)
    ne = np.array([0, 1, 2, 3, 0, 5, 7, 1, 0, 12, 11, 9, 4, 6, 2, 8])
    ni = np.array([0, 0, 1, 1, 3, 2, 5, 1, 1, 5, 1, 3, 5, 4, 5, 2])
    spec, parts = cases.one_run(ne.size, ne, ni, 200.0, 1.0, seed=88, lnl=3.0,
                                photon_hv=(1800.0,), photon_n=(3e30,))
    parts.iz[:] = rng.integers(3, 14, parts.ni)
    parts.ik[:] = np.where(parts.iz < 12, rng.integers(0, 2, parts.ni), 0)
    parts.ew[:] = rng.choice([1, 2, 3], parts.ne)
    run_pair(ctx, spec, parts, 10, check_every=1, label="groups/%d" % sched, schedule=sched,
             capacity=(3, 4))
    spec, parts = W.config_c3(nx=48, ny=3)
    run_pair(ctx, spec, parts, 10, check_every=5, label="C3s/%d" % sched, schedule=sched,
             capacity=(1, 16))


def test_photo_auger_step_alone(ctx):
    n = 200
    spec, parts = cases.one_run(6, 3 * n, n, 10.0, 0.1, k0=1, seed=77, dt=0.1e-15,
                                photon_hv=(1650.0, 1900.0), photon_n=(2e29, 1e29))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(1, 16), cell_records=True)
    for s in range(4):
        bat.photo_auger(s)
        sim.step(s, O.PHOTO | O.DECAY)
        torch.cuda.synchronize()
        compare(bat.state(), sim.state(), "photo step %d" % s)
        gc, _, _ = bat.cell_records_of()
        oc, _ = sim.counters()
        assert np.array_equal(gc, oc)
    assert sim.counters()[0][:, O.COUNTERS.index("DECAY")].sum() >= 0


def _therm_edge_case(seed):
    # empty cells, lone electrons, one velocity for a whole cell (no thermal
    # energy), keV electrons among cold ones, mixed weights
    rng = np.random.default_rng(seed)
    ne = np.array([0, 1, 2, 5, 7, 12, 3, 9, 0, 4])
    ni = np.array([1, 0, 2, 3, 1, 2, 4, 3, 2, 1])
    spec, parts = cases.one_run(ne.size, ne, ni, 50.0, 0.5, seed=seed, lnl=3.0,
                                photon_hv=(1800.0,), photon_n=(3e30,))
    cell = np.floor(parts.ex / spec.dx).astype(int)
    one = cell == 3
    parts.evx[one], parts.evy[one], parts.evz[one] = 2.0e5, -1.0e5, 4.0e5
    hot = rng.random(parts.ne) < 0.2
    parts.evx[hot] *= 8.0
    parts.ew[:] = rng.choice([1, 2, 3], parts.ne)
    return spec, parts


def test_forced_thermalization(ctx):
    # the variant of Sec. VI.C after the whole step: C1 (keV source electrons
    # among 10 eV ones) and edge cells on every LDS schedule
    spec, parts = W.config_c1()
    bat, sim = run_pair(ctx, spec, parts, 8, flags=O.ALL | O.THERM, check_every=4, label="C1/therm")
    oc = sim.counters()[0]
    assert oc[:, O.COUNTERS.index("THERM")].sum() == 64
    for sched in (1, 2, 5):
        spec, parts = _therm_edge_case(41)
        bat, sim = run_pair(ctx, spec, parts, 6, flags=O.ALL | O.THERM, check_every=1,
                            capacity=(3, 4), schedule=sched, label="therm/%d" % sched)
        oc = sim.counters()[0]
        assert oc[:, O.COUNTERS.index("THERM")].sum() > 0
        assert oc[:, O.COUNTERS.index("THERM_SKIPPED")].sum() > 0


def _mixed_charge_case(seed, n_cells=12, ne_hi=40, ni_hi=20):
    rng = np.random.default_rng(seed)
    ne = rng.integers(0, ne_hi, n_cells)
    ni = rng.integers(0, ni_hi, n_cells)
    spec, parts = cases.one_run(n_cells, ne, ni, 120.0, 0.5, seed=seed, lnl=3.0,
                                photon_hv=(1800.0,), photon_n=(3e30,))
    parts.iz[:] = rng.integers(3, 14, parts.ni)
    parts.ik[:] = np.where(parts.iz < 12, rng.integers(0, 2, parts.ni), 0)
    parts.ew[:] = rng.choice([1, 2, 3], parts.ne)
    return spec, parts


def test_per_charge_state_ionization(ctx):
    # the S3 variant with every ion's own charge state (Sec. IV), alone and
    # with the forced thermalization, on every LDS schedule
    spec, parts = _mixed_charge_case(51)
    bat, sim = run_pair(ctx, spec, parts, 8, flags=O.ALL | O.ION_Z, check_every=1,
                        label="ionz")
    assert (sim.moments()[:, 11] > 1).any()
    for sched in (1, 2, 5):
        # small slabs for the lane groups: at most 48 electron slots per cell
        # (the oracle keeps these cells within them over the 6 steps)
        spec, parts = _mixed_charge_case(52, ne_hi=12, ni_hi=6)
        run_pair(ctx, spec, parts, 6, flags=O.ALL | O.ION_Z | O.THERM, check_every=2,
                 capacity=(5, 4), schedule=sched, label="ionz+therm/%d" % sched)
    spec, parts = W.config_c2(nx=6, ny=6)
    run_pair(ctx, spec, parts, 16, flags=O.ALL | O.ION_Z, check_every=8, label="C2r/ionz")


def test_nanbu_scattering(ctx):
    # Nanbu's cumulative scattering law in S1/S2: C1 (nu dt >> 1 for its 10 eV
    # electrons, small angles for the keV ones), edge cells, mixed charges with
    # the other variants on every LDS schedule, and a reduced C2
    spec, parts = W.config_c1()
    bat, sim = run_pair(ctx, spec, parts, 100, flags=O.ALL | O.NANBU, check_every=25,
                        label="C1/nanbu")
    assert sim.counters()[0][:, O.COUNTERS.index("DELTA2_GT1")].sum() > 0
    spec, parts = _therm_edge_case(47)
    run_pair(ctx, spec, parts, 6, flags=O.ALL | O.NANBU, check_every=1, capacity=(3, 4),
             label="nanbu/edge")
    for sched in (1, 2, 5):
        spec, parts = _mixed_charge_case(54, ne_hi=12, ni_hi=6)
        run_pair(ctx, spec, parts, 6, flags=O.ALL | O.NANBU | O.ION_Z | O.THERM, check_every=2,
                 capacity=(5, 4), schedule=sched, label="nanbu+ionz+therm/%d" % sched)
    spec, parts = W.config_c2(nx=6, ny=6)
    run_pair(ctx, spec, parts, 12, flags=O.ALL | O.NANBU, check_every=6, label="C2r/nanbu")


def test_thermalization_after_source_terms_alone(ctx):
    n = 120
    spec, parts = cases.one_run(5, 3 * n, n, 10.0, 0.1, k0=1, seed=79, dt=0.1e-15,
                                photon_hv=(1650.0, 1900.0), photon_n=(2e29, 1e29))
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(1, 16), cell_records=True)
    for s in range(3):
        bat.photo_auger(s, flags=B.XP_PHOTO | B.XP_DECAY | B.XP_THERM)
        sim.step(s, O.PHOTO | O.DECAY | O.THERM)
        torch.cuda.synchronize()
        compare(bat.state(), sim.state(), "photo+therm step %d" % s)
        gc, _, _ = bat.cell_records_of()
        oc, _ = sim.counters()
        assert np.array_equal(gc, oc)
        assert oc[:, O.COUNTERS.index("THERM")].sum() == 5
    say("photo_auger_step + thermalization ok")


def test_edge_cells(ctx):
    # empty cells, lone particles, odd counts, bare nuclei, ions without electrons
    rng = np.random.default_rng(5)
    ne = np.array([0, 1, 2, 3, 0, 5, 7, 1, 0, 64, 65, 129])
    ni = np.array([0, 0, 1, 1, 3, 2, 7, 1, 1, 63, 1, 3])
    spec, parts = cases.one_run(ne.size, ne, ni, 200.0, 1.0, seed=78, lnl=3.0,
                                photon_hv=(1800.0,), photon_n=(3e30,))
    parts.iz[:] = rng.integers(3, 14, parts.ni)
    parts.ik[:] = np.where(parts.iz < 12, rng.integers(0, 2, parts.ni), 0)
    parts.ew[:] = rng.choice([1, 2, 3], parts.ne)
    run_pair(ctx, spec, parts, 12, check_every=1, label="edge")


def test_ion_heavy_cells(ctx):
    # far more ions than electrons: small plans defer these cells for their
    # ions, and the last plan takes them
    ne = np.array([1, 2, 0, 3, 4, 64, 9, 0])
    ni = np.array([100, 60, 70, 5, 47, 2, 130, 1])
    spec, parts = cases.one_run(ne.size, ne, ni, 100.0, 1.0, seed=61, lnl=3.0)
    bat, _ = run_pair(ctx, spec, parts, 6, check_every=1, label="ion-heavy")
    assert bat.stats()[1] > 0


def test_diagnostics_match_oracle(ctx):
    spec, parts = W.config_c2(nx=10, ny=10)
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    bat = RT.Batch(ctx, [(spec, parts)])
    for s in range(10):
        bat.step(s)
        sim.step(s)
    d = bat.diagnostics()[0]
    csd, fe, out = sim.diag()
    assert list(d.csd) == list(csd)
    assert list(d.fe_hist) == list(fe)
    assert d.w_e == int(out[0]) and d.w_i == int(out[1]) and d.sum_z == int(out[2])
    assert d.ke_ev == out[4]
    assert d.te_ev == out[5]


def test_capacity_overflow_leaves_cell_unchanged(ctx):
    # a cell whose ionization needs more slots than its slab fails visibly: the
    # oracle accepts more ionizations than the two spare slots of a 32-slot
    # slab holding 30 electrons, so the step must flag XP_ST_CAPACITY and
    # leave every particle of the batch as it was
    spec, parts = cases.one_run(2, 30, 30, 3000.0, 1.0, seed=79, e_weight=3)
    sim = O.Sim(ctx.tables, spec)
    sim.bin(parts)
    sim.step(0, O.ION)
    acc = sim.counters()[0][:, O.COUNTERS.index("ION_ACCEPTED")]
    assert (30 + acc > 32).all(), acc
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(0, 0))
    before = bat.state()
    bat.step(0, O.ION)
    torch.cuda.synchronize()
    after = bat.state()
    assert bat.status() & B.XP_ST_CAPACITY
    for f in ("e_start", "evx", "evy", "evz", "ew", "iz", "ik", "ivx", "ex"):
        assert np.array_equal(getattr(before, f), getattr(after, f)), f


def test_lotz_full_form_parity(ctx):
    # the Lotz factor (1 - b exp(-c (E/P - 1))) of Eq. 4 with b, c != 0 on
    # the LDS step (C1, where the keV source electrons ionize every step) and
    # on the global-memory path
    import dataclasses
    tb = dataclasses.replace(ctx.tables,
                             lotz_b=np.array([0.7, 0.45, 0.6, 0.35, 0.25]),
                             lotz_c=np.array([0.3, 1.1, 0.85, 0.5, 2.0]))
    c2 = RT.Context(tb)
    spec, parts = W.config_c1()
    bat, sim = run_pair(c2, spec, parts, 20, check_every=5, capacity=(3, 16), label="C1/lotz-bc")
    assert bat.run_counters()[0][O.COUNTERS.index("ION_ACCEPTED")] > 0
    run_pair(c2, spec, parts, 6, check_every=3, capacity=(3, 16), label="C1/lotz-bc/global",
             schedule=3, big="all")
    spec, parts = W.config_c2(nx=6, ny=6)
    run_pair(c2, spec, parts, 8, check_every=4, label="C2r/lotz-bc")


def test_recombination_selection_lds(ctx):
    # three-body recombination on the LDS step: the first step recombines
    # 11-78 times per cell (more than the extraction limit of 12 in most
    # cells, the full-sort path), the second 1-8 times (the extraction path);
    # a wave and a block per cell
    ne = [200, 120, 90, 60, 33, 140]
    ni = [60, 100, 40, 30, 50, 12]
    for sched in (0, 1, 2):
        spec, parts = cases.one_run(6, ne, ni, 2.0, 0.1, seed=96, z0=4, e_weight=1)
        parts.iz[:] = np.random.default_rng(3).integers(3, 8, parts.ni)
        bat, sim = run_pair(ctx, spec, parts, 3, check_every=1, schedule=sched,
                            flags=O.ALL & ~(O.PHOTO | O.DECAY), label="rec/lds/%d" % sched)
        rec = bat.run_counters()[0][O.COUNTERS.index("REC")]
        assert rec == 46 + 78 + 34 + 24 + 11 + 1 + 8, rec
    # (C1 recombines a few times per cell and step from step 55 on, through
    # both paths: test_c1_parity)


def test_relativistic_collisions(ctx):
    # the relativistic variant of S1/S2 (XP_REL): C1 (1.35-1.5 keV source
    # electrons), keV-hot cells under the wave, block and lane-group schedules
    # with and without Nanbu's law, the global-memory path, a reduced C2
    spec, parts = W.config_c1()
    run_pair(ctx, spec, parts, 30, flags=O.ALL | O.REL, check_every=10, capacity=(3, 16),
             label="C1/rel")
    for sched in (1, 2, 5):
        for law in (O.REL, O.REL | O.NANBU):
            rng = np.random.default_rng(61)
            ne = rng.integers(1, 14, 10)
            ni = rng.integers(1, 7, 10)
            spec, parts = cases.one_run(10, ne, ni, 8000.0, 5.0, seed=62, lnl=4.0, dt=0.05e-15)
            parts.iz[:] = rng.integers(3, 12, parts.ni)
            parts.ew[:] = rng.choice([1, 2, 3], parts.ne)
            run_pair(ctx, spec, parts, 6, flags=O.ALL | law, check_every=2, capacity=(5, 4),
                     schedule=sched, label="rel/%d/%d" % (sched, law))
    run_pair(ctx, spec, parts, 6, flags=O.ALL | O.REL, check_every=3, capacity=(5, 16),
             schedule=3, big="all", label="rel/global")
    ne = np.array([60, 3000, 2600, 45, 0])
    ni = np.array([50, 1500, 600, 40, 20])
    spec, parts = cases.one_run(ne.size, ne, ni, 2000.0, 0.1, seed=98, e_weight=1, dt=0.05e-15,
                                photon_hv=(1850.0,), photon_n=(4e29,))
    bat, _ = run_pair(ctx, spec, parts, 4, check_every=2, label="oversized/rel",
                      flags=O.ALL | O.REL | O.NANBU)
    assert bat.stats()[2] == 2
    spec, parts = W.config_c2(nx=6, ny=6)
    run_pair(ctx, spec, parts, 10, flags=O.ALL | O.REL, check_every=5, label="C2r/rel")


def test_recombination_cross_section(ctx):
    # three-body recombination from the detailed-balance rate per charge
    # state (XP_REC_XS, with the per-charge-state ionization of XP_ION_Z):
    # cold dense cells where tens to hundreds of ions fire per step and some
    # charge states clamp P at 1, under the wave, block, two-wave and
    # lane-group schedules; C1 through the step where its electrons have
    # cooled enough to recombine; a reduced C2
    flags = (O.ALL & ~(O.PHOTO | O.DECAY)) | O.ION_Z | O.REC_XS
    ne = [200, 120, 90, 60, 33, 140]
    ni = [60, 100, 40, 30, 50, 12]
    for sched in (0, 1, 2, 5):
        spec, parts = cases.one_run(6, ne, ni, 1.0, 0.1, seed=96, z0=4, e_weight=1,
                                    n_i=W.SOLID_NI * 4)
        parts.iz[:] = np.random.default_rng(3).integers(3, 12, parts.ni)
        bat, sim = run_pair(ctx, spec, parts, 3, check_every=1, schedule=sched, flags=flags,
                            label="recxs/%d" % sched)
        rc = bat.run_counters()[0]
        assert rc[O.COUNTERS.index("REC")] > 0 and rc[O.COUNTERS.index("P_CLAMPED")] > 0
    spec, parts = W.config_c1()
    bat, _ = run_pair(ctx, spec, parts, 60, flags=O.ALL | O.ION_Z | O.REC_XS, check_every=20,
                      capacity=(3, 16), label="C1/recxs")
    assert bat.run_counters()[0][O.COUNTERS.index("REC")] > 0
    spec, parts = W.config_c2(nx=6, ny=6)
    run_pair(ctx, spec, parts, 10, flags=O.ALL | O.ION_Z | O.REC_XS, check_every=5,
             label="C2r/recxs")
