"""GPU parity of the global-memory path (cells beyond one workgroup's LDS).

Two ways in: schedule 3 sends every cell of a batch through it, so the
workloads of the LDS parity tests check it cell for cell; and cells with more
particles than the largest LDS plan take it by themselves, beside small cells
that stay in LDS.  Same bar as the LDS path: counts, weights, charge states,
counters and moments identical, velocities identical to 1e-12 relative.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import binding as B
from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import workloads as W
from tests import cases
from tests.test_gpu_parity import compare, ctx, run_pair, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_big_path_c1(ctx):
    spec, parts = W.config_c1()
    run_pair(ctx, spec, parts, 30, check_every=10, capacity=(3, 16), label="C1/global",
             schedule=3, big="all")


def test_big_path_c2_reduced(ctx):
    spec, parts = W.config_c2(nx=8, ny=6)
    run_pair(ctx, spec, parts, 24, check_every=8, label="C2r/global", schedule=3, big="all")


def test_big_path_edge_cells(ctx):
    rng = np.random.default_rng(5)
    ne = np.array([0, 1, 2, 3, 0, 5, 7, 1, 0, 64, 65, 129])
    ni = np.array([0, 0, 1, 1, 3, 2, 7, 1, 1, 63, 1, 3])
    spec, parts = cases.one_run(ne.size, ne, ni, 200.0, 1.0, seed=78, lnl=3.0,
                                photon_hv=(1800.0,), photon_n=(3e30,))
    parts.iz[:] = rng.integers(3, 14, parts.ni)
    parts.ik[:] = np.where(parts.iz < 12, rng.integers(0, 2, parts.ni), 0)
    parts.ew[:] = rng.choice([1, 2, 3], parts.ne)
    run_pair(ctx, spec, parts, 12, check_every=1, label="edge/global", schedule=3, big="all")


def test_big_path_recombination(ctx):
    # cold electrons around highly charged ions: Zbar_EOS far below Zbar, so
    # three-body recombination removes electrons every step
    spec, parts = cases.one_run(3, [1800, 700, 90], [600, 1200, 40], 2.0, 0.1, seed=91, z0=6,
                                e_weight=1)
    bat, sim = run_pair(ctx, spec, parts, 6, check_every=1, label="rec/global", schedule=3,
                        big="all", flags=O.ALL & ~(O.PHOTO | O.DECAY))
    # the ions reach the Z = 3 floor within a few steps: count over the run
    assert bat.run_counters()[0][O.COUNTERS.index("REC")] > 0


def test_big_path_recombination_many(ctx):
    # thousands of recombinations per cell and step (5000, 8000 and 700 in the
    # first step, up to every eligible ion; 3977 and 450 in the second): the
    # REC_E and REC_I ranks taken from candidates across many chunks, the
    # ordered sum of the pair energies over several 512-term spans with ragged
    # tails, and the drift-frame rescale of the survivors as they are compacted
    spec, parts = cases.one_run(3, [20000, 9000, 3300], [5000, 8000, 700], 2.0, 0.1, seed=93,
                                z0=6, e_weight=1)
    bat, _ = run_pair(ctx, spec, parts, 3, check_every=1, label="rec/global/many", schedule=3,
                      big="all", flags=O.ALL & ~(O.PHOTO | O.DECAY))
    assert bat.run_counters()[0][O.COUNTERS.index("REC")] >= 18000


def test_oversized_cells_take_global_path(ctx):
    # cells beyond the LDS plans (1500 ions; 2600 electrons; 9000 electrons)
    # beside small cells that stay in LDS
    ne = np.array([60, 3000, 2600, 9000, 45, 0])
    ni = np.array([50, 1500, 600, 500, 40, 20])
    spec, parts = cases.one_run(ne.size, ne, ni, 30.0, 0.1, seed=93, e_weight=1, dt=0.05e-15,
                                photon_hv=(1850.0,), photon_n=(4e29,))
    bat, sim = run_pair(ctx, spec, parts, 8, check_every=2, label="oversized")
    st = bat.stats()
    assert st[2] == 3, "cells on the global-memory path: %s" % st
    d = bat.diagnostics()[0]
    csd, fe, out = sim.diag()
    assert list(d.fe_hist) == list(fe)
    assert d.ke_ev == out[4]
    assert d.te_ev == out[5]


def test_big_path_thermalization(ctx):
    # the forced thermalization of Sec. VI.C through the global-memory path:
    # C1 and edge cells with every cell on the path, then oversized cells
    # beside LDS cells
    from tests.test_gpu_parity import _therm_edge_case
    spec, parts = W.config_c1()
    run_pair(ctx, spec, parts, 8, check_every=4, capacity=(3, 16), label="C1/global/therm",
             schedule=3, big="all", flags=O.ALL | O.THERM)
    spec, parts = _therm_edge_case(43)
    bat, sim = run_pair(ctx, spec, parts, 6, check_every=1, capacity=(3, 4), label="therm/global",
                        schedule=3, big="all", flags=O.ALL | O.THERM)
    oc = sim.counters()[0]
    assert oc[:, O.COUNTERS.index("THERM_SKIPPED")].sum() > 0
    ne = np.array([60, 3000, 2600, 45, 0])
    ni = np.array([50, 1500, 600, 40, 20])
    spec, parts = cases.one_run(ne.size, ne, ni, 30.0, 0.1, seed=95, e_weight=1, dt=0.05e-15,
                                photon_hv=(1850.0,), photon_n=(4e29,))
    bat, sim = run_pair(ctx, spec, parts, 4, check_every=2, label="oversized/therm",
                        flags=O.ALL | O.THERM)
    assert bat.stats()[2] == 2


def test_big_path_per_charge_state_ionization(ctx):
    from tests.test_gpu_parity import _mixed_charge_case
    spec, parts = _mixed_charge_case(53)
    bat, sim = run_pair(ctx, spec, parts, 8, check_every=1, label="ionz/global", schedule=3,
                        big="all", flags=O.ALL | O.ION_Z)
    assert (sim.moments()[:, 11] > 1).any()
    spec, parts = W.config_c1()
    parts.iz[:] = np.random.default_rng(7).integers(3, 9, parts.ni)
    run_pair(ctx, spec, parts, 8, check_every=4, capacity=(3, 16), label="C1/global/ionz+therm",
             schedule=3, big="all", flags=O.ALL | O.ION_Z | O.THERM)


def test_big_path_capacity_flag(ctx):
    spec, parts = cases.one_run(2, 30, 30, 3000.0, 1.0, seed=79, e_weight=3)
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(0, 0), big="all")
    bat.step(0, O.ION, schedule=3)
    torch.cuda.synchronize()
    st = bat.status()
    after = bat.state()
    # the oracle accepts more ionizations than the slabs' two spare slots
    # (test_capacity_overflow_leaves_cell_unchanged): the overflow is flagged
    # and the electron count kept
    assert st == B.XP_ST_CAPACITY
    assert bat.run_status()[0] == B.XP_ST_CAPACITY
    assert after.e_start[-1] == parts.ne


def test_big_path_nanbu(ctx):
    # Nanbu's scattering law through the global-memory path: C1 with every
    # cell on the path, then oversized cells beside LDS cells
    spec, parts = W.config_c1()
    run_pair(ctx, spec, parts, 6, check_every=3, capacity=(3, 16), label="C1/global/nanbu",
             schedule=3, big="all", flags=O.ALL | O.NANBU)
    ne = np.array([60, 3000, 2600, 45, 0])
    ni = np.array([50, 1500, 600, 40, 20])
    spec, parts = cases.one_run(ne.size, ne, ni, 30.0, 0.1, seed=97, e_weight=1, dt=0.05e-15,
                                photon_hv=(1850.0,), photon_n=(4e29,))
    bat, sim = run_pair(ctx, spec, parts, 4, check_every=2, label="oversized/nanbu",
                        flags=O.ALL | O.NANBU)
    assert bat.stats()[2] == 2


def test_big_path_recombination_cross_section(ctx):
    # XP_REC_XS on the global-memory path: hundreds of firing ions per cell
    # listed in slot order across chunks, fewer electrons than firing ions in
    # one cell, clamped charge states; every cell through the path, then the
    # same cells where only the large ones leave LDS
    flags = (O.ALL & ~(O.PHOTO | O.DECAY)) | O.ION_Z | O.REC_XS
    for big, sched in (("all", 3), ("auto", 0)):
        spec, parts = cases.one_run(3, [1800, 700, 90], [600, 1200, 40], 1.0, 0.1, seed=91,
                                    z0=8, e_weight=1, n_i=W.SOLID_NI * 4)
        bat, _ = run_pair(ctx, spec, parts, 4, check_every=1, label="recxs/global/" + big,
                          schedule=sched, big=big, flags=flags)
        rc = bat.run_counters()[0]
        assert rc[O.COUNTERS.index("REC")] > 0 and rc[O.COUNTERS.index("P_CLAMPED")] > 0
    spec, parts = cases.one_run(3, [1800, 700, 90], [600, 1200, 40], 0.5, 0.1, seed=91,
                                z0=10, e_weight=1, n_i=W.SOLID_NI * 20)
    run_pair(ctx, spec, parts, 3, check_every=1, label="recxs/global/dense", schedule=3,
             big="all", flags=flags)
    spec, parts = W.config_c1()
    run_pair(ctx, spec, parts, 6, flags=O.ALL | O.ION_Z | O.REC_XS, check_every=3,
             capacity=(3, 16), label="C1/recxs/global", schedule=3, big="all")
