"""Pins of the oracle's per-charge-state collisional ionization (ION_Z): the
Lotz cross section of every ion's own charge state instead of the average
cell ion (Sec. IV; the paper's stated simplification, lifted).

* With every ion in one charge state the variant is the average-ion step,
  bit for bit.
* With mixed charge states, the ions of each state fire at the Maxwellian
  rate of their own cross section (E1 closed form), within binomial noise,
  while the average-ion step fires all states at one rate.
"""

import math

import numpy as np
import pytest

from tests import cases
from tests.test_oracle_step import _lotz_rate


def test_one_charge_state_equals_average_ion(orc, tables):
    outs = []
    for flags in (orc.ALL, orc.ALL | orc.ION_Z):
        spec, parts = cases.one_run(6, 300, 100, 80.0, 0.1, seed=21, dt=0.05e-15,
                                    photon_hv=(1800.0,), photon_n=(1e30,))
        sim = orc.Sim(tables, spec)
        sim.bin(parts)
        sim.step(0, flags)
        cnt, led = sim.counters()
        outs.append((sim.state(), cnt, led, sim.moments()))
    (a, ca, la, ma), (b, cb, lb, mb) = outs
    for f in ("evx", "evy", "evz", "ew", "iz", "ik", "e_start"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.array_equal(ca, cb) and np.array_equal(la, lb)
    keep = [k for k in range(ma.shape[1]) if k != 11]
    assert np.array_equal(ma[:, keep], mb[:, keep])
    assert np.all(mb[:, 11] == 1)


def _mixed(orc, tables, flags, seed):
    n_i = 9000
    spec, parts = cases.one_run(1, 30000, n_i, 60.0, 0.1, seed=seed, dt=0.05e-15, e_weight=1)
    parts.iz[:] = np.repeat([3, 7, 10], n_i // 3)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    st0 = sim.state()
    sim.step(0, flags)
    st1 = sim.state()
    m = sim.moments()[0]
    cnt, _ = sim.counters()
    fired = {z: int(((st0.iz == z) & (st1.iz == z + 1)).sum()) for z in (3, 7, 10)}
    return spec, st0, m, dict(zip(orc.COUNTERS, cnt[0])), fired


def test_per_charge_state_rates(orc, tables):
    spec, st0, m, c, fired = _mixed(orc, tables, orc.ION | orc.ION_Z, 33)
    assert c["ION_STARVED"] == 0 and m[11] == 3
    ke0, _ = cases.kinetic(st0, tables.mass_ion)
    tev = 2.0 * ke0 / (3.0 * st0.ew.sum())
    n_e = st0.ew.sum() * spec.w0 / spec.volume
    n = 3000
    ps = {}
    for z in (3, 7, 10):
        p = n_e * _lotz_rate(tables, z, m[16 + z], tev) * spec.dt
        ps[z] = p
        assert abs(fired[z] - n * p) < 5 * math.sqrt(n * p * (1 - p)), (z, fired[z], n * p)
    assert m[12] == pytest.approx(max(ps.values()), rel=0.05)
    # the states differ enough for the test to tell them apart
    assert abs(ps[3] - ps[10]) > 5 * math.sqrt(n * ps[3]) / n
    # the average-ion step fires every state at the one rate of Z_c = 7
    spec, st0, m, c, fired = _mixed(orc, tables, orc.ION, 33)
    p4 = m[12]
    for z in (3, 7, 10):
        assert abs(fired[z] - n * p4) < 5 * math.sqrt(n * p4 * (1 - p4)), (z, fired[z])
