"""Pins of the oracle's cross-section three-body recombination (variant
REC_XS: Sec. IV names a recombination model from interaction cross sections
as the step after its EOS-constrained one).

* exp(x) E1(x) against scipy.special.exp1 over 1e-6 .. 700.
* The recombination probability against an independent closed form: detailed
  balance with the Lotz ionization of Z-1, S_{Z-1}(T) n_e^2 dt / Phi_Z(T),
  with scipy's E1 and ground-configuration degeneracies from math.comb; with
  and without the b, c term of Eq. 4.
* A cell whose electrons are re-drawn from a fixed Maxwellian every step, with
  per-charge-state ionization (ION_Z) and REC_XS on, relaxes to the
  stationary distribution of the step's Markov chain, which is the
  Saha-Boltzmann distribution with the lowered potentials up to the O(P) terms
  of one ionization-then-recombination step.
* Charge and weight bookkeeping of the recombination step.
"""

import dataclasses
import math

import numpy as np
import pytest
from scipy import special

from tests import cases

# CODATA 2018 (the values the method is specified with)
QE = 1.602176634e-19
ME = 9.1093837015e-31
HBAR = 1.054571817e-34
CAP = [2, 2, 6, 2, 6]


def _g(orc, z):
    occ = orc.occupancy(z)
    r = 1
    for s in range(5):
        r *= math.comb(CAP[s], int(occ[s]))
    return r


def _lotz_rate(orc, tab, zl, tev, dE):
    occ = orc.occupancy(zl)
    vbar = math.sqrt(8 * tev * QE / (math.pi * ME))
    r = 0.0
    for s in range(5):
        if occ[s] == 0:
            continue
        p = max(tab.bind[zl, s] - dE[zl], 1.0)
        x, b, c = p / tev, tab.lotz_b[s], tab.lotz_c[s]
        br = special.exp1(x) - b * math.exp(c) * x / (x + c) * special.exp1(x + c)
        r += tab.lotz_a[s] * 1e-4 * occ[s] * vbar / (p * tev) * br
    return r


def _phi(orc, tab, z, tev, dE):
    zl = z - 1
    occ = orc.occupancy(zl)
    v = max(q for q in range(5) if occ[q] > 0)
    pv = max(tab.bind[zl, v] - dE[zl], 1.0)
    q = ME * tev * QE / (2 * math.pi * HBAR ** 2)
    return 2.0 * _g(orc, z) / _g(orc, zl) * q ** 1.5 * math.exp(-pv / tev)


def test_e1x_against_scipy(orc):
    xs = np.exp(np.linspace(math.log(1e-6), math.log(699.0), 3000))
    for x in xs:
        want = math.exp(x) * special.exp1(x)
        assert orc.e1x(x) == pytest.approx(want, rel=1e-13), x


def _rec_mp(orc, tab, z, tev, ne, dE, dt):
    """S_{z-1} n_e^2 dt / Phi_z in 30-digit arithmetic (no under- or overflow)."""
    import mpmath as mp
    mp.mp.dps = 30
    zl = z - 1
    occ = orc.occupancy(zl)
    T = mp.mpf(tev)
    vbar = mp.sqrt(8 * T * mp.mpf(QE) / (mp.pi * mp.mpf(ME)))
    S = mp.mpf(0)
    for s in range(5):
        if occ[s] == 0:
            continue
        p = mp.mpf(max(tab.bind[zl, s] - dE[zl], 1.0))
        x, b, c = p / T, mp.mpf(tab.lotz_b[s]), mp.mpf(tab.lotz_c[s])
        br = mp.e1(x) - b * mp.exp(c) * x / (x + c) * mp.e1(x + c)
        S += mp.mpf(tab.lotz_a[s]) * mp.mpf("1e-4") * occ[s] * vbar / (p * T) * br
    v = max(q for q in range(5) if occ[q] > 0)
    pv = mp.mpf(max(tab.bind[zl, v] - dE[zl], 1.0))
    q = mp.mpf(ME) * T * mp.mpf(QE) / (2 * mp.pi * mp.mpf(HBAR) ** 2)
    phi = 2 * mp.mpf(_g(orc, z)) / _g(orc, zl) * q ** mp.mpf(1.5) * mp.exp(-pv / T)
    return float(S * mp.mpf(ne) ** 2 * mp.mpf(dt) / phi)


@pytest.mark.parametrize("bc", [False, True])
def test_rec_probability_closed_form(orc, tables, bc):
    tab = tables
    if bc:
        tab = dataclasses.replace(tables, lotz_b=np.array([0.7, 0.45, 0.6, 0.35, 0.25]),
                                  lotz_c=np.array([0.3, 1.1, 0.85, 0.5, 2.0]))
    T = orc.Tables(tab)
    rng = np.random.default_rng(3)
    for _ in range(200):
        z = int(rng.integers(1, 14))
        tev = 10 ** rng.uniform(0, 3)
        ne = 10 ** rng.uniform(26, 30.5)
        dE = rng.uniform(0, 150, 13)
        dt = 1e-16
        got = T.rec_xs(z, tev, ne, dE, dt)
        want = _rec_mp(orc, tab, z, tev, ne, dE, dt)
        assert got == pytest.approx(want, rel=1e-11, abs=1e-300), (z, tev, ne)
    assert T.rec_xs(0, 30.0, 1e29, np.zeros(13), 1e-16) == 0.0
    assert T.rec_xs(5, 30.0, 0.0, np.zeros(13), 1e-16) == 0.0


def test_rec_xs_relaxes_to_saha_stationary_distribution(orc, tables):
    tev, dt, nsteps, ni, z0 = 40.0, 6e-17, 1200, 2000, 5
    spec, parts = cases.one_run(1, ni * z0, ni, tev, 0.5, seed=5, z0=z0, e_weight=1, dt=dt,
                                lnl=3.0, ipd=0)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    rng = np.random.default_rng(9)
    flags = orc.ION | orc.REC | orc.ION_Z | orc.REC_XS
    acc = np.zeros(14)
    expect = []
    sig = math.sqrt(tev * QE / ME)
    for s in range(nsteps):
        sim.step(s, flags)
        st = sim.state()
        m = sim.moments()[0]
        n = st.ew.size
        # the electrons are re-drawn from the fixed Maxwellian (frozen temperature)
        st.evx[:] = rng.normal(0, sig, n)
        st.evy[:] = rng.normal(0, sig, n)
        st.evz[:] = rng.normal(0, sig, n)
        sim.load(st)
        assert st.ew.sum() == st.iz.astype(np.int64).sum()       # charge neutrality
        if s < nsteps // 2:
            continue
        acc += np.bincount(st.iz, minlength=14)
        ne = st.ew.sum() * spec.w0 / spec.volume
        dE, tp = m[16:29], m[15]
        row = []
        for z in range(4, 10):
            # ionization z-1 -> z (S3, at the drawn temperature), then
            # recombination z -> z-1 (S4, at the temperature after S3): the
            # birth-death chain balances pi_z a_{z-1} (1 - b_z) = pi_z ... giving
            # pi_z / pi_{z-1} = a_{z-1} (1 - b_z) / ((1 - a_z) b_z)
            a = _lotz_rate(orc, tables, z - 1, tev, dE) * ne * dt
            b = _lotz_rate(orc, tables, z - 1, tp, dE) * ne * ne * dt / _phi(orc, tables, z, tp, dE)
            a2 = _lotz_rate(orc, tables, z, tev, dE) * ne * dt
            row.append(a * (1 - b) / ((1 - a2) * b))
        expect.append(row)
    expect = np.mean(expect, axis=0)
    pops = acc / (nsteps - nsteps // 2)
    checked = 0
    for k, z in enumerate(range(4, 10)):
        if pops[z - 1] < 150 or pops[z] < 150:
            continue
        ratio = acc[z] / acc[z - 1]
        assert ratio == pytest.approx(expect[k], rel=0.06), (z, ratio, expect[k])
        checked += 1
    assert checked >= 3
    # the step's O(P) terms are small here: Saha itself is within 8 %
    saha = [_phi(orc, tables, z, tev, dE) / ne for z in (5, 6)]
    assert acc[5] / acc[4] == pytest.approx(saha[0], rel=0.08)


def test_rec_xs_bookkeeping(orc, tables):
    # cold electrons around highly charged ions: many recombinations; each
    # takes one weight unit from one electron and one charge from one ion
    spec, parts = cases.one_run(4, [300, 150, 40, 7], [40, 30, 20, 10], 3.0, 0.1, seed=17,
                                z0=8, e_weight=1, dt=1e-16)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    st0 = sim.state()
    total_rec = 0
    charge = st0.ew.astype(np.int64).sum() - st0.iz.astype(np.int64).sum()
    for s in range(4):
        before = sim.state()
        sim.step(s, orc.REC | orc.REC_XS)
        st = sim.state()
        c = sim.counters()[0]
        rec = c[:, orc.COUNTERS.index("REC")]
        total_rec += int(rec.sum())
        assert before.iz.astype(np.int64).sum() - st.iz.astype(np.int64).sum() == rec.sum()
        assert before.ew.astype(np.int64).sum() - st.ew.astype(np.int64).sum() == rec.sum()
        assert st.ew.astype(np.int64).sum() - st.iz.astype(np.int64).sum() == charge
        # at most one recombination per electron of the cell
        assert (rec <= np.diff(before.e_start)).all()
    assert total_rec > 10
    assert (sim.state().iz >= 3).all()
