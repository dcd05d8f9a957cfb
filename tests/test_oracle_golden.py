"""Pins of the oracle against figures the paper states (tests/golden/).

Each figure is checked on the oracle's own step, not on a formula retyped
here:
* cold K-edge (Sec. VI.A): on cold solid Al3+, photons 10 eV below the stated
  edge open no K shell, photons 10 eV above it do;
* photoelectrons at 1700 eV (Sec. VI.C): every K-shell photoelectron a step
  emits carries less than the stated bound;
* KLL Auger energy (Sec. VI.C): every Auger electron a step emits from Al3+
  with one K vacancy lies within the stated band.
"""

import os

import numpy as np

from tests import cases

QE = 1.602176634e-19
ME = 9.1093837015e-31
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, value, tol, unit = line.split()[:4]
            out[name] = (float(value), float(tol), unit)
    return out


def _new_energies(st0, st1):
    new = slice(st0.ew.size, st1.ew.size)
    return 0.5 * ME * (st1.evx[new] ** 2 + st1.evy[new] ** 2 + st1.evz[new] ** 2) / QE


def _photo_step(orc, tables, hv, seed):
    n = 4000
    # charge-neutral solid Al3+: n macro-electrons of 3 weight units per n ions
    spec, parts = cases.one_run(1, n, n, 10.0, 0.1, e_weight=3, seed=seed, dt=0.1e-15,
                                photon_hv=(hv,), photon_n=(3e29,))
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    st0 = sim.state()
    sim.step(0, orc.PHOTO)
    cnt, _ = sim.counters()
    return dict(zip(orc.COUNTERS, cnt[0])), _new_energies(st0, sim.state())


def test_golden_file_entries():
    g = _golden()
    assert set(g) == {"cold_k_edge", "photoelectron_max_1700", "kll_auger_energy"}
    assert all(u == "eV" for _, _, u in g.values())


def test_cold_k_edge(orc, tables):
    edge, tol, _ = _golden()["cold_k_edge"]
    below, _ = _photo_step(orc, tables, edge - tol, seed=81)
    above, _ = _photo_step(orc, tables, edge + tol, seed=82)
    assert below["PHOTO_1S"] == 0
    assert above["PHOTO_1S"] > 100
    # below the K-edge the L shell still absorbs
    assert below["PHOTO_2P"] > 0


def test_photoelectrons_at_1700_ev(orc, tables):
    bound, _, _ = _golden()["photoelectron_max_1700"]
    c, e = _photo_step(orc, tables, 1700.0, seed=83)
    assert c["PHOTO_1S"] > 100
    k_shell = e[e < 1000.0]          # L-shell photoelectrons carry most of hv
    assert k_shell.size == c["PHOTO_1S"]
    assert np.all(k_shell < bound)
    assert np.all(k_shell > 0.0)


def test_kll_auger_energy(orc, tables):
    centre, tol, _ = _golden()["kll_auger_energy"]
    n = 20000
    spec, parts = cases.one_run(1, n, n, 10.0, 0.1, e_weight=3, k0=1, seed=84, dt=0.1e-15)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    st0 = sim.state()
    sim.step(0, orc.DECAY)
    cnt, _ = sim.counters()
    c = dict(zip(orc.COUNTERS, cnt[0]))
    e = _new_energies(st0, sim.state())
    assert c["AUGER"] > 0 and e.size == c["AUGER"]
    assert np.all(np.abs(e - centre) < tol)
