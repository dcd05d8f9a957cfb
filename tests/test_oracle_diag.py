"""Pin of the oracle's run diagnostics (Sec. II, Sec. VI.B, Fig. 7-9).

The oracle's orc_diag is checked against plain numpy definitions on a
multi-cell state built to reach every branch:

* charge-state distribution: np.bincount of the ions' Z over 0..13;
* electron energy histogram: 64 logarithmic bins with edges
  0.1 eV * 10^(6 k / 64), k = 0..64, weighted by the electrons' weight units;
  energies below 0.1 eV (and E = 0) count in bin 0, energies above the last
  inner edge (including those beyond 1e5 eV) in bin 63;
* W_e = sum of weight units, W_i = number of ions, sum Z, Zbar = sum Z / W_i;
* K_e = sum over electrons of w m_e v^2 / 2 in eV (math.fsum as the exact
  reference), T_e = (2/3) K_e / W_e.
"""

import math

import numpy as np
import pytest

from tests import cases

QE = 1.602176634e-19
ME = 9.1093837015e-31


def _state(seed):
    rng = np.random.default_rng(seed)
    ne = np.array([0, 3, 40, 17, 1, 64, 0, 9, 33, 5])
    ni = np.array([2, 1, 20, 7, 0, 30, 4, 3, 11, 2])
    spec, parts = cases.one_run(ne.size, ne, ni, 30.0, 0.5, seed=seed, lnl=3.0)
    n = parts.ne
    # energies spread over 1e-3 .. 1e6 eV (log-uniform), isotropic directions
    e = 10.0 ** rng.uniform(-3.0, 6.0, n)
    mu = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * math.pi, n)
    v = np.sqrt(2 * e * QE / ME)
    st = np.sqrt(1 - mu * mu)
    parts.evx[:] = v * st * np.cos(ph)
    parts.evy[:] = v * st * np.sin(ph)
    parts.evz[:] = v * mu
    # a few electrons at rest (E = 0) and a few at exactly 1 eV and 1e5 eV
    parts.evx[:4] = parts.evy[:4] = parts.evz[:4] = 0.0
    parts.ew[:] = rng.integers(1, 7, n)
    parts.iz[:] = rng.integers(0, 14, parts.ni)
    parts.ik[:] = 0
    return spec, parts


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_diag_against_plain_definitions(orc, tables, seed):
    spec, parts = _state(seed)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    st = sim.state()
    csd, fe, out = sim.diag()

    want_csd = np.bincount(st.iz.astype(np.int64), minlength=14)
    assert np.array_equal(csd, want_csd)

    v2 = (st.evx * st.evx + st.evy * st.evy) + st.evz * st.evz
    e = (0.5 * ME / QE) * v2
    w = st.ew.astype(np.int64)
    edges = 0.1 * 10.0 ** (6.0 * np.arange(65) / 64.0)
    # no electron may sit within rounding of an inner edge, or the bin would
    # depend on the logarithm's last bit
    pos = e[e > 0]
    near = np.min(np.abs(pos[:, None] / edges[None, 1:64] - 1.0))
    assert near > 1e-9
    b = np.searchsorted(edges, e, side="right") - 1
    b = np.clip(b, 0, 63)
    want_fe = np.bincount(b, weights=w, minlength=64).astype(np.int64)
    assert np.array_equal(fe, want_fe)
    assert want_fe[0] > 0 and want_fe[63] > 0   # both clamps are exercised

    we, wi, sz = int(w.sum()), int(st.iz.size), int(st.iz.astype(np.int64).sum())
    assert out[0] == we and out[1] == wi and out[2] == sz
    assert out[3] == sz / wi
    ke = math.fsum((w.astype(np.float64) * e).tolist())
    assert out[4] == pytest.approx(ke, rel=1e-13)
    assert out[5] == pytest.approx((2.0 / 3.0) * ke / we, rel=1e-13)
    assert out[6] == spec.nx * spec.ny


def test_diag_empty_run(orc, tables):
    # no electrons and no ions at all: zero counts, Zbar and T_e 0
    spec, parts = cases.one_run(3, 0, 0, 10.0, 0.5, seed=3)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    csd, fe, out = sim.diag()
    assert not csd.any() and not fe.any()
    assert out[0] == 0 and out[1] == 0 and out[3] == 0.0 and out[4] == 0.0 and out[5] == 0.0
