"""Pins of the oracle's reduced radiation transport (the photon bookkeeping of
Sec. III with a quasi-static Beer-Lambert profile along the beam).

* Beer-Lambert: a cold, uniform Al3+ target under a beam that ionizes few
  ions has, after one step, a mean field (1 - kappa dx)^i in cell i of a row,
  kappa = n_i sum_s N_b,s sigma_s(h nu) (ground configuration, every subshell
  below h nu), which is also exp(-kappa x) to O((kappa dx)^2 i).  kappa comes
  from the cross-section table, the expectation from Eq. 3's per-ion
  probability; the transport only sees the Monte-Carlo event counts.
* Cells without ions (vacuum) transmit exactly; a row of vacuum keeps the
  incident density.
* Saturable absorption: an intense beam strips the absorbing ions and the
  target becomes more transparent step by step, a weak beam does not
  (Sec. VI.A discusses this saturation).
"""

import math

import numpy as np

from paper_1704_01202_amd import workloads as W
from tests import cases

CL = 299792458.0


def _slab(nx, ny, ni, n_photon, seed, dt=0.1e-15):
    spec, parts = cases.one_run(nx, 2, ni, 10.0, 0.1, seed=seed, ny=ny, dt=dt,
                                photon_hv=(1850.0,), photon_n=(n_photon,), shuffle=False)
    return spec, parts


def test_beer_lambert_profile(orc, tables):
    nx, ny, ni = 64, 1000, 100
    spec, parts = _slab(nx, ny, ni, 1.0e30, 61)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    sim.step(0, orc.PHOTO)
    nabs = sim.absorbed()[:, 0]
    assert nabs.sum() > 0
    t = sim.transport()
    field = sim.cell_field()[:, 0].reshape(ny, nx) / 1.0e30
    T = orc.Tables(tables)
    sig = [T.photo_sigma(s, 1850.0) for s in range(3)]
    n_i = spec.w0 * ni / spec.volume
    kdx = n_i * (2 * sig[0] + 2 * sig[1] + 6 * sig[2]) * spec.dx
    # the per-ion probability stays far from its clamp, so the expectation holds
    assert CL * spec.dt_rad * 1.0e30 * 2 * sig[0] < 0.5
    mean = field.mean(axis=0)
    sd = field.std(axis=0) / math.sqrt(ny)
    i = np.arange(nx)
    expect = (1.0 - kdx) ** i
    assert field[:, 0].min() == 1.0 and field[:, 0].max() == 1.0
    assert np.all(np.abs(mean - expect) <= 5 * sd + 1e-15), np.abs(mean - expect).max()
    assert np.all(np.abs(mean - np.exp(-kdx * i)) <= 5 * sd + i * kdx * kdx)
    # the row transmission is the mean density leaving the rows
    assert abs(t[0] - (1.0 - kdx) ** nx) <= 5 * sd[-1] * 1.5
    assert 0.8 < t[0] < 0.9


def test_vacuum_transmits(orc, tables):
    nx, ny = 8, 3
    ni = np.zeros(nx * ny, dtype=int)
    ni[8:16] = 50                     # only the middle row holds ions
    spec, parts = cases.one_run(nx, 2, ni, 10.0, 0.1, seed=62, ny=ny, photon_hv=(1850.0,),
                                photon_n=(1.0e30,), shuffle=False)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    sim.step(0, orc.PHOTO)
    sim.transport()
    f = sim.cell_field()[:, 0].reshape(ny, nx)
    assert np.all(f[0] == 1.0e30) and np.all(f[2] == 1.0e30)
    assert f[1, 0] == 1.0e30 and np.all(np.diff(f[1]) <= 0.0) and f[1, -1] < 1.0e30
    # a second step with the attenuated field, then transport again
    sim.step(1, orc.PHOTO)
    t = sim.transport()
    assert 0.0 < t[0] < 1.0


def test_saturable_absorption(orc, tables):
    nx, ny, ni = 48, 40, 60
    out = {}
    for label, n in (("weak", 2.0e28), ("strong", 3.0e30)):
        spec, parts = _slab(nx, ny, ni, n, 63)
        sim = orc.Sim(tables, spec)
        sim.bin(parts)
        ts = []
        for s in range(12):
            sim.step(s, orc.PHOTO | orc.DECAY)
            ts.append(sim.transport()[0])
        out[label] = ts
    weak, strong = out["weak"], out["strong"]
    # weak beam: transmission stays at the cold value (within its noise)
    assert abs(weak[-1] - weak[1]) < 0.05
    # both start in the linear regime at the same cold transmission
    assert abs(strong[0] - weak[0]) < 0.03
    # strong beam: the absorbers deplete and the target opens up step by step
    assert strong[-1] > strong[0] + 0.06
    assert all(b >= a - 0.005 for a, b in zip(strong, strong[1:]))
    assert strong[-1] > weak[-1] + 0.05
