"""Pins of the oracle's Nanbu scattering law (variant of S1, S2).

Nanbu (Phys. Rev. E 55, 4642 (1997)) replaces the many small deflections of a
pair over one step by one angle chi whose cosine has the density
A exp(A cos chi) / (2 sinh A), with A fixed by the mean deflection
<cos chi> = coth A - 1/A = exp(-s).  The variant takes s = 2 <delta^2> of
Takizuka-Abe, so both laws agree on the mean of 1 - cos chi at small angles.

* A solves its defining equation: coth A - 1/A is evaluated in 50-digit
  decimal arithmetic at the oracle's A and compared with exp(-s).
* Samples follow the law: Kolmogorov-Smirnov against the distribution
  function with A from an independent root finder, and the sample mean of
  cos chi against exp(-s); s >= 15 is isotropic.
* At small s the mean of 1 - cos chi equals Takizuka-Abe's.
* A collision conserves momentum and energy and keeps |u|.
* The whole step composes deflections: an electron-ion pair whose |u| is kept
  has, after n steps, <cos(u_n, u_0)> = exp(-n s) (each step's rotation has a
  uniform azimuth, so mean cosines multiply).  Takizuka-Abe's law misses this
  at s = 1, Nanbu's does not.
"""

import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import optimize, stats

from paper_1704_01202_amd import workloads as W
from tests import cases

QE, ME = cases.QE, cases.ME
EPS0 = 8.8541878128e-12


def _langevin_dec(a):
    getcontext().prec = 50
    a = Decimal(repr(a))
    e = (-2 * a).exp()
    return (1 + e) / (1 - e) - 1 / a


def test_a_solves_defining_equation(orc):
    getcontext().prec = 50
    grid = np.concatenate([np.logspace(-9, math.log10(0.05), 60), np.linspace(0.0501, 14.99, 240)])
    worst = 0.0
    for s in grid:
        a = orc.nanbu_a(float(s))
        assert a > 0.0
        lhs = _langevin_dec(a)
        m = Decimal(repr(-float(s))).exp()
        # compare the small side: 1 - L against 1 - exp(-s) for small s
        err = abs(((1 - lhs) - (1 - m)) / (1 - m)) if s <= 0.05 else abs((lhs - m) / m)
        worst = max(worst, float(err))
    assert worst < 1e-13, worst
    assert orc.nanbu_a(15.0) == 0.0 and orc.nanbu_a(40.0) == 0.0
    # A decreases with s (more deflection, flatter law)
    a = [orc.nanbu_a(float(s)) for s in grid]
    assert all(x > y for x, y in zip(a, a[1:]))


def _a_ref(s):
    """A by bracketing on coth A - 1/A = exp(-s) (math.tanh), independent of the
    oracle's Newton iteration."""
    m = math.exp(-s)

    def f(a):
        lang = a / 3.0 - a ** 3 / 45.0 if a < 1e-3 else 1.0 / math.tanh(a) - 1.0 / a
        return lang - m
    return optimize.brentq(f, 1e-12, 1e6, xtol=1e-15, rtol=1e-14)


@pytest.mark.parametrize("s", [0.02, 0.3, 1.0, 3.0, 8.0])
def test_samples_follow_the_law(orc, s):
    rng = np.random.default_rng(int(s * 1000) + 7)
    u = rng.random(20000) * (1 - 2 ** -40) + 2 ** -41
    cos = np.array([1.0 - orc.nanbu_omc(s, float(x)) for x in u])
    a = _a_ref(s)

    def cdf(c):
        # P(cos chi <= c) = (exp(A c) - exp(-A)) / (exp(A) - exp(-A))
        return np.expm1(a * (c + 1.0)) / math.expm1(2.0 * a)
    assert stats.kstest(cos, cdf).pvalue > 1e-3
    mean_sd = math.sqrt(max(np.var(cos), 1e-30) / cos.size)
    assert abs(cos.mean() - math.exp(-s)) < 5 * mean_sd + 1e-12


def test_isotropic_limit(orc):
    rng = np.random.default_rng(3)
    u = rng.random(20000) * (1 - 2 ** -40) + 2 ** -41
    for s in (15.0, 50.0):
        cos = np.array([1.0 - orc.nanbu_omc(s, float(x)) for x in u])
        assert stats.kstest(cos, stats.uniform(loc=-1.0, scale=2.0).cdf).pvalue > 1e-3
    assert orc.nanbu_omc(0.0, 0.5) == 0.0


def _random_pairs(rng, n):
    return rng.normal(0.0, 3.0e6, size=(n, 3)), rng.normal(0.0, 3.0e6, size=(n, 3))


def _draws(rng):
    return rng.integers(0, 2 ** 32, size=4, dtype=np.uint64).astype(np.uint32)


def test_small_angle_mean_matches_takizuka_abe(orc):
    # a fixed pair with <delta^2> = 1e-3: the mean of 1 - cos(theta) over draws
    # is 2 <delta^2> (1 + O(<delta^2>)) under both laws
    rng = np.random.default_rng(11)
    va, vb = np.array([2.0e6, 0.0, 0.0]), np.zeros(3)
    u = 2.0e6
    d2_target = 1e-3
    coef = d2_target * u ** 3
    omc = {0: [], 1: []}
    for _ in range(20000):
        d = _draws(rng)
        for law in (0, 1):
            a2, b2, d2, _, _ = orc.collide(va, vb, ME, ME, 1, 1, coef, 1.0, d, law)
            assert abs(d2 - d2_target) < 1e-15
            un = a2 - b2
            omc[law].append(1.0 - float(un @ (va - vb)) / (u * u))
    m0, m1 = np.mean(omc[0]), np.mean(omc[1])
    sd = math.sqrt(np.var(omc[0]) / 20000)
    assert abs(m0 - 2e-3) < 5 * sd + 2e-5
    assert abs(m1 - 2e-3) < 5 * sd + 2e-5
    assert abs(m1 - m0) < 7 * sd + 2e-5


@pytest.mark.parametrize("mb", [ME, W.M_AL])
def test_collision_conserves(orc, mb):
    rng = np.random.default_rng(5)
    va_all, vb_all = _random_pairs(rng, 300)
    for va, vb in zip(va_all, vb_all):
        coef = rng.choice([1e17, 1e19, 1e21])   # s from small angles to isotropic
        a2, b2, d2, aa, ab = orc.collide(va, vb, ME, mb, 1, 1, coef, 1.0, _draws(rng), 1)
        assert aa == 1 and ab == 1
        p0 = ME * va + mb * vb
        p1 = ME * a2 + mb * b2
        assert np.abs(p1 - p0).max() <= 1e-12 * (ME * np.abs(va).max() + mb * np.abs(vb).max())
        k0 = ME * (va @ va) + mb * (vb @ vb)
        k1 = ME * (a2 @ a2) + mb * (b2 @ b2)
        assert abs(k1 - k0) <= 1e-12 * k0
        assert abs(np.linalg.norm(a2 - b2) - np.linalg.norm(va - vb)) <= 1e-12 * np.linalg.norm(va - vb)


def _pair_run(orc, n_cells, speed, seed):
    """One electron (weight 1) and one Al3+ ion at rest per cell, electron speed
    fixed, isotropic direction; fixed Coulomb logarithm."""
    spec, parts = cases.one_run(n_cells, 1, 1, 10.0, 0.0, seed=seed, e_weight=1, lnl=5.0,
                                dt=0.1e-15)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(3, n_cells))
    d /= np.linalg.norm(d, axis=0)
    parts.evx[:], parts.evy[:], parts.evz[:] = speed * d
    parts.ivx[:] = parts.ivy[:] = parts.ivz[:] = 0.0
    return spec, parts


def _s_per_step(spec, speed):
    """s = 2 <delta^2> of the e-i pair (Takizuka-Abe variance, Z = 3)."""
    qe4 = QE ** 4
    mei = ME * W.M_AL / (ME + W.M_AL)
    kei = qe4 / (8.0 * math.pi * EPS0 ** 2 * mei ** 2)
    n_unit = spec.w0 / spec.volume
    return 2.0 * kei * 5.0 * spec.dt * 9.0 * n_unit / speed ** 3


@pytest.mark.parametrize("law,composes", [(1, True), (0, False)])
def test_step_composes_deflections(orc, tables, law, composes):
    n = 20000
    # electron speed giving s = 1 per step
    spec0, _ = _pair_run(orc, 2, 1.0e6, 1)
    speed = (_s_per_step(spec0, 1.0) / 1.0) ** (1.0 / 3.0)
    spec, parts = _pair_run(orc, n, speed, 21)
    s = _s_per_step(spec, speed)
    assert abs(s - 1.0) < 1e-9
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    st0 = sim.state()
    u0 = np.stack([st0.evx - st0.ivx, st0.evy - st0.ivy, st0.evz - st0.ivz])
    flags = orc.EI | (orc.NANBU if law else 0)
    for k in range(1, 4):
        sim.step(k - 1, flags)
        st = sim.state()
        u = np.stack([st.evx - st.ivx, st.evy - st.ivy, st.evz - st.ivz])
        nu, n0 = np.linalg.norm(u, axis=0), np.linalg.norm(u0, axis=0)
        assert np.abs(nu - n0).max() <= 1e-12 * n0.max()       # |u| kept
        cos = (u * u0).sum(axis=0) / (nu * n0)
        sd = math.sqrt(np.var(cos) / n)
        ok = abs(cos.mean() - math.exp(-k * s)) < 5 * sd
        if composes:
            assert ok, (k, cos.mean(), math.exp(-k * s))
        elif k == 1:
            # one Takizuka-Abe step at s = 1 leaves far more forward scattering
            assert cos.mean() - math.exp(-s) > 10 * sd
