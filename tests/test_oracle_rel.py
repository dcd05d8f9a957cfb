"""Pins of the oracle's relativistic binary collision (variant REL, Sec. IV:
the cited collision model is relativistic and weighted).

* Equal weights: total relativistic energy sum gamma m c^2 and momentum sum
  gamma m v are conserved per collision to rounding, from 10 eV to 1 MeV.
* A pair already in its centre-of-momentum frame keeps |p| and is turned by
  the angle of Takizuka-Abe's law drawn from <delta^2> = s / 2.
* For v << c the collision is Takizuka-Abe's: same <delta^2> and the same
  velocities up to O((v/c)^2).
* The scattering parameter s against an independent 40-digit evaluation
  (mpmath) that boosts 4-momenta with the Lorentz matrix.
* Whole steps at keV temperatures against the naive third implementation,
  which boosts 4-vectors and rotates in an explicit orthonormal frame.
"""

import math

import numpy as np
import pytest

from tests import brute, cases

QE = 1.602176634e-19
ME = 9.1093837015e-31
MAL = 26.9815385 * 1.66053906660e-27
EPS0 = 8.8541878128e-12
C = 299792458.0


def _speed(ek_ev, m):
    g = 1.0 + ek_ev * QE / (m * C * C)
    return C * math.sqrt(1.0 - 1.0 / (g * g))


def _e_p(v, m):
    g = 1.0 / math.sqrt(1.0 - float(np.dot(v, v)) / C ** 2)
    return g * m * C * C, g * m * np.asarray(v)


def _qq(ma, mb, lnl=5.0, dt=1e-16, zb=1):
    mab = ma * mb / (ma + mb)
    return (QE ** 4) * zb * zb * lnl * dt / (8 * math.pi * EPS0 ** 2 * mab ** 2)


def _draws(rng):
    return rng.integers(0, 1 << 32, 4, dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("mb", [ME, MAL])
def test_rel_conserves_energy_and_momentum(orc, mb):
    rng = np.random.default_rng(7)
    worst_e = worst_p = 0.0
    for ek in (10.0, 300.0, 1.5e3, 8e3, 1e5, 1e6):
        for _ in range(300):
            va = rng.normal(size=3)
            va *= _speed(ek, ME) / np.linalg.norm(va)
            vb = rng.normal(size=3)
            vb *= _speed(ek * rng.uniform(0.01, 1.0), mb) / np.linalg.norm(vb)
            ea, pa = _e_p(va, ME)
            eb, pb = _e_p(vb, mb)
            a, b, d2, aa, ab = orc.collide(va, vb, ME, mb, 1, 1, _qq(ME, mb), 1e28, _draws(rng), 2)
            assert d2 > 0 and aa == 1 and ab == 1
            ea2, pa2 = _e_p(a, ME)
            eb2, pb2 = _e_p(b, mb)
            worst_e = max(worst_e, abs((ea2 + eb2) - (ea + eb)) / (ea + eb))
            scale = np.abs(pa).sum() + np.abs(pb).sum()
            worst_p = max(worst_p, float(np.abs((pa2 + pb2) - (pa + pb)).max()) / scale)
    assert worst_e < 4e-15, worst_e
    assert worst_p < 4e-15, worst_p


def test_rel_in_com_frame_turns_by_the_drawn_angle(orc):
    rng = np.random.default_rng(8)
    for ek in (50.0, 5e3, 5e5):
        for _ in range(200):
            # equal masses with opposite momenta: the centre of momentum is at rest
            va = rng.normal(size=3)
            va *= _speed(ek, ME) / np.linalg.norm(va)
            vb = -va
            d = _draws(rng)
            a, b, d2, _, _ = orc.collide(va, vb, ME, ME, 1, 1, _qq(ME, ME), 1e28, d, 2)
            # Takizuka-Abe's law from <delta^2> = d2, with the oracle's own
            # log and sin/cos (the same elementary functions on both sides)
            r1 = (float(d[0]) + 0.5) * 2.0 ** -32
            _, c2 = orc.sincos2pi(int(d[1]) << 20)
            g = math.sqrt(-2.0 * orc.log(r1)) * c2
            dl = math.sqrt(d2) * g
            omc = 2 * dl * dl / (1 + dl * dl)
            cos_chi = float(np.dot(a, va)) / (np.linalg.norm(a) * np.linalg.norm(va))
            assert cos_chi == pytest.approx(1.0 - omc, abs=2e-14)
            assert np.linalg.norm(a) == pytest.approx(np.linalg.norm(va), rel=1e-14)
            assert np.allclose(b, -a, rtol=1e-13, atol=0.0)


@pytest.mark.parametrize("law", [0, 1])
def test_rel_reduces_to_nonrelativistic_law(orc, law):
    rng = np.random.default_rng(9)
    for mb in (ME, MAL):
        for _ in range(300):
            beta = 10 ** rng.uniform(-5, -3.5)
            va = rng.normal(size=3)
            va *= beta * C / np.linalg.norm(va)
            vb = rng.normal(size=3)
            vb *= beta * C * rng.uniform(0.0, 1.0) * math.sqrt(ME / mb) / np.linalg.norm(vb)
            d = _draws(rng)
            q = _qq(ME, mb)
            a0, b0, d20, _, _ = orc.collide(va, vb, ME, mb, 1, 1, q, 1e26, d, law)
            a1, b1, d21, _, _ = orc.collide(va, vb, ME, mb, 1, 1, q, 1e26, d, law | 2)
            assert d21 == pytest.approx(d20, rel=50 * beta * beta + 1e-12)
            dv = np.linalg.norm(a0 - va) + 1e-300
            assert np.linalg.norm(a1 - a0) <= (50 * beta * beta + 1e-9) * max(dv, 1e-6 * np.linalg.norm(va))


def test_rel_scattering_parameter_against_mpmath(orc):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = np.random.default_rng(10)
    c = mp.mpf(C)
    for mb in (ME, MAL):
        for _ in range(60):
            ek = 10 ** rng.uniform(1, 6)
            va = rng.normal(size=3)
            va *= _speed(ek, ME) / np.linalg.norm(va)
            vb = rng.normal(size=3)
            vb *= _speed(ek * rng.uniform(0.01, 1), mb) / np.linalg.norm(vb)
            q = _qq(ME, mb)
            _, _, d2, _, _ = orc.collide(va, vb, ME, mb, 2, 3, q, 1e27, _draws(rng), 2)

            def four(v, m):
                v = [mp.mpf(float(x)) for x in v]
                g = 1 / mp.sqrt(1 - (v[0] ** 2 + v[1] ** 2 + v[2] ** 2) / c ** 2)
                return g, [g * m * c] + [g * m * x for x in v]

            ma_, mb_ = mp.mpf(ME), mp.mpf(mb)
            ga, pa = four(va, ma_)
            gb, pb = four(vb, mb_)
            beta = [(pa[k] + pb[k]) / (pa[0] + pb[0]) for k in (1, 2, 3)]
            b2 = sum(x * x for x in beta)
            gc = 1 / mp.sqrt(1 - b2)

            def boost(p):
                bx = sum(beta[k] * p[k + 1] for k in range(3))
                t = gc * (p[0] - bx)
                k_ = (gc - 1) * bx / b2 - gc * p[0]
                return [t] + [p[k + 1] + k_ * beta[k] for k in range(3)]

            sa, sb = boost(pa), boost(pb)
            p = mp.sqrt(sum(x * x for x in sa[1:]))
            gas, gbs = sa[0] / (ma_ * c), sb[0] / (mb_ * c)
            mab = ma_ * mb_ / (ma_ + mb_)
            n = 3 * mp.mpf(1e27)
            s = (2 * mp.mpf(q) * n * mab ** 2 / (ma_ * ga * mb_ * gb) * gc * p / (ma_ * ga + mb_ * gb)
                 * (ma_ * gas * mb_ * gbs * c * c / p ** 2 + 1) ** 2 / c ** 4)
            assert d2 == pytest.approx(float(s / 2), rel=1e-12)


def test_rel_steps_match_brute_force_at_kev(orc, tables):
    # keV electrons (v/c up to 0.2) through whole steps: the oracle against
    # the third implementation's 4-vector boosts
    from tests.test_oracle_brute import _cells_from_state
    rng = np.random.default_rng(47)
    ncell = 6
    ne = rng.integers(2, 7, ncell)
    ni = rng.integers(1, 4, ncell)
    spec, parts = cases.one_run(ncell, ne, ni, 8000.0, 2.0, seed=47, ipd=1, lnl=4.0, dt=0.1e-15)
    parts.iz[:] = rng.integers(3, 10, parts.ni)
    parts.ew[:] = rng.choice([1, 3], parts.ne)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    cells = _cells_from_state(sim.state())
    bf = brute.Brute(tables, spec)
    flags = orc.EE | orc.EI | orc.REL
    moved = 0.0
    for step in range(4):
        for c, cell in enumerate(cells):
            bf.step(c, cell, step, flags)
        v0 = sim.state().evx.copy()
        sim.step(step, flags)
        st = sim.state()
        moved = max(moved, float(np.abs(st.evx - v0).max()))
        for c, cell in enumerate(cells):
            e0, e1 = st.e_start[c], st.e_start[c + 1]
            ve = np.array([[e[2], e[3], e[4]] for e in cell.e]).reshape(-1, 3)
            vo = np.stack([st.evx[e0:e1], st.evy[e0:e1], st.evz[e0:e1]], axis=1)
            assert np.abs(ve - vo).max() <= 1e-9 * np.abs(ve).max(), (step, c)
    assert moved > 1e5
