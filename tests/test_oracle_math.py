"""Pins of the oracle's elementary functions and random numbers.

The oracle defines log, exp, cbrt and sin/cos of 2 pi u with its own
algorithms (so that an independent implementation can match it bit for bit);
here they are held against the C library and numpy's extended precision.
Philox4x32-10 is held against rocRAND's independent header-only engine.
"""

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ULP = np.finfo(np.float64).eps


def ulp_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    sp = np.spacing(np.abs(ref))
    return np.abs(got - ref) / sp


def test_log_vs_libm(orc):
    rng = np.random.default_rng(11)
    xs = np.concatenate([
        np.exp(rng.uniform(-700, 700, 20000)),
        rng.uniform(0.5, 2.0, 20000),
        1.0 + rng.uniform(-1e-6, 1e-6, 2000),
        np.array([1.0, 2.0, 0.5, math.sqrt(2.0), 5e-324, 2.2250738585072014e-308,
                  1.7976931348623157e308, 1e-300, 3.0, 10.0]),
    ])
    got = np.array([orc.log(x) for x in xs])
    ref = np.log(xs)
    err = ulp_err(got, ref)
    err[ref == 0.0] = np.abs(got[ref == 0.0]) / 5e-324
    assert orc.log(1.0) == 0.0
    assert err.max() <= 2.0, err.max()
    assert math.isinf(orc.log(0.0)) and orc.log(0.0) < 0
    assert math.isnan(orc.log(-1.0))


def test_exp_vs_libm(orc):
    rng = np.random.default_rng(12)
    xs = np.concatenate([rng.uniform(-700, 700, 20000), rng.uniform(-1, 1, 20000),
                         np.array([0.0, 1.0, -1.0, 709.0, -708.0, 1e-10])])
    got = np.array([orc.exp(x) for x in xs])
    ref = np.exp(xs)
    assert ulp_err(got, ref).max() <= 2.0
    assert orc.exp(0.0) == 1.0
    assert orc.exp(710.0) == math.inf
    assert orc.exp(-746.0) == 0.0
    # subnormal results stay within a few units of the smallest subnormal
    for x in (-720.0, -740.0):
        assert abs(orc.exp(x) - math.exp(x)) <= 4 * 5e-324 + 4 * ULP * math.exp(x)


def test_cbrt_vs_libm(orc):
    rng = np.random.default_rng(13)
    xs = np.concatenate([np.exp(rng.uniform(-700, 700, 20000)), rng.uniform(0.1, 10, 5000),
                         np.array([1.0, 8.0, 27.0, 0.125, 1e-310, 3.0])])
    got = np.array([orc.cbrt(x) for x in xs])
    ref = np.cbrt(xs)
    assert ulp_err(got, ref).max() <= 2.0
    assert orc.cbrt(8.0) == 2.0 and orc.cbrt(1.0) == 1.0
    assert orc.cbrt(0.0) == 0.0


def test_sincos2pi_vs_extended(orc):
    rng = np.random.default_rng(14)
    ks = np.concatenate([rng.integers(0, 1 << 52, 20000, dtype=np.int64),
                         np.array([0, 1, (1 << 50) - 1, 1 << 50, (1 << 51), (1 << 52) - 1,
                                   (1 << 49), (1 << 49) - 1, 3 << 50], dtype=np.int64)])
    two_pi = np.longdouble(2) * np.arccos(np.longdouble(-1))
    worst = 0.0
    for k in ks:
        s, c = orc.sincos2pi(int(k))
        t = (np.longdouble(int(k)) + np.longdouble(0.5)) / np.longdouble(2.0 ** 52)
        rs, rc = np.sin(two_pi * t), np.cos(two_pi * t)
        worst = max(worst, abs(float(np.longdouble(s) - rs)), abs(float(np.longdouble(c) - rc)))
        assert s * s + c * c == pytest.approx(1.0, abs=8 * ULP)
    assert worst <= 2.5 * ULP, worst


def test_u52_open_interval(orc):
    assert orc.u52(0, 0) == 2.0 ** -53
    assert orc.u52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert 0.0 < orc.u52(0, 4095) < 1.0


def _rocrand_ref(tmp_path, lines):
    src = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")
    inc = "/opt/rocm/include"
    if not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers not installed")
    exe = str(tmp_path / "rr")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + inc,
                    "-o", exe, src], check=True)
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout
    return np.array([[int(v) for v in l.split()] for l in out.strip().splitlines()],
                    dtype=np.uint64)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_philox_matches_rocrand(orc, tmp_path):
    rng = np.random.default_rng(15)
    n = 4000
    ctr = rng.integers(0, 1 << 32, (n, 4), dtype=np.uint64)
    key = rng.integers(0, 1 << 32, (n, 2), dtype=np.uint64)
    # the engine reaches counter word 1 through a 64-bit offset 4 (c0 | c1 << 32),
    # so word 1 stays below 2^30 here
    ctr[:, 1] &= (1 << 30) - 1
    ctr[:8] = 0
    ctr[8:16] = 0xFFFFFFFF
    ctr[8:16, 1] = (1 << 30) - 1
    key[:4] = 0
    # counters of the shape the method uses: (step, cell, index, purpose << 24 | sub)
    ctr[16:64, 3] = (rng.integers(1, 11, 48) << 24) | rng.integers(0, 4, 48)
    lines = ["%d %d %d %d %d %d" % (c[0], c[1], c[2], c[3], k[0], k[1]) for c, k in zip(ctr, key)]
    ref = _rocrand_ref(tmp_path, lines)
    got = orc.philox(ctr.astype(np.uint32), key.astype(np.uint32)).astype(np.uint64)
    assert np.array_equal(got, ref)


def test_philox_uniformity(orc):
    n = 200000
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = 7
    ctr[:, 1] = np.arange(n) % 997
    ctr[:, 2] = np.arange(n) // 997
    ctr[:, 3] = 5 << 24
    key = np.tile(np.array([[1, 0]], dtype=np.uint32), (n, 1))
    w = orc.philox(ctr, key)
    a = (w[:, 0].astype(np.uint64) << np.uint64(32)) | w[:, 1].astype(np.uint64)
    u = ((a >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
    hist, _ = np.histogram(u, bins=100, range=(0, 1))
    exp = n / 100
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 160  # 99 dof, p ~ 1e-4
    # 32-bit words too
    hist2 = np.bincount((w[:, 2] >> np.uint32(25)).astype(np.int64), minlength=128)
    chi2b = ((hist2 - n / 128) ** 2 / (n / 128)).sum()
    assert chi2b < 200


def test_perm_is_bijection(orc):
    rng = np.random.default_rng(16)
    for n in list(range(1, 130)) + [255, 256, 257, 1000, 1023, 1024, 1025, 4097]:
        for _ in range(3):
            k = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
            if n > 4:
                k[1] = k[3]  # a tie is broken by slot order
            p = orc.perm(n, k)
            assert sorted(p.tolist()) == list(range(n))
            ks = [(int(k[s]), int(s)) for s in p]
            assert ks == sorted(ks)


def test_perm_pairing_uniform(orc):
    # Every unordered pair of a 6-particle cell must be equally likely to be
    # an adjacent pair (p0,p1), (p2,p3) or (p4,p5).
    rng = np.random.default_rng(17)
    n, trials = 6, 20000
    counts = {}
    for _ in range(trials):
        k = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        p = orc.perm(n, k)
        for j in range(0, n, 2):
            key = tuple(sorted((int(p[j]), int(p[j + 1]))))
            counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 15
    exp = trials * 3 / 15
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 40  # 14 dof
    # first element position uniform too
    firsts = np.zeros(n)
    for _ in range(6000):
        k = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        firsts[orc.perm(n, k)[0]] += 1
    chi2f = ((firsts - 1000) ** 2 / 1000).sum()
    assert chi2f < 25
