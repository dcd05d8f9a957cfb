"""The canonical pairwise sum of a cell equals the pairwise sum of the
pairwise sums of its aligned chunks (padded with +0 to a power of two).

The device takes sums over cells larger than one workgroup in aligned chunks
(1024 particles for the step, 8192 for the diagnostics) and relies on this
identity to keep the bits of the one-workgroup sum.  Checked here in exact
IEEE double arithmetic on values with mixed signs and magnitudes, including
signed zeros, against the definition written out level by level.
"""

import numpy as np
import pytest


def tree(y):
    """Pad to the next power of two with +0, then y[i] = y[2i] + y[2i+1] level by level."""
    n = len(y)
    if n == 0:
        return 0.0
    p = 1
    while p < n:
        p *= 2
    a = np.zeros(p)
    a[:n] = y
    while len(a) > 1:
        a = a[0::2] + a[1::2]
    return float(a[0]) + 0.0


def chunked(y, ch):
    parts = []
    for b in range(0, len(y), ch):
        c = np.zeros(ch)
        seg = y[b:b + ch]
        c[:len(seg)] = seg
        parts.append(tree(c))
    return tree(np.array(parts))


@pytest.mark.parametrize("ch", [64, 1024])
def test_chunked_tree_is_the_tree(ch):
    rng = np.random.default_rng(17)
    sizes = [1, 2, 3, ch - 1, ch, ch + 1, 2 * ch - 3, 3 * ch + 5, 5 * ch, 7 * ch + 1]
    for n in sizes:
        for trial in range(4):
            y = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
            y[rng.random(n) < 0.05] = -0.0
            if trial == 3:
                y = np.abs(y) * 1e-300   # subnormal and tiny sums
            assert tree(y) == chunked(y, ch), (n, trial)
    # every leaf a negative zero: both give +0
    assert str(chunked(np.full(3 * ch, -0.0), ch)) == str(tree(np.full(3 * ch, -0.0))) == "0.0"
