"""collide_ionize_step_static, the step for callers that cannot allocate:
through the C ABI, its results must be bit-identical to collide_ionize_step's
on the same batches, over two calls in a row whose second input is smaller
(the static scratch keeps the first call's contents), with cells on the LDS
path and on the global-memory path; a batch whose workspace exceeds the
static scratch is refused before any device work."""

import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_1704_01202_amd import binding as B
from paper_1704_01202_amd import runtime as RT
from paper_1704_01202_amd import workloads as W
from tests import cases
from tests.test_gpu_parity import ctx, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = ("e_start", "i_start", "ew", "iz", "ik", "evx", "evy", "evz", "ivx", "ivy", "ivz",
          "ex", "ey")


def _params(bat, step, flags):
    return B.XpStepParams(int(flags), int(step), None, 0, 0, 0, 0)


def _pair(ctx, spec, parts, steps, flags, capacity=(7, 16)):
    """The same batch stepped by both entry points; returns (static, plain)."""
    a = RT.Batch(ctx, [(spec, parts)], capacity=capacity, cell_records=True)
    b = RT.Batch(ctx, [(spec, parts)], capacity=capacity, cell_records=True)
    for s in range(steps):
        B.collide_ionize_step_static(ctx.h, a.struct(), _params(a, s, flags), RT._stream())
        B.collide_ionize_step(ctx.h, b.struct(), _params(b, s, flags), RT._stream())
    torch.cuda.synchronize()
    return a, b


def _same(a, b, label):
    assert a.status() == b.status() == 0, label
    sa, sb = a.state(), b.state()
    for f in FIELDS:
        x, y = getattr(sa, f), getattr(sb, f)
        if x.dtype == np.float64:
            x, y = x.view(np.uint64), y.view(np.uint64)
        assert np.array_equal(x, y), (label, f)
    ca, la, ma = a.cell_records_of()
    cb, lb, mb = b.cell_records_of()
    assert np.array_equal(ca, cb), label
    assert np.array_equal(ma.view(np.uint64), mb.view(np.uint64)), label
    # the energy tallies of the global-memory path add chunk partials with
    # atomics, so their last bits follow the chunks' completion order
    assert np.allclose(la, lb, rtol=1e-12, atol=0.0), label
    assert np.array_equal(a.run_counters(), b.run_counters()), label
    assert np.array_equal(a.stats(), b.stats()), label


def test_static_step_matches_plain_step_twice(ctx):
    # first call: a 2D target with oversized cells on the global-memory path
    # (scratch for the LDS lists and the path's records, keys and chunks)
    ne = np.array([60, 3000, 2600, 9000, 45, 0, 64, 70])
    ni = np.array([50, 1500, 600, 500, 40, 20, 64, 60])
    spec, parts = cases.one_run(ne.size, ne, ni, 30.0, 0.1, seed=93, e_weight=1, dt=0.05e-15,
                                photon_hv=(1850.0,), photon_n=(4e29,))
    a, b = _pair(ctx, spec, parts, 4, O.ALL)
    assert a.stats()[2] == 3
    _same(a, b, "oversized cells")
    say("static step: oversized cells identical to the plain step")
    # second call, smaller input: a few small LDS cells; whatever the first
    # call left in the scratch must not leak into it
    spec, parts = W.config_c2(nx=4, ny=3)
    a, b = _pair(ctx, spec, parts, 3, O.ALL)
    assert a.stats()[2] == 0
    _same(a, b, "small 2D target")
    say("static step: small target identical to the plain step")


def test_static_step_refuses_oversized_workspace(ctx):
    bat = B.XpBatch()
    bat.n_runs, bat.n_cells = 1, 600000
    need = B.xp_step_work_bytes(bat)
    assert need > B.XP_STATIC_SCRATCH_BYTES
    prm = B.XpStepParams(B.XP_ALL, 0, None, 0, 0, 0, 0)
    with pytest.raises(B.XpError) as ei:
        B.collide_ionize_step_static(ctx.h, bat, prm, RT._stream())
    assert "status -5" in str(ei.value)
    # one that fits is accepted (the 64 MiB also holds a 512 x 512 target's lists)
    bat.n_cells = 262144
    assert B.xp_step_work_bytes(bat) <= B.XP_STATIC_SCRATCH_BYTES
