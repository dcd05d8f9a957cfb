"""The oracle against a naive pure-Python third implementation (tests/brute.py)
on cells of 2-6 particles, all stages on, for several steps: pairings, events,
charge states and new-particle order must agree exactly; velocities to a
relative 1e-9 (the two use different elementary-function libraries)."""

import numpy as np
import pytest

from tests import brute, cases


def _cells_from_state(st):
    cells = []
    for c in range(st.e_start.size - 1):
        es = [[st.ex[j], st.ey[j], st.evx[j], st.evy[j], st.evz[j], int(st.ew[j])]
              for j in range(st.e_start[c], st.e_start[c + 1])]
        is_ = [[st.ix[j], st.iy[j], st.ivx[j], st.ivy[j], st.ivz[j], int(st.iz[j]), int(st.ik[j])]
               for j in range(st.i_start[c], st.i_start[c + 1])]
        cells.append(brute.Cell(es, is_))
    return cells


@pytest.mark.parametrize("ipd,seed,nanbu,rel", [(0, 41, False, False), (1, 42, False, False),
                                                (1, 43, False, False), (1, 44, True, False),
                                                (0, 45, False, True), (1, 46, True, True)])
def test_oracle_matches_brute_force(orc, tables, ipd, seed, nanbu, rel):
    rng = np.random.default_rng(seed)
    ncell = 10
    ne = rng.integers(1, 7, ncell)
    ni = rng.integers(1, 5, ncell)
    spec, parts = cases.one_run(ncell, ne, ni, 300.0, 2.0, seed=seed, ipd=ipd, lnl=4.0,
                                dt=0.1e-15, photon_hv=(1650.0, 1900.0), photon_n=(8e30, 5e30))
    parts.iz[:] = rng.integers(3, 10, parts.ni)
    parts.ik[:] = rng.integers(0, 2, parts.ni)
    parts.ew[:] = rng.choice([1, 3], parts.ne)
    sim = orc.Sim(tables, spec)
    sim.bin(parts)
    cells = _cells_from_state(sim.state())
    bf = brute.Brute(tables, spec)
    totals = {"pairs": 0, "ion": 0, "rec": 0, "photo": 0, "decay": 0, "auger": 0}
    for step in range(5):
        flags = orc.ALL | (orc.NANBU if nanbu else 0) | (orc.REL if rel else 0)
        for c, cell in enumerate(cells):
            cnt = bf.step(c, cell, step, flags)
            for k in totals:
                totals[k] += cnt[k]
        sim.step(step, flags)
        st = sim.state()
        for c, cell in enumerate(cells):
            e0, e1 = st.e_start[c], st.e_start[c + 1]
            i0, i1 = st.i_start[c], st.i_start[c + 1]
            assert e1 - e0 == len(cell.e), (step, c)
            assert [int(z) for z in st.iz[i0:i1]] == [i[5] for i in cell.i], (step, c)
            assert [int(k) for k in st.ik[i0:i1]] == [i[6] for i in cell.i], (step, c)
            assert [int(w) for w in st.ew[e0:e1]] == [e[5] for e in cell.e], (step, c)
            ve = np.array([[e[2], e[3], e[4]] for e in cell.e]).reshape(-1, 3)
            vo = np.stack([st.evx[e0:e1], st.evy[e0:e1], st.evz[e0:e1]], axis=1)
            scale = max(np.abs(ve).max(), 1.0)
            assert np.abs(ve - vo).max() <= 1e-9 * scale, (step, c)
            vi = np.array([[i[2], i[3], i[4]] for i in cell.i]).reshape(-1, 3)
            vio = np.stack([st.ivx[i0:i1], st.ivy[i0:i1], st.ivz[i0:i1]], axis=1)
            assert np.abs(vi - vio).max() <= 1e-9 * max(np.abs(vi).max(), 1.0), (step, c)
            xe = np.array([e[0] for e in cell.e])
            assert np.array_equal(xe, st.ex[e0:e1])
    # the run exercised every stage
    assert totals["pairs"] > 50
    assert totals["ion"] > 0 and totals["photo"] > 0 and totals["rec"] > 0
    assert totals["decay"] > 0
