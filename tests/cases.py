"""Small hand-built workloads for the oracle and parity tests."""

import dataclasses
import math

import numpy as np

from paper_1704_01202_amd import workloads as W

QE = 1.602176634e-19
ME = 9.1093837015e-31


def maxwell(rng, n, t_ev, mass):
    return rng.normal(0.0, math.sqrt(t_ev * QE / mass), size=(3, n))


def one_run(nx, ne_cell, ni_cell, e_t_ev, i_t_ev, *, seed=5, z0=3, k0=0, e_weight=3,
            n_i=W.SOLID_NI, dt=0.1e-15, dt_rad=None, ipd=W.IPD_EK, lnl=0.0, ny=1,
            photon_hv=(), photon_n=(), mass_ion=W.M_AL, shuffle=True, z_floor=3):
    """A run of nx*ny cells with the given counts per cell and Maxwellian species."""
    vol = W.DX_PIC ** 3
    ni_arr = np.broadcast_to(np.asarray(ni_cell), (nx * ny,))
    nref = max(1, int(ni_arr.max()))
    spec = W.RunSpec(seed=seed, nx=nx, ny=ny, dx=W.DX_PIC, dy=W.DX_PIC, volume=vol,
                     w0=n_i * vol / nref, dt=dt, dt_rad=dt if dt_rad is None else dt_rad,
                     ipd_model=ipd, lnl_fixed=lnl, photon_hv=tuple(photon_hv),
                     photon_n=tuple(photon_n), z_floor=z_floor)
    rng = np.random.default_rng(seed)

    def evel(rng, cid, slot):
        return maxwell(rng, cid.size, e_t_ev, ME)

    parts = W.build_particles(spec, np.broadcast_to(np.asarray(ne_cell), (nx * ny,)),
                              ni_arr, evel, i_t_ev, rng, e_weight=e_weight,
                              shuffle=shuffle)
    if mass_ion != W.M_AL:
        parts.ivx[:] = maxwell(rng, parts.ni, i_t_ev, mass_ion)[0]
        parts.ivy[:] = maxwell(rng, parts.ni, i_t_ev, mass_ion)[1]
        parts.ivz[:] = maxwell(rng, parts.ni, i_t_ev, mass_ion)[2]
    parts.iz[:] = z0
    parts.ik[:] = k0
    return spec, parts


def tables_with(tables, **kw):
    return dataclasses.replace(tables, **kw)


def kinetic(state, mass_ion):
    ke = 0.5 * ME * (state.evx ** 2 + state.evy ** 2 + state.evz ** 2) * state.ew
    ki = 0.5 * mass_ion * (state.ivx ** 2 + state.ivy ** 2 + state.ivz ** 2)
    return ke.sum() / QE, ki.sum() / QE


def momentum(state, mass_ion):
    w = state.ew.astype(np.float64)
    pe = ME * np.array([(w * state.evx).sum(), (w * state.evy).sum(), (w * state.evz).sum()])
    pi = mass_ion * np.array([state.ivx.sum(), state.ivy.sum(), state.ivz.sum()])
    return pe + pi, ME * (w * np.abs(state.evx)).sum() + mass_ion * np.abs(state.ivx).sum()
