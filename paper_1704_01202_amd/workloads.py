"""Seeded synthetic inputs: atomic tables and particle workloads.

This module is the only code shared by the HIP path and the CPU oracle.  It
holds none of the method's arithmetic: it draws initial particle states and
writes the atomic data tables that the paper takes from external atomic-physics
codes (subshell binding energies, photoionization cross sections, K-vacancy
decay rates, Lotz constants and the equation of state).  Those tables are not
available here, so the values below are SYNTHETIC stand-ins with the shapes the
paper describes (Sec. III, Sec. IV, Fig. 2, Fig. 3):

* binding energies per charge state and subshell from screened-hydrogenic
  (Slater) estimates, scaled per shell so that the K edge of solid-density
  Al3+ lowered by Ecker-Kroll sits near the cold edge of about 1560 eV and the
  KLL Auger energy is near 1.4 keV (Sec. VI.A, Sec. VI.B);
* subshell photoionization cross sections per electron, neutral atom,
  Kramers-like (hv^-3), K shell an order of magnitude above L (Sec. III);
* K-vacancy Auger and radiative rates giving a 1 fs lifetime with a full L
  shell and a 4 % fluorescence yield (Sec. III), the lifetime growing as the
  L shell empties;
* Lotz constants a = 4.5e-14 cm^2 eV^2, b = c = 0 (Eq. 4);
* an equation of state Zbar(T) = 3 + 10 T / (T + 150 eV), density
  independent, passing through the state point T = 100 eV, Zbar = 7 of
  Sec. V and the Al3+ floor of Sec. V.

Every array returned here is plain numpy; nothing imports torch or the HIP
library.  Units: SI for positions (m), velocities (m/s), volumes (m^3) and
densities (m^-3); energies in eV; table cross sections in cm^2 (the consumers
convert once).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Subshell order used everywhere: 1s, 2s, 2p, 3s, 3p.
NSUB = 5
SUB_CAP = (2, 2, 6, 2, 6)
SUB_N = (1, 2, 2, 3, 3)
Z_NUC = 13

# CODATA 2018 values used only to draw initial velocities from temperatures.
_QE = 1.602176634e-19
_ME = 9.1093837015e-31
_AMU = 1.66053906660e-27
M_AL = 26.9815385 * _AMU
_C = 299792458.0

SOLID_NI = 6.0e28          # m^-3, 6.0e22 cm^-3
DX_PIC = 1.0e-6 / 150.0    # PIC cell, 150 cells per micron (Sec. VI)

IPD_SP = 0
IPD_EK = 1


def ground_occupancy(zion: int, kvac: int = 0):
    """Lowest-energy configuration with kvac K vacancies (Sec. III)."""
    nb = Z_NUC - zion
    occ = [0] * NSUB
    occ[0] = max(0, min(2 - kvac, nb))
    rem = nb - occ[0]
    for s in range(1, NSUB):
        occ[s] = min(SUB_CAP[s], rem)
        rem -= occ[s]
    return occ


def _slater_binding(zion: int, s: int) -> float:
    """Screened hydrogenic binding, Rydberg units -> eV.

    Slater (1930) screening by same and inner shells, plus a small screening by
    outer-shell electrons (0.22 per L electron on K, 0.10 per M electron on K,
    0.20 per M electron on L) so that inner edges move up as outer shells are
    stripped, as the paper describes for the K edge (Sec. III, Sec. VI.A).
    """
    occ = ground_occupancy(zion, 0)
    n = SUB_N[s]
    nk, nl, nm = occ[0], occ[1] + occ[2], occ[3] + occ[4]
    if n == 1:
        screen = 0.30 * max(nk - 1, 0) + 0.22 * nl + 0.10 * nm
    elif n == 2:
        screen = 0.35 * max(nl - 1, 0) + 0.85 * nk + 0.20 * nm
    else:
        screen = 0.35 * max(nm - 1, 0) + 0.85 * nl + 1.0 * nk
    zeff = max(Z_NUC - screen, 1.0)
    return 13.605693 * zeff * zeff / (n * n)


# Per-shell scale factors that place the synthetic edges: the K binding of Al3+
# is 1617.7 eV (1560 eV after the 57.7 eV Ecker-Kroll lowering of solid Al3+)
# and its L binding 137.7 eV (KLL Auger energy near 1.4 keV).
_SHELL_SCALE = {1: 1617.7 / _slater_binding(3, 0),
                2: 137.7 / _slater_binding(3, 2),
                3: 0.40}


@dataclass
class AtomicTables:
    """Synthetic Al tables in the layout the library's init_species expects."""
    z_nuc: int = Z_NUC
    mass_ion: float = M_AL
    bind: np.ndarray = None          # [14, 5] eV, subshell binding of charge state Z
    lotz_a: np.ndarray = None        # [5] cm^2 eV^2
    lotz_b: np.ndarray = None        # [5]
    lotz_c: np.ndarray = None        # [5]
    gamma_a: np.ndarray = None       # [14, 3] s^-1, KLL Auger rate for (Z, k)
    gamma_x: np.ndarray = None       # [14, 3] s^-1, K-alpha radiative rate for (Z, k)
    e_kalpha: np.ndarray = None      # [14] eV
    photo_lnhv0: float = 0.0         # ln(eV) of the first grid point
    photo_dlnhv: float = 0.0         # uniform ln spacing
    photo_lnsig: np.ndarray = None   # [5, nh] ln(cm^2) per electron
    eos_lnn0: float = 0.0            # ln(m^-3)
    eos_dlnn: float = 0.0
    eos_lnt0: float = 0.0            # ln(eV)
    eos_dlnt: float = 0.0
    eos_zbar: np.ndarray = None      # [nn, nt]
    synthetic: bool = True
    notes: dict = field(default_factory=dict)


def make_tables() -> AtomicTables:
    t = AtomicTables()
    bind = np.zeros((Z_NUC + 1, NSUB))
    for z in range(Z_NUC + 1):
        for s in range(NSUB):
            bind[z, s] = _SHELL_SCALE[SUB_N[s]] * _slater_binding(z, s)
    t.bind = bind
    t.lotz_a = np.full(NSUB, 4.5e-14)
    t.lotz_b = np.zeros(NSUB)
    t.lotz_c = np.zeros(NSUB)

    ga = np.zeros((Z_NUC + 1, 3))
    gx = np.zeros((Z_NUC + 1, 3))
    for z in range(Z_NUC + 1):
        for k in (1, 2):
            occ = ground_occupancy(z, k)
            nl = occ[1] + occ[2]
            ga[z, k] = k * 0.96e15 * (nl * (nl - 1) / 2.0) / 28.0
            gx[z, k] = k * 0.04e15 * occ[2] / 6.0
    # Lifetime of states with 10 or more bound electrons: linear in N_b between
    # N_b = 10 and the neutral atom (Sec. III).  With the synthetic rates the
    # neutral value equals the N_b = 10 value, so the rule is a constant.
    for k in (1, 2):
        r10 = ga[3, k] + gx[3, k]
        for z in range(0, 3):
            w = ga[3, k] / r10 if r10 > 0 else 0.0
            ga[z, k] = r10 * w
            gx[z, k] = r10 * (1.0 - w)
    t.gamma_a = ga
    t.gamma_x = gx
    t.e_kalpha = bind[:, 0] - bind[:, 2]

    nh = 96
    lo, hi = math.log(5.0), math.log(3.0e4)
    t.photo_lnhv0 = lo
    t.photo_dlnhv = (hi - lo) / (nh - 1)
    lnhv = lo + t.photo_dlnhv * np.arange(nh)
    ref = math.log(1600.0)
    sig_ref = np.array([4.0e-20, 3.0e-21, 3.0e-21, 3.0e-22, 3.0e-22])
    t.photo_lnsig = np.log(sig_ref)[:, None] - 3.0 * (lnhv[None, :] - ref)

    nn, nt = 9, 81
    t.eos_lnn0 = math.log(1.0e26)
    t.eos_dlnn = (math.log(1.0e30) - t.eos_lnn0) / (nn - 1)
    t.eos_lnt0 = math.log(0.01)
    t.eos_dlnt = (math.log(1.0e4) - t.eos_lnt0) / (nt - 1)
    tgrid = np.exp(t.eos_lnt0 + t.eos_dlnt * np.arange(nt))
    zt = 3.0 + 10.0 * tgrid / (tgrid + 150.0)
    t.eos_zbar = np.repeat(zt[None, :], nn, axis=0)
    t.notes = {"label": "SYNTHETIC Al tables; not the paper's atomic data"}
    return t


# --------------------------------------------------------------------------
# Particle workloads
# --------------------------------------------------------------------------

@dataclass
class RunSpec:
    """Per-run physical parameters (one independent simulation)."""
    seed: int
    nx: int
    ny: int
    dx: float
    dy: float
    x0: float = 0.0
    y0: float = 0.0
    volume: float = 0.0       # cell volume, m^3
    w0: float = 1.0           # real particles per weight unit
    dt: float = 0.1e-15
    dt_rad: float = 0.1e-15
    ipd_model: int = IPD_SP
    lnl_fixed: float = 0.0    # > 0 selects a fixed Coulomb logarithm
    e_bulk: float = math.inf  # eV
    z_floor: int = 3
    photon_hv: tuple = ()     # eV per bin
    photon_n: tuple = ()      # photons per m^3 per bin (uniform over cells)
    nsteps: int = 1

    @property
    def ncells(self) -> int:
        return self.nx * self.ny


@dataclass
class Particles:
    """Unsorted particle arrays of one run (input to bin_particles)."""
    ex: np.ndarray
    ey: np.ndarray
    evx: np.ndarray
    evy: np.ndarray
    evz: np.ndarray
    ew: np.ndarray      # uint32 weight units
    ix: np.ndarray
    iy: np.ndarray
    ivx: np.ndarray
    ivy: np.ndarray
    ivz: np.ndarray
    iz: np.ndarray      # uint8 charge state
    ik: np.ndarray      # uint8 K vacancies

    @property
    def ne(self):
        return int(self.ex.shape[0])

    @property
    def ni(self):
        return int(self.ix.shape[0])


def _maxwell(rng, n, t_ev, mass):
    sig = math.sqrt(t_ev * _QE / mass)
    return rng.normal(0.0, sig, size=(3, n))


def _isotropic(rng, n, e_ev, mass):
    speed = math.sqrt(2.0 * e_ev * _QE / mass)
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(1.0 - mu * mu)
    return np.stack([speed * st * np.cos(phi), speed * st * np.sin(phi), speed * mu])


def build_particles(spec: RunSpec, ne_cell, ni_cell, e_vel_fn, i_temp_ev,
                    rng, e_weight=3, shuffle=True) -> Particles:
    """Place ne_cell[c] electrons and ni_cell[c] ions in every cell c.

    e_vel_fn(rng, cell_ids, slot_in_cell) returns (3, n) electron velocities.
    Particle order is shuffled so that binning has real work to do.
    """
    ne_cell = np.asarray(ne_cell, dtype=np.int64)
    ni_cell = np.asarray(ni_cell, dtype=np.int64)
    ncell = spec.ncells

    def positions(counts):
        cid = np.repeat(np.arange(ncell, dtype=np.int64), counts)
        cx = cid % spec.nx
        cy = cid // spec.nx
        x = spec.x0 + (cx + rng.uniform(0.02, 0.98, cid.size)) * spec.dx
        if spec.ny > 1:
            y = spec.y0 + (cy + rng.uniform(0.02, 0.98, cid.size)) * spec.dy
        else:
            y = np.zeros(cid.size)
        return cid, x, y

    ecid, ex, ey = positions(ne_cell)
    starts = np.concatenate([[0], np.cumsum(ne_cell)[:-1]])
    eslot = np.arange(ecid.size) - np.repeat(starts, ne_cell)
    ev = e_vel_fn(rng, ecid, eslot)
    icid, ix, iy = positions(ni_cell)
    iv = _maxwell(rng, icid.size, i_temp_ev, M_AL)
    ew = np.full(ecid.size, e_weight, dtype=np.uint32)
    iz = np.full(icid.size, 3, dtype=np.uint8)
    ik = np.zeros(icid.size, dtype=np.uint8)
    if shuffle:
        pe = rng.permutation(ecid.size)
        pi = rng.permutation(icid.size)
    else:
        pe = np.arange(ecid.size)
        pi = np.arange(icid.size)
    return Particles(ex=ex[pe].copy(), ey=ey[pe].copy(), evx=ev[0][pe].copy(),
                     evy=ev[1][pe].copy(), evz=ev[2][pe].copy(), ew=ew[pe].copy(),
                     ix=ix[pi].copy(), iy=iy[pi].copy(), ivx=iv[0][pi].copy(),
                     ivy=iv[1][pi].copy(), ivz=iv[2][pi].copy(), iz=iz[pi].copy(),
                     ik=ik[pi].copy())


def photon_density(intensity_w_cm2: float, hv_ev: float) -> float:
    """Photon number density n = I / (c hv) for a prescribed flux, m^-3."""
    return intensity_w_cm2 * 1.0e4 / (_C * hv_ev * _QE)


def config_c1(seed=1, ncells=64, nsteps=100):
    """Tiny 1D slab: 64 cells x (200 e + 200 Al ions), Stewart-Pyatt, dt 0.1 fs.

    Electrons per cell: slots 0-179 Maxwellian at 10 eV, 180-191 isotropic
    1.5 keV photoelectrons, 192-199 isotropic 1.35 keV Auger electrons.
    """
    vol = DX_PIC ** 3
    spec = RunSpec(seed=seed, nx=ncells, ny=1, dx=DX_PIC, dy=DX_PIC, volume=vol,
                   w0=SOLID_NI * vol / 200.0, dt=0.1e-15, dt_rad=0.1e-15,
                   ipd_model=IPD_SP, nsteps=nsteps)
    rng = np.random.default_rng(seed)

    def evel(rng, cid, slot):
        v = _maxwell(rng, cid.size, 10.0, _ME)
        hot = (slot >= 180) & (slot < 192)
        aug = slot >= 192
        v[:, hot] = _isotropic(rng, int(hot.sum()), 1500.0, _ME)
        v[:, aug] = _isotropic(rng, int(aug.sum()), 1350.0, _ME)
        return v

    parts = build_particles(spec, np.full(ncells, 200), np.full(ncells, 200),
                            evel, 0.1, rng)
    return spec, parts


def config_c2(seed=2, nx=512, ny=512, nsteps=200):
    """2D uniform target: nx x ny cells x (64 e + 64 ions), Ecker-Kroll, dt 0.05 fs,
    photoionization by a uniform 1.7e17 W/cm^2, 1.85 keV photon flux."""
    vol = DX_PIC ** 3
    hv = 1850.0
    spec = RunSpec(seed=seed, nx=nx, ny=ny, dx=DX_PIC, dy=DX_PIC, volume=vol,
                   w0=SOLID_NI * vol / 64.0, dt=0.05e-15, dt_rad=0.05e-15,
                   ipd_model=IPD_EK, photon_hv=(hv,),
                   photon_n=(photon_density(1.7e17, hv),), nsteps=nsteps)
    rng = np.random.default_rng(seed)

    def evel(rng, cid, slot):
        return _maxwell(rng, cid.size, 10.0, _ME)

    parts = build_particles(spec, np.full(nx * ny, 64), np.full(nx * ny, 64),
                            evel, 0.1, rng)
    return spec, parts


def config_c3(seed=3, nx=1024, ny=256, nsteps=100):
    """Uneven occupancy: density ramp 0.01x..1x solid along x (20-cell
    exponential scale length), Poisson particle counts about 512 n/n_s clamped
    to [2, 512] ions per cell with as many electrons, T_e ~ U(5, 50) eV per column."""
    vol = DX_PIC ** 3
    spec = RunSpec(seed=seed, nx=nx, ny=ny, dx=DX_PIC, dy=DX_PIC, volume=vol,
                   w0=SOLID_NI * vol / 512.0, dt=0.05e-15, dt_rad=0.05e-15,
                   ipd_model=IPD_EK, nsteps=nsteps)
    rng = np.random.default_rng(seed)
    col = np.arange(nx)
    rel = np.maximum(0.01, np.exp(-(nx - 1 - col) / 20.0))
    lam = np.tile(512.0 * rel, ny)
    ni = np.clip(rng.poisson(lam), 2, 512)
    tcol = rng.uniform(5.0, 50.0, nx)

    def evel(rng, cid, slot):
        t = tcol[cid % nx]
        sig = np.sqrt(t * _QE / _ME)
        return rng.normal(0.0, 1.0, size=(3, cid.size)) * sig[None, :]

    parts = build_particles(spec, ni, ni, evel, 0.1, rng)
    return spec, parts


def config_c4_runs(seed=4, nruns=256, nsteps=500, size_lo=1e4, size_hi=2e6):
    """Batched scan: independent single-cell (0D) runs, sizes log-uniform,
    intensity log-uniform 1e16..1e18 W/cm^2 (flat top), hv uniform 1.55..1.9 keV,
    IPD alternating SP (even runs) / EK (odd runs), dt 0.1 fs."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(size_lo), math.log(size_hi), nruns))
    inten = np.exp(rng.uniform(math.log(1e16), math.log(1e18), nruns))
    hvs = rng.uniform(1550.0, 1900.0, nruns)
    runs = []
    for r in range(nruns):
        nion = max(2, int(sizes[r]) // 2)
        w0 = 100.0
        vol = nion * w0 / SOLID_NI
        spec = RunSpec(seed=(seed << 32) + r, nx=1, ny=1, dx=vol ** (1 / 3),
                       dy=vol ** (1 / 3), volume=vol, w0=w0, dt=0.1e-15,
                       dt_rad=0.1e-15, ipd_model=IPD_SP if r % 2 == 0 else IPD_EK,
                       photon_hv=(float(hvs[r]),),
                       photon_n=(photon_density(float(inten[r]), float(hvs[r])),),
                       nsteps=nsteps)
        prng = np.random.default_rng([seed, r])

        def evel(rng, cid, slot):
            return _maxwell(rng, cid.size, 10.0, _ME)

        # electrons carry 3 units so that the plasma starts neutral at Al3+
        parts = build_particles(spec, np.array([nion]), np.array([nion]), evel,
                                0.1, prng)
        runs.append((spec, parts))
    return runs


@dataclass
class Request:
    """One served run: arrival time (s from the start of the trace), the run and
    its particles, and the steps it asks for."""
    rid: int
    arrival: float
    spec: RunSpec
    parts: Particles
    nsteps: int


def config_c5_trace(seed=5, n_requests=1000, rate=20.0, size_lo=1e4, size_hi=5e6,
                    cells_lo=64, cells_hi=4096, steps_lo=100, steps_hi=2000):
    """Served stream: Poisson arrivals at `rate` runs/s; half 0D runs (one
    cell), half 1D runs of log-uniform-integer cells; particles log-uniform,
    split evenly e/i (electrons carry 3 units, Al3+); steps uniform-integer;
    intensity, photon energy and IPD model drawn as in the batched scan."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(n_requests):
        t += rng.exponential(1.0 / rate)
        size = math.exp(rng.uniform(math.log(size_lo), math.log(size_hi)))
        one_d = rng.random() < 0.5
        ncell = int(round(math.exp(rng.uniform(math.log(cells_lo), math.log(cells_hi))))) if one_d else 1
        nsteps = int(rng.integers(steps_lo, steps_hi + 1))
        inten = math.exp(rng.uniform(math.log(1e16), math.log(1e18)))
        hv = float(rng.uniform(1550.0, 1900.0))
        nion_total = max(2 * ncell, int(size) // 2)
        per_cell = max(1, nion_total // ncell)
        w0 = 100.0
        vol = per_cell * w0 / SOLID_NI
        dx = vol ** (1.0 / 3.0)
        spec = RunSpec(seed=(seed << 32) + q, nx=ncell, ny=1, dx=dx, dy=dx, volume=vol, w0=w0,
                       dt=0.1e-15, dt_rad=0.1e-15, ipd_model=IPD_SP if q % 2 == 0 else IPD_EK,
                       photon_hv=(hv,), photon_n=(photon_density(inten, hv),), nsteps=nsteps)
        prng = np.random.default_rng([seed, q])

        def evel(rng, cid, slot):
            return _maxwell(rng, cid.size, 10.0, _ME)

        counts = np.full(ncell, per_cell, dtype=np.int64)
        parts = build_particles(spec, counts, counts, evel, 0.1, prng)
        out.append(Request(rid=q, arrival=t, spec=spec, parts=parts, nsteps=nsteps))
    return out
