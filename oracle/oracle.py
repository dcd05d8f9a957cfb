"""ctypes front end of the CPU oracle (oracle/liborc.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.
"""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

NSUB = 5
ZMAX = 13
MAX_BINS = 16
MAX_NH = 128
MAX_EOS = 16 * 128
NMOM = 32

EE, EI, ION, REC, PHOTO, DECAY = 0x01, 0x02, 0x04, 0x08, 0x10, 0x20
ALL = EE | EI | ION | REC | PHOTO | DECAY
THERM = 0x40   # variant: forced thermalization after S5 (Sec. VI.C), not in ALL
ION_Z = 0x80   # variant: S3 cross section per ion charge state (Sec. IV), not in ALL
NANBU = 0x100  # variant: Nanbu's cumulative scattering law in S1, S2, not in ALL
REL = 0x200    # variant: relativistic binary collisions in S1, S2, not in ALL
REC_XS = 0x400  # variant: S4 per ion from the Lotz rate by detailed balance, not in ALL
PHOTO_FRAC = 0x800  # variant: S5 photo events limited by the bin's photons in the cell
KA_FIELD = 0x1000   # variant: K-alpha photons return to the photon field

COUNTERS = ["EE", "EI", "TRIPLET", "ACCEPT", "U0", "DELTA2_GT1",
            "ION_FIRED", "ION_ACCEPTED", "ION_STARVED",
            "REC", "REC_SKIPPED", "E_REMOVED",
            "PHOTO_1S", "PHOTO_2S", "PHOTO_2P", "PHOTO_SKIPPED",
            "DECAY", "AUGER", "KALPHA", "P_CLAMPED", "IPD_CLAMPED", "E_NEW",
            "THERM", "THERM_SKIPPED", "PHOTO_STARVED", "PHOTO_PARTIAL", "KA_FIELD"]
NCOUNT = 27
LEDGER = ["PHOTO_E", "AUGER_E", "ION_DEBIT", "REC_ADD", "REC_BIND", "KALPHA",
          "PHOTON_ABS"]
NLEDGER = 8


class OrcTables(C.Structure):
    _fields_ = [
        ("bind", C.c_double * NSUB * (ZMAX + 1)),
        ("lotz_a", C.c_double * NSUB),
        ("lotz_b", C.c_double * NSUB),
        ("lotz_c", C.c_double * NSUB),
        ("gamma_a", C.c_double * 3 * (ZMAX + 1)),
        ("gamma_x", C.c_double * 3 * (ZMAX + 1)),
        ("e_kalpha", C.c_double * (ZMAX + 1)),
        ("mass_ion", C.c_double),
        ("photo_lnhv0", C.c_double),
        ("photo_dlnhv", C.c_double),
        ("photo_lnsig", C.c_double * MAX_NH * NSUB),
        ("photo_nh", C.c_int32),
        ("eos_nn", C.c_int32),
        ("eos_nt", C.c_int32),
        ("pad0", C.c_int32),
        ("eos_lnn0", C.c_double),
        ("eos_dlnn", C.c_double),
        ("eos_lnt0", C.c_double),
        ("eos_dlnt", C.c_double),
        ("eos_zbar", C.c_double * MAX_EOS),
    ]


class OrcRun(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
        ("volume", C.c_double), ("w0", C.c_double),
        ("dt", C.c_double), ("dt_rad", C.c_double),
        ("lnl_fixed", C.c_double), ("e_bulk", C.c_double),
        ("ipd_model", C.c_int32), ("z_floor", C.c_int32),
        ("n_bins", C.c_int32), ("pad1", C.c_int32),
        ("hv", C.c_double * MAX_BINS), ("nhv", C.c_double * MAX_BINS),
    ]


def build():
    """Compile oracle/liborc.so (gcc)."""
    subprocess.run(["sh", os.path.join(HERE, "build.sh")], check=True)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        d, u32, u64, i32, i64, vp = (C.c_double, C.c_uint32, C.c_uint64, C.c_int32,
                                    C.c_int64, C.c_void_p)
        L.orc_log.restype = d; L.orc_log.argtypes = [d]
        L.orc_exp.restype = d; L.orc_exp.argtypes = [d]
        L.orc_cbrt.restype = d; L.orc_cbrt.argtypes = [d]
        L.orc_sincos2pi.restype = None; L.orc_sincos2pi.argtypes = [u64, vp, vp]
        L.orc_philox_many.restype = None; L.orc_philox_many.argtypes = [i64, vp, vp, vp]
        L.orc_u52.restype = d; L.orc_u52.argtypes = [u32, u32]
        L.orc_perm.restype = None; L.orc_perm.argtypes = [i32, vp, vp]
        L.orc_occupancy.restype = None; L.orc_occupancy.argtypes = [i32, i32, vp]
        L.orc_ipd.restype = d; L.orc_ipd.argtypes = [i32, i32, d, d, d, d, d]
        L.orc_lotz.restype = d; L.orc_lotz.argtypes = [vp, i32, vp, d]
        L.orc_eos.restype = d; L.orc_eos.argtypes = [vp, d, d]
        L.orc_photo_sigma.restype = d; L.orc_photo_sigma.argtypes = [vp, i32, d]
        L.orc_coulomb_log.restype = d; L.orc_coulomb_log.argtypes = [d, d, d]
        L.orc_ta77.restype = d
        L.orc_ta77.argtypes = [vp, vp, d, d, u32, u32, d, d, vp, vp, vp]
        L.orc_collide.restype = d
        L.orc_collide.argtypes = [vp, vp, d, d, u32, u32, d, d, vp, i32, vp, vp]
        L.orc_nanbu_a.restype = d; L.orc_nanbu_a.argtypes = [d]
        L.orc_e1x.restype = d; L.orc_e1x.argtypes = [d]
        L.orc_rec_xs.restype = d; L.orc_rec_xs.argtypes = [vp, i32, d, d, vp, d]
        L.orc_nanbu_omc.restype = d; L.orc_nanbu_omc.argtypes = [d, d]
        L.orc_u32.restype = d; L.orc_u32.argtypes = [u32]
        L.orc_create.restype = vp; L.orc_create.argtypes = [vp, vp]
        L.orc_destroy.restype = None; L.orc_destroy.argtypes = [vp]
        L.orc_bin.restype = i32
        L.orc_bin.argtypes = [vp, i64] + [vp] * 6 + [i64] + [vp] * 7
        L.orc_load.restype = i32
        L.orc_load.argtypes = [vp] + [vp] * 7 + [vp] * 8
        L.orc_set_cell_field.restype = None; L.orc_set_cell_field.argtypes = [vp, vp]
        L.orc_step.restype = None; L.orc_step.argtypes = [vp, u32, u32, i32]
        L.orc_counts.restype = None; L.orc_counts.argtypes = [vp, vp, vp]
        L.orc_export.restype = None; L.orc_export.argtypes = [vp] + [vp] * 15
        L.orc_last_counters.restype = None; L.orc_last_counters.argtypes = [vp, vp, vp]
        L.orc_last_moments.restype = None; L.orc_last_moments.argtypes = [vp, vp]
        L.orc_diag.restype = None; L.orc_diag.argtypes = [vp, vp, vp, vp]
        L.orc_last_absorbed.restype = None; L.orc_last_absorbed.argtypes = [vp, vp]
        L.orc_last_kalpha_field.restype = None; L.orc_last_kalpha_field.argtypes = [vp, vp]
        L.orc_get_cell_field.restype = None; L.orc_get_cell_field.argtypes = [vp, vp]
        L.orc_transport.restype = None; L.orc_transport.argtypes = [vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_tables(t) -> OrcTables:
    """Fill the oracle's table struct from workloads.AtomicTables."""
    o = OrcTables()
    for z in range(ZMAX + 1):
        for s in range(NSUB):
            o.bind[z][s] = float(t.bind[z, s])
        for k in range(3):
            o.gamma_a[z][k] = float(t.gamma_a[z, k])
            o.gamma_x[z][k] = float(t.gamma_x[z, k])
        o.e_kalpha[z] = float(t.e_kalpha[z])
    for s in range(NSUB):
        o.lotz_a[s] = float(t.lotz_a[s])
        o.lotz_b[s] = float(t.lotz_b[s])
        o.lotz_c[s] = float(t.lotz_c[s])
    o.mass_ion = float(t.mass_ion)
    nh = t.photo_lnsig.shape[1]
    assert nh <= MAX_NH
    o.photo_nh = nh
    o.photo_lnhv0 = float(t.photo_lnhv0)
    o.photo_dlnhv = float(t.photo_dlnhv)
    for s in range(NSUB):
        for h in range(nh):
            o.photo_lnsig[s][h] = float(t.photo_lnsig[s, h])
    nn, nt = t.eos_zbar.shape
    assert nn * nt <= MAX_EOS
    o.eos_nn, o.eos_nt = nn, nt
    o.eos_lnn0, o.eos_dlnn = float(t.eos_lnn0), float(t.eos_dlnn)
    o.eos_lnt0, o.eos_dlnt = float(t.eos_lnt0), float(t.eos_dlnt)
    flat = np.ascontiguousarray(t.eos_zbar, dtype=np.float64).ravel()
    for q in range(flat.size):
        o.eos_zbar[q] = float(flat[q])
    return o


def make_run(spec) -> OrcRun:
    r = OrcRun()
    r.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
    r.nx, r.ny = spec.nx, spec.ny
    r.dx, r.dy, r.x0, r.y0 = spec.dx, spec.dy, spec.x0, spec.y0
    r.volume, r.w0 = spec.volume, spec.w0
    r.dt, r.dt_rad = spec.dt, spec.dt_rad
    r.lnl_fixed = spec.lnl_fixed
    r.e_bulk = spec.e_bulk if math.isfinite(spec.e_bulk) else 1.0e300
    r.ipd_model, r.z_floor = spec.ipd_model, spec.z_floor
    nb = len(spec.photon_hv)
    assert nb <= MAX_BINS
    r.n_bins = nb
    for b in range(nb):
        r.hv[b] = float(spec.photon_hv[b])
        r.nhv[b] = float(spec.photon_n[b])
    return r


# --- scalar functions -------------------------------------------------------

def log(x):
    return lib().orc_log(float(x))


def exp(x):
    return lib().orc_exp(float(x))


def cbrt(x):
    return lib().orc_cbrt(float(x))


def sincos2pi(k52):
    s, c = C.c_double(), C.c_double()
    lib().orc_sincos2pi(int(k52), C.byref(s), C.byref(c))
    return s.value, c.value


def philox(ctr, key):
    """ctr: [n, 4] uint32, key: [n, 2] uint32 -> [n, 4] uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().orc_philox_many(ctr.shape[0], _p(ctr), _p(key), _p(out))
    return out


def u52(hi, lo):
    return lib().orc_u52(int(hi), int(lo))


def perm(n, keys):
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    out = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_perm(int(n), _p(k), _p(out))
    return out[:n]


def occupancy(z, k=0):
    o = np.zeros(NSUB, dtype=np.int32)
    lib().orc_occupancy(int(z), int(k), _p(o))
    return o


def ipd(model, z, t_ev, n_e, n_i, zbar, zstar):
    return lib().orc_ipd(int(model), int(z), float(t_ev), float(n_e), float(n_i),
                         float(zbar), float(zstar))


def coulomb_log(t_ev, n_e, zbar):
    return lib().orc_coulomb_log(float(t_ev), float(n_e), float(zbar))


class Tables:
    """Holds an OrcTables struct for the table-driven scalar functions."""

    def __init__(self, atomic):
        self.s = make_tables(atomic)

    def lotz(self, zc, dE, e_ev):
        d = np.ascontiguousarray(dE, dtype=np.float64)
        return lib().orc_lotz(C.byref(self.s), int(zc), _p(d), float(e_ev))

    def eos(self, n_i, t_ev):
        return lib().orc_eos(C.byref(self.s), float(n_i), float(t_ev))

    def photo_sigma(self, s, hv):
        return lib().orc_photo_sigma(C.byref(self.s), int(s), float(hv))

    def rec_xs(self, z, t_ev, n_e, dE, dt):
        d = np.ascontiguousarray(dE, dtype=np.float64)
        return lib().orc_rec_xs(C.byref(self.s), int(z), float(t_ev), float(n_e), _p(d), float(dt))


def u32(x):
    return lib().orc_u32(int(x))


def ta77(va, vb, ma, mb, wa, wb, coef, nunit, draws):
    va = np.array(va, dtype=np.float64)
    vb = np.array(vb, dtype=np.float64)
    d = np.ascontiguousarray(draws, dtype=np.uint32)
    aa, ab = C.c_int32(), C.c_int32()
    d2 = lib().orc_ta77(_p(va), _p(vb), float(ma), float(mb), int(wa), int(wb),
                        float(coef), float(nunit), _p(d), C.byref(aa), C.byref(ab))
    return va, vb, d2, aa.value, ab.value


def collide(va, vb, ma, mb, wa, wb, coef, nunit, draws, law):
    """One collision: law bit 0 Nanbu (else Takizuka-Abe), bit 1 relativistic."""
    va = np.array(va, dtype=np.float64)
    vb = np.array(vb, dtype=np.float64)
    d = np.ascontiguousarray(draws, dtype=np.uint32)
    aa, ab = C.c_int32(), C.c_int32()
    d2 = lib().orc_collide(_p(va), _p(vb), float(ma), float(mb), int(wa), int(wb),
                           float(coef), float(nunit), _p(d), int(law), C.byref(aa), C.byref(ab))
    return va, vb, d2, aa.value, ab.value


def e1x(x):
    """exp(x) E1(x)."""
    return lib().orc_e1x(float(x))


def nanbu_a(s):
    return lib().orc_nanbu_a(float(s))


def nanbu_omc(s, u):
    return lib().orc_nanbu_omc(float(s), float(u))


# --- whole-run simulation -----------------------------------------------------

class State:
    """Particle state in the compact cell-major layout (starts[ncells + 1])."""

    def __init__(self, e_start, ex, ey, evx, evy, evz, ew, i_start, ix, iy, ivx, ivy,
                 ivz, iz, ik):
        self.e_start, self.ex, self.ey = e_start, ex, ey
        self.evx, self.evy, self.evz, self.ew = evx, evy, evz, ew
        self.i_start, self.ix, self.iy = i_start, ix, iy
        self.ivx, self.ivy, self.ivz, self.iz, self.ik = ivx, ivy, ivz, iz, ik

    @property
    def ne_cell(self):
        return np.diff(self.e_start)

    @property
    def ni_cell(self):
        return np.diff(self.i_start)


class Sim:
    def __init__(self, atomic, spec):
        self.tables = make_tables(atomic)
        self.run = make_run(spec)
        self.spec = spec
        self.ncells = spec.nx * spec.ny
        self.n_bins = len(spec.photon_hv)
        self.h = lib().orc_create(C.byref(self.tables), C.byref(self.run))

    def __del__(self):
        try:
            if self.h:
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def bin(self, p):
        a = [np.ascontiguousarray(x) for x in (p.ex, p.ey, p.evx, p.evy, p.evz)]
        ew = np.ascontiguousarray(p.ew, dtype=np.uint32)
        b = [np.ascontiguousarray(x) for x in (p.ix, p.iy, p.ivx, p.ivy, p.ivz)]
        iz = np.ascontiguousarray(p.iz, dtype=np.uint8)
        ik = np.ascontiguousarray(p.ik, dtype=np.uint8)
        lib().orc_bin(self.h, a[0].size, *[_p(x) for x in a], _p(ew), b[0].size,
                      *[_p(x) for x in b], _p(iz), _p(ik))

    def load(self, st: State):
        lib().orc_load(self.h, _p(st.e_start), _p(st.ex), _p(st.ey), _p(st.evx),
                       _p(st.evy), _p(st.evz), _p(st.ew), _p(st.i_start), _p(st.ix),
                       _p(st.iy), _p(st.ivx), _p(st.ivy), _p(st.ivz), _p(st.iz),
                       _p(st.ik))

    def set_cell_field(self, nhv_cells):
        if nhv_cells is None:
            lib().orc_set_cell_field(self.h, None)
        else:
            a = np.ascontiguousarray(nhv_cells, dtype=np.float64)
            lib().orc_set_cell_field(self.h, _p(a))

    def step(self, step, flags=ALL, nthreads=0):
        lib().orc_step(self.h, int(step), int(flags), int(nthreads))

    def state(self) -> State:
        ne, ni = C.c_int64(), C.c_int64()
        lib().orc_counts(self.h, C.byref(ne), C.byref(ni))
        ne, ni = ne.value, ni.value
        es = np.zeros(self.ncells + 1, dtype=np.int64)
        is_ = np.zeros(self.ncells + 1, dtype=np.int64)
        f = lambda n: np.zeros(max(n, 1), dtype=np.float64)
        ex, ey, evx, evy, evz = f(ne), f(ne), f(ne), f(ne), f(ne)
        ew = np.zeros(max(ne, 1), dtype=np.uint32)
        ix, iy, ivx, ivy, ivz = f(ni), f(ni), f(ni), f(ni), f(ni)
        iz = np.zeros(max(ni, 1), dtype=np.uint8)
        ik = np.zeros(max(ni, 1), dtype=np.uint8)
        lib().orc_export(self.h, _p(es), _p(ex), _p(ey), _p(evx), _p(evy), _p(evz),
                         _p(ew), _p(is_), _p(ix), _p(iy), _p(ivx), _p(ivy), _p(ivz),
                         _p(iz), _p(ik))
        return State(es, ex[:ne], ey[:ne], evx[:ne], evy[:ne], evz[:ne], ew[:ne], is_,
                     ix[:ni], iy[:ni], ivx[:ni], ivy[:ni], ivz[:ni], iz[:ni], ik[:ni])

    def counters(self):
        cnt = np.zeros((self.ncells, NCOUNT), dtype=np.int64)
        led = np.zeros((self.ncells, NLEDGER), dtype=np.float64)
        lib().orc_last_counters(self.h, _p(cnt), _p(led))
        return cnt, led

    def moments(self):
        m = np.zeros((self.ncells, NMOM), dtype=np.float64)
        lib().orc_last_moments(self.h, _p(m))
        return m

    def absorbed(self):
        """Photon events per bin of the last step, [ncells][MAX_BINS]."""
        a = np.zeros((self.ncells, MAX_BINS), dtype=np.int32)
        lib().orc_last_absorbed(self.h, _p(a))
        return a

    def kalpha_field(self):
        """K-alpha macro-photons returned per bin in the last step (KA_FIELD),
        [ncells][MAX_BINS]."""
        g = np.zeros((self.ncells, MAX_BINS), dtype=np.float64)
        lib().orc_last_kalpha_field(self.h, _p(g))
        return g

    def cell_field(self):
        """The photon field per cell, [ncells][n_bins]."""
        f = np.zeros((self.ncells, self.n_bins), dtype=np.float64)
        lib().orc_get_cell_field(self.h, _p(f))
        return f

    def transport(self):
        """Reduced radiation transport after a step; returns the mean row
        transmission per bin."""
        t = np.zeros(MAX_BINS, dtype=np.float64)
        lib().orc_transport(self.h, _p(t))
        return t[:self.n_bins]

    def diag(self):
        csd = np.zeros(ZMAX + 1, dtype=np.int64)
        fe = np.zeros(64, dtype=np.int64)
        out = np.zeros(8, dtype=np.float64)
        lib().orc_diag(self.h, _p(csd), _p(fe), _p(out))
        return csd, fe, out
