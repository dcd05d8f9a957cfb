"""ctypes binding of libxpic.so (include/xpic.h).

Argument marshalling only: PyTorch supplies device memory and streams; every
step of the method runs in the library's HIP kernels.  Loading fails loudly when
the library has not been built or no HIP device is present.
"""

from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxpic.so")

XP_EE, XP_EI, XP_ION, XP_REC, XP_PHOTO, XP_DECAY = 0x01, 0x02, 0x04, 0x08, 0x10, 0x20
XP_ALL = 0x3F
XP_THERM = 0x40   # variant: forced thermalization after S5 (Sec. VI.C), not in XP_ALL
XP_ION_Z = 0x80   # variant: S3 cross section per ion charge state (Sec. IV), not in XP_ALL
XP_NANBU = 0x100  # variant: Nanbu's cumulative scattering law in e-e and e-i, not in XP_ALL
XP_REL = 0x200    # variant: relativistic binary collisions in e-e and e-i, not in XP_ALL
XP_REC_XS = 0x400  # variant: recombination from cross sections by detailed balance, not in XP_ALL
XP_PHOTO_FRAC = 0x800  # variant: photo events limited by the bin's photons in the cell, not in XP_ALL
XP_KA_FIELD = 0x1000   # variant: K-alpha photons return to the photon field, not in XP_ALL
XP_ST_CAPACITY, XP_ST_NONFINITE, XP_ST_BIN_SIZE, XP_ST_RUN_TABLE = 0x1, 0x2, 0x4, 0x8
XP_NCOUNT, XP_NLEDGER, XP_NMOM, XP_MAX_BINS = 27, 8, 32, 16
XP_NSTATS = 68
XP_DIAG_RESET = 0x1

COUNTERS = ["EE", "EI", "TRIPLET", "ACCEPT", "U0", "DELTA2_GT1",
            "ION_FIRED", "ION_ACCEPTED", "ION_STARVED",
            "REC", "REC_SKIPPED", "E_REMOVED",
            "PHOTO_1S", "PHOTO_2S", "PHOTO_2P", "PHOTO_SKIPPED",
            "DECAY", "AUGER", "KALPHA", "P_CLAMPED", "IPD_CLAMPED", "E_NEW",
            "THERM", "THERM_SKIPPED"]

_vp = C.c_void_p
_d = C.c_double
_i32 = C.c_int32
_i64 = C.c_int64
_u32 = C.c_uint32
_u64 = C.c_uint64


class XpAtomicTables(C.Structure):
    _fields_ = [("z_nuc", _i32), ("photo_nh", _i32), ("eos_nn", _i32), ("eos_nt", _i32),
                ("mass_ion", _d), ("bind", _vp), ("lotz_a", _vp), ("lotz_b", _vp),
                ("lotz_c", _vp), ("gamma_a", _vp), ("gamma_x", _vp), ("e_kalpha", _vp),
                ("photo_lnhv0", _d), ("photo_dlnhv", _d), ("photo_lnsig", _vp),
                ("eos_lnn0", _d), ("eos_dlnn", _d), ("eos_lnt0", _d), ("eos_dlnt", _d),
                ("eos_zbar", _vp)]


class XpRun(C.Structure):
    _fields_ = [("seed", _u64), ("nx", _i32), ("ny", _i32), ("dx", _d), ("dy", _d),
                ("x0", _d), ("y0", _d), ("volume", _d), ("w0", _d), ("dt", _d),
                ("dt_rad", _d), ("lnl_fixed", _d), ("e_bulk", _d), ("ipd_model", _i32),
                ("z_floor", _i32), ("cell_begin", _i32), ("ncells", _i32), ("n_bins", _i32),
                ("field_per_cell", _i32), ("hv", _d * XP_MAX_BINS), ("nhv", _d * XP_MAX_BINS)]


class XpBatch(C.Structure):
    _fields_ = [("n_runs", _i32), ("n_cells", _i32), ("d_runs", _vp), ("d_cell_run", _vp),
                ("d_e_off", _vp), ("d_e_cap", _vp), ("d_e_cnt", _vp),
                ("d_i_off", _vp), ("d_i_cap", _vp), ("d_i_cnt", _vp),
                ("e_slots", _i64), ("i_slots", _i64),
                ("d_ex", _vp), ("d_ey", _vp), ("d_evx", _vp), ("d_evy", _vp), ("d_evz", _vp),
                ("d_ew", _vp),
                ("d_ix", _vp), ("d_iy", _vp), ("d_ivx", _vp), ("d_ivy", _vp), ("d_ivz", _vp),
                ("d_iz", _vp), ("d_ik", _vp), ("d_cell_nhv", _vp),
                ("d_run_counters", _vp), ("d_run_ledger", _vp), ("d_cell_counters", _vp),
                ("d_cell_ledger", _vp), ("d_cell_moments", _vp), ("d_status", _vp),
                ("d_work", _vp), ("work_bytes", C.c_size_t),
                ("e_cap_max", _i32), ("i_cap_max", _i32), ("d_stats", _vp),
                ("big_cells_max", _i32), ("reserved0", _i32), ("big_e_slots", _i64),
                ("big_i_slots", _i64), ("d_cell_nabs", _vp), ("d_run_status", _vp),
                ("d_cell_nka", _vp)]


class XpParticles(C.Structure):
    _fields_ = [("ne", _i64), ("ni", _i64), ("d_e_run", _vp), ("d_i_run", _vp),
                ("d_ex", _vp), ("d_ey", _vp), ("d_evx", _vp), ("d_evy", _vp), ("d_evz", _vp),
                ("d_ew", _vp), ("d_ix", _vp), ("d_iy", _vp), ("d_ivx", _vp), ("d_ivy", _vp),
                ("d_ivz", _vp), ("d_iz", _vp), ("d_ik", _vp)]


class XpCapacity(C.Structure):
    _fields_ = [("e_per_ion", _i32), ("e_extra", _i32)]


class XpStepParams(C.Structure):
    _fields_ = [("flags", _u32), ("step", _u32), ("d_step", _vp), ("schedule", _i32),
                ("e_hint", _i32), ("big_grid", _i32), ("reserved", _i32)]


class XpDiag(C.Structure):
    _fields_ = [("csd", _i64 * 14), ("fe_hist", _i64 * 64), ("w_e", _i64), ("w_i", _i64),
                ("sum_z", _i64), ("n_e_macro", _i64), ("zbar", _d), ("ke_ev", _d),
                ("te_ev", _d), ("reserved", _d), ("counters", _u64 * XP_NCOUNT),
                ("ledger", _d * XP_NLEDGER)]


XP_STATIC_SCRATCH_BYTES = 64 << 20   # static workspace of collide_ionize_step_static

ABI_VERSION = 4   # struct layouts mirrored below (XP_ABI_VERSION of include/xpic.h)

EXPORTS = ["xp_abi_version", "xp_last_error", "xp_ctx_create", "xp_ctx_destroy",
           "xp_table_bytes", "init_species", "xp_work_bytes", "xp_step_work_bytes",
           "xp_lds_limits", "bin_particles", "collide_ionize_step", "collide_ionize_step_static",
           "photo_auger_step",
           "diagnostics", "transport_photons", "xp_selftest"]

_lib = None


class XpError(RuntimeError):
    pass


def load(path=LIB_PATH):
    """Load libxpic.so (built in-tree by paper_1704_01202_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    # the library must bind to the HIP runtime that torch brings (the device
    # memory and streams it is handed come from there): load torch first
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise XpError("libxpic.so is not built: run __graft_entry__.build() or "
                      "python paper_1704_01202_amd/build.py")
    L = C.CDLL(path)
    L.xp_abi_version.restype = _u32
    L.xp_abi_version.argtypes = []
    if L.xp_abi_version() != ABI_VERSION:
        raise XpError("libxpic.so has ABI version %d, the binding mirrors %d: rebuild the library"
                      % (L.xp_abi_version(), ABI_VERSION))
    L.xp_last_error.restype = C.c_char_p
    L.xp_last_error.argtypes = []
    L.xp_ctx_create.restype = _i32
    L.xp_ctx_create.argtypes = [C.POINTER(_vp), _i32]
    L.xp_ctx_destroy.restype = None
    L.xp_ctx_destroy.argtypes = [_vp]
    L.xp_table_bytes.restype = C.c_size_t
    L.xp_table_bytes.argtypes = [C.POINTER(XpAtomicTables)]
    L.init_species.restype = _i32
    L.init_species.argtypes = [_vp, C.POINTER(XpAtomicTables), _vp, C.c_size_t, _vp]
    L.xp_work_bytes.restype = C.c_size_t
    L.xp_work_bytes.argtypes = [_i64, _i64, _i32, _i32]
    L.xp_step_work_bytes.restype = C.c_size_t
    L.xp_step_work_bytes.argtypes = [C.POINTER(XpBatch)]
    L.xp_lds_limits.restype = _i32
    L.xp_lds_limits.argtypes = [_vp, C.POINTER(_i32), C.POINTER(_i32)]
    L.bin_particles.restype = _i32
    L.bin_particles.argtypes = [_vp, C.POINTER(XpParticles), C.POINTER(XpBatch),
                                C.POINTER(XpCapacity), _vp, _vp]
    L.collide_ionize_step.restype = _i32
    L.collide_ionize_step.argtypes = [_vp, C.POINTER(XpBatch), C.POINTER(XpStepParams), _vp]
    L.collide_ionize_step_static.restype = _i32
    L.collide_ionize_step_static.argtypes = [_vp, C.POINTER(XpBatch), C.POINTER(XpStepParams), _vp]
    L.photo_auger_step.restype = _i32
    L.photo_auger_step.argtypes = [_vp, C.POINTER(XpBatch), C.POINTER(XpStepParams), _vp]
    L.transport_photons.restype = _i32
    L.transport_photons.argtypes = [_vp, C.POINTER(XpBatch), _vp, _vp]
    L.diagnostics.restype = _i32
    L.diagnostics.argtypes = [_vp, C.POINTER(XpBatch), _vp, _u32, _vp]
    L.xp_selftest.restype = _i32
    L.xp_selftest.argtypes = [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _vp]
    _lib = L
    return L


def check(status):
    if status != 0:
        msg = load().xp_last_error().decode(errors="replace")
        raise XpError("xpic status %d: %s" % (status, msg))


# --- thin wrappers with the C names -----------------------------------------

def xp_ctx_create(device_id=0):
    h = _vp()
    check(load().xp_ctx_create(C.byref(h), int(device_id)))
    return h


def xp_ctx_destroy(ctx):
    load().xp_ctx_destroy(ctx)


def init_species(ctx, tables, d_buf, nbytes, stream):
    check(load().init_species(ctx, C.byref(tables), _vp(d_buf), nbytes, _vp(stream)))


def xp_work_bytes(ne, ni, n_cells, n_runs):
    return int(load().xp_work_bytes(int(ne), int(ni), int(n_cells), int(n_runs)))


def xp_step_work_bytes(batch):
    return int(load().xp_step_work_bytes(C.byref(batch)))


def xp_lds_limits(ctx):
    e, i = _i32(), _i32()
    check(load().xp_lds_limits(ctx, C.byref(e), C.byref(i)))
    return int(e.value), int(i.value)


def bin_particles(ctx, parts, batch, cap, d_need, stream):
    check(load().bin_particles(ctx, C.byref(parts), C.byref(batch), C.byref(cap), _vp(d_need),
                               _vp(stream)))


def collide_ionize_step(ctx, batch, params, stream):
    check(load().collide_ionize_step(ctx, C.byref(batch), C.byref(params), _vp(stream)))


def collide_ionize_step_static(ctx, batch, params, stream):
    check(load().collide_ionize_step_static(ctx, C.byref(batch), C.byref(params), _vp(stream)))


def transport_photons(ctx, batch, d_trans, stream):
    check(load().transport_photons(ctx, C.byref(batch), _vp(d_trans), _vp(stream)))


def photo_auger_step(ctx, batch, params, stream):
    check(load().photo_auger_step(ctx, C.byref(batch), C.byref(params), _vp(stream)))


def diagnostics(ctx, batch, d_out, what, stream):
    check(load().diagnostics(ctx, C.byref(batch), _vp(d_out), int(what), _vp(stream)))


def xp_selftest(ctx, which, n, d_x, d_u, d_out, d_words, stream):
    check(load().xp_selftest(ctx, int(which), int(n), _vp(d_x), _vp(d_u), _vp(d_out),
                             _vp(d_words), _vp(stream)))


def make_tables(t):
    """xp_atomic_tables from workloads.AtomicTables; returns (struct, keepalive)."""
    arrs = {
        "bind": np.ascontiguousarray(t.bind, dtype=np.float64),
        "lotz_a": np.ascontiguousarray(t.lotz_a, dtype=np.float64),
        "lotz_b": np.ascontiguousarray(t.lotz_b, dtype=np.float64),
        "lotz_c": np.ascontiguousarray(t.lotz_c, dtype=np.float64),
        "gamma_a": np.ascontiguousarray(t.gamma_a, dtype=np.float64),
        "gamma_x": np.ascontiguousarray(t.gamma_x, dtype=np.float64),
        "e_kalpha": np.ascontiguousarray(t.e_kalpha, dtype=np.float64),
        "photo_lnsig": np.ascontiguousarray(t.photo_lnsig, dtype=np.float64),
        "eos_zbar": np.ascontiguousarray(t.eos_zbar, dtype=np.float64),
    }
    s = XpAtomicTables()
    s.z_nuc = int(t.z_nuc)
    s.photo_nh = int(t.photo_lnsig.shape[1])
    s.eos_nn, s.eos_nt = (int(v) for v in t.eos_zbar.shape)
    s.mass_ion = float(t.mass_ion)
    for k, a in arrs.items():
        setattr(s, k, a.ctypes.data)
    s.photo_lnhv0, s.photo_dlnhv = float(t.photo_lnhv0), float(t.photo_dlnhv)
    s.eos_lnn0, s.eos_dlnn = float(t.eos_lnn0), float(t.eos_dlnn)
    s.eos_lnt0, s.eos_dlnt = float(t.eos_lnt0), float(t.eos_dlnt)
    return s, arrs


def make_run(spec, cell_begin, field_per_cell=False):
    r = XpRun()
    r.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
    r.nx, r.ny = int(spec.nx), int(spec.ny)
    r.dx, r.dy, r.x0, r.y0 = spec.dx, spec.dy, spec.x0, spec.y0
    r.volume, r.w0, r.dt, r.dt_rad = spec.volume, spec.w0, spec.dt, spec.dt_rad
    r.lnl_fixed = spec.lnl_fixed
    r.e_bulk = spec.e_bulk if math.isfinite(spec.e_bulk) else 1.0e300
    r.ipd_model, r.z_floor = int(spec.ipd_model), int(spec.z_floor)
    r.cell_begin, r.ncells = int(cell_begin), int(spec.nx * spec.ny)
    nb = len(spec.photon_hv)
    if nb > XP_MAX_BINS:
        raise ValueError("at most %d photon bins" % XP_MAX_BINS)
    r.n_bins = nb
    r.field_per_cell = 1 if field_per_cell else 0
    for b in range(nb):
        r.hv[b] = float(spec.photon_hv[b])
        r.nhv[b] = float(spec.photon_n[b])
    return r
