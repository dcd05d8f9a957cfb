"""Device-resident runs driven through the C ABI.

`Context` owns an xp_ctx and the device copy of the atomic tables.  `Batch`
owns the device memory of one or more independent runs (run table, cell slabs,
counters, workspace) as torch tensors and calls the library entry points on
torch's current stream.  Nothing here computes any part of the method.
"""

from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B


def plan_hint(stats, quantile=0.9):
    """LDS plan size for the next step from a step's stats: the electron
    count that covers `quantile` of the cells stepped in LDS (16-electron
    buckets); cells above it are re-planned with more LDS in the same call.
    quantile >= 1: the largest cell."""
    stats = np.asarray(stats)
    if quantile >= 1.0:
        m = int(stats[0])
        return m if m > 0 else 0
    hist = stats[4:4 + 64].astype(np.int64)
    tot = int(hist.sum())
    if tot == 0:
        return 0
    need = quantile * tot
    cum = np.cumsum(hist)
    b = int(np.searchsorted(cum, need))
    if b >= 63:
        return int(stats[0])
    return max(16, 16 * b)


def count_stats(e_cnt):
    """d_stats-shaped record of the electron counts per cell (the largest and
    the 16-electron histogram), for the plan of a batch's first step."""
    n = np.asarray(e_cnt, dtype=np.int64)
    st = np.zeros(B.XP_NSTATS, dtype=np.int32)
    if n.size:
        st[0] = int(n.max())
        b = np.minimum((n + 15) // 16, 63)
        st[4:4 + 64] = np.bincount(b, minlength=64)[:64]
    return st


class StatsMirror:
    """Host copy of a batch's per-step stats (d_stats) for the LDS plan hint.

    The copy after each step is asynchronous, into a ring of pinned buffers;
    the hint uses the newest copy that has landed.  At most DEPTH copies are in
    flight: a host that runs further ahead of the device waits for the oldest,
    so the plan is never more than DEPTH steps old.
    """

    DEPTH = 4

    def __init__(self, d_stats, initial):
        self.d = d_stats
        self.bufs = [torch.zeros(B.XP_NSTATS, dtype=torch.int32, pin_memory=True)
                     for _ in range(self.DEPTH)]
        self.pending = []          # (event, buffer index), oldest first
        self.k = 0
        self.last = np.asarray(initial, dtype=np.int32).copy()

    def _harvest(self, wait_oldest=False):
        while self.pending:
            ev, i = self.pending[0]
            if wait_oldest:
                ev.synchronize()
                wait_oldest = False
            elif not ev.query():
                break
            self.last = self.bufs[i].numpy().copy()
            self.pending.pop(0)

    def after_step(self):
        if len(self.pending) >= self.DEPTH:
            self._harvest(wait_oldest=True)
        i = self.k % self.DEPTH
        self.k += 1
        self.bufs[i].copy_(self.d, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        self.pending.append((ev, i))

    def stats(self):
        self._harvest()
        return self.last

    def hint(self, quantile=0.9):
        return plan_hint(self.stats(), quantile)


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dev(a, device, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def _ptr(t):
    return None if t is None else t.data_ptr()


class Context:
    """An xp_ctx bound to one device with the atomic tables uploaded."""

    def __init__(self, tables, device="cuda:0"):
        if not torch.cuda.is_available():
            raise B.XpError("no HIP device is available")
        self.device = torch.device(device)
        B.load()
        self.h = B.xp_ctx_create(self.device.index or 0)
        s, keep = B.make_tables(tables)
        nbytes = B.load().xp_table_bytes(C.byref(s))
        self.table_buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        B.init_species(self.h, s, self.table_buf.data_ptr(), nbytes, _stream())
        self._keep = keep
        self.tables = tables

    def close(self):
        if getattr(self, "h", None):
            B.xp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class CompactState:
    """Particle state gathered into the compact cell-major layout."""
    e_start: np.ndarray
    ex: np.ndarray
    ey: np.ndarray
    evx: np.ndarray
    evy: np.ndarray
    evz: np.ndarray
    ew: np.ndarray
    i_start: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    ivx: np.ndarray
    ivy: np.ndarray
    ivz: np.ndarray
    iz: np.ndarray
    ik: np.ndarray

    @property
    def ne_cell(self):
        return np.diff(self.e_start)

    @property
    def ni_cell(self):
        return np.diff(self.i_start)


class Batch:
    """Independent runs resident in device memory.

    runs: list of (workloads.RunSpec, workloads.Particles).  capacity =
    (electron slots per ion, extra slots) of every cell's electron slab.
    cell_records keeps per-cell counters, tallies and moments of the last step.
    cell_nhv: initial photon field per cell ([n_cells][n_bins], photons / m^3);
    the runs then read it instead of their uniform field, and transport()
    rebuilds it after a step (the batch records photon events per cell).
    big: workspace of the global-memory path -- "auto" for the cells whose
    slabs may outgrow one workgroup's LDS, "all" so that every cell can take it
    (step(..., schedule=3)).
    """

    def __init__(self, ctx: Context, runs, capacity=(7, 16), cell_records=False,
                 cell_nhv=None, big="auto", kalpha_return=False):
        if big not in ("auto", "all"):
            raise ValueError("big must be 'auto' or 'all'")
        self.big = big
        self.big_cells_max, self.big_e_slots, self.big_i_slots = 0, 0, 0
        self.ctx = ctx
        dev = ctx.device
        self.device = dev
        self.n_runs = len(runs)
        self.specs = [r[0] for r in runs]
        structs, begin = [], 0
        self.cell_begin = []
        for spec, _ in runs:
            structs.append(B.make_run(spec, begin, field_per_cell=cell_nhv is not None))
            self.cell_begin.append(begin)
            begin += spec.nx * spec.ny
        self.n_cells = begin
        arr = (B.XpRun * self.n_runs)(*structs)
        self.d_runs = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(dev)
        self.d_cell_run = _dev(np.repeat(np.arange(self.n_runs, dtype=np.int32),
                                         [s.nx * s.ny for s in self.specs]), dev)
        nc = max(self.n_cells, 1)
        self.d_e_off = torch.zeros(nc, dtype=torch.int64, device=dev)
        self.d_i_off = torch.zeros(nc, dtype=torch.int64, device=dev)
        self.d_e_cap = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.d_i_cap = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.d_e_cnt = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.d_i_cnt = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.d_run_status = torch.zeros(self.n_runs, dtype=torch.int32, device=dev)
        self.d_need = torch.zeros(8, dtype=torch.int64, device=dev)
        self.d_stats = torch.zeros(B.XP_NSTATS, dtype=torch.int32, device=dev)
        self.mirror = None          # set after binning
        self.e_hint = 0
        self.d_run_cnt = torch.zeros((self.n_runs, B.XP_NCOUNT), dtype=torch.int64, device=dev)
        self.d_run_led = torch.zeros((self.n_runs, B.XP_NLEDGER), dtype=torch.float64, device=dev)
        self.d_cell_nhv = None
        if cell_nhv is not None:
            f = np.zeros((self.n_cells, B.XP_MAX_BINS))
            f[:, :np.asarray(cell_nhv).shape[1]] = cell_nhv
            self.d_cell_nhv = _dev(f, dev)
        self.d_cell_nabs = None
        self.d_trans = None
        if cell_nhv is not None:
            self.d_cell_nabs = torch.zeros((max(self.n_cells, 1), B.XP_MAX_BINS), dtype=torch.int32,
                                           device=dev)
            self.d_trans = torch.zeros((self.n_runs, B.XP_MAX_BINS), dtype=torch.float64, device=dev)
        # K-alpha photons returned to the field per cell and bin (steps with
        # XP_KA_FIELD write them, transport_photons adds them to the beam)
        self.d_cell_nka = None
        if kalpha_return:
            self.d_cell_nka = torch.zeros((max(self.n_cells, 1), B.XP_MAX_BINS), dtype=torch.float64,
                                          device=dev)
        self.cell_records = cell_records
        if cell_records:
            self.d_cell_cnt = torch.zeros((nc, B.XP_NCOUNT), dtype=torch.int64, device=dev)
            self.d_cell_led = torch.zeros((nc, B.XP_NLEDGER), dtype=torch.float64, device=dev)
            self.d_cell_mom = torch.zeros((nc, B.XP_NMOM), dtype=torch.float64, device=dev)
        else:
            self.d_cell_cnt = self.d_cell_led = self.d_cell_mom = None
        self._inputs(runs)
        self.capacity = B.XpCapacity(int(capacity[0]), int(capacity[1]))
        self._bin()

    # -- setup ----------------------------------------------------------------
    def _inputs(self, runs):
        dev = self.device
        cat = lambda f: np.concatenate([getattr(p, f) for _, p in runs])
        self.in_ne = int(sum(p.ne for _, p in runs))
        self.in_ni = int(sum(p.ni for _, p in runs))
        self.in_e = {f: _dev(cat(f), dev) for f in ("ex", "ey", "evx", "evy", "evz")}
        self.in_e["ew"] = _dev(cat("ew").astype(np.uint32).view(np.int32), dev)
        self.in_i = {f: _dev(cat(f), dev) for f in ("ix", "iy", "ivx", "ivy", "ivz")}
        self.in_i["iz"] = _dev(cat("iz").astype(np.uint8), dev)
        self.in_i["ik"] = _dev(cat("ik").astype(np.uint8), dev)
        self.in_e_run = _dev(np.repeat(np.arange(self.n_runs, dtype=np.int32),
                                       [p.ne for _, p in runs]), dev)
        self.in_i_run = _dev(np.repeat(np.arange(self.n_runs, dtype=np.int32),
                                       [p.ni for _, p in runs]), dev)
        self.two_d = any(s.ny > 1 for s in self.specs)
        self.work_bytes = int(B.load().xp_work_bytes(self.in_ne, self.in_ni, self.n_cells,
                                                     self.n_runs))
        self.d_work = torch.empty(self.work_bytes, dtype=torch.uint8, device=dev)

    def _alloc_slabs(self, e_slots, i_slots):
        dev = self.device
        e, i = max(int(e_slots), 1), max(int(i_slots), 1)
        self.e_slots, self.i_slots = int(e_slots), int(i_slots)
        f64 = lambda n: torch.zeros(n, dtype=torch.float64, device=dev)
        self.ex, self.ey = f64(e), f64(e)
        self.evx, self.evy, self.evz = f64(e), f64(e), f64(e)
        self.ew = torch.zeros(e, dtype=torch.int32, device=dev)
        self.ix, self.iy = f64(i), f64(i)
        self.ivx, self.ivy, self.ivz = f64(i), f64(i), f64(i)
        self.iz = torch.zeros(i, dtype=torch.uint8, device=dev)
        self.ik = torch.zeros(i, dtype=torch.uint8, device=dev)

    def _particles(self):
        p = B.XpParticles()
        p.ne, p.ni = self.in_ne, self.in_ni
        p.d_e_run, p.d_i_run = _ptr(self.in_e_run), _ptr(self.in_i_run)
        p.d_ex, p.d_ey = _ptr(self.in_e["ex"]), _ptr(self.in_e["ey"]) if self.two_d else None
        p.d_evx, p.d_evy, p.d_evz = (_ptr(self.in_e[k]) for k in ("evx", "evy", "evz"))
        p.d_ew = _ptr(self.in_e["ew"])
        p.d_ix, p.d_iy = _ptr(self.in_i["ix"]), _ptr(self.in_i["iy"]) if self.two_d else None
        p.d_ivx, p.d_ivy, p.d_ivz = (_ptr(self.in_i[k]) for k in ("ivx", "ivy", "ivz"))
        p.d_iz, p.d_ik = _ptr(self.in_i["iz"]), _ptr(self.in_i["ik"])
        return p

    def struct(self) -> B.XpBatch:
        b = B.XpBatch()
        b.n_runs, b.n_cells = self.n_runs, self.n_cells
        b.d_runs, b.d_cell_run = _ptr(self.d_runs), _ptr(self.d_cell_run)
        b.d_e_off, b.d_e_cap, b.d_e_cnt = _ptr(self.d_e_off), _ptr(self.d_e_cap), _ptr(self.d_e_cnt)
        b.d_i_off, b.d_i_cap, b.d_i_cnt = _ptr(self.d_i_off), _ptr(self.d_i_cap), _ptr(self.d_i_cnt)
        b.e_slots, b.i_slots = self.e_slots, self.i_slots
        if self.e_slots > 0:
            b.d_ex, b.d_ey = _ptr(self.ex), _ptr(self.ey) if self.two_d else None
            b.d_evx, b.d_evy, b.d_evz = _ptr(self.evx), _ptr(self.evy), _ptr(self.evz)
            b.d_ew = _ptr(self.ew)
        if self.i_slots > 0:
            b.d_ix, b.d_iy = _ptr(self.ix), _ptr(self.iy) if self.two_d else None
            b.d_ivx, b.d_ivy, b.d_ivz = _ptr(self.ivx), _ptr(self.ivy), _ptr(self.ivz)
            b.d_iz, b.d_ik = _ptr(self.iz), _ptr(self.ik)
        b.d_cell_nhv = _ptr(self.d_cell_nhv)
        b.d_run_counters, b.d_run_ledger = _ptr(self.d_run_cnt), _ptr(self.d_run_led)
        b.d_cell_counters = _ptr(self.d_cell_cnt)
        b.d_cell_ledger = _ptr(self.d_cell_led)
        b.d_cell_moments = _ptr(self.d_cell_mom)
        b.d_status = _ptr(self.d_status)
        b.d_work, b.work_bytes = _ptr(self.d_work), self.work_bytes
        b.e_cap_max = getattr(self, "e_cap_max", 0)
        b.i_cap_max = getattr(self, "i_cap_max", 0)
        b.d_stats = _ptr(self.d_stats)
        b.big_cells_max = self.big_cells_max
        b.big_e_slots, b.big_i_slots = self.big_e_slots, self.big_i_slots
        b.d_cell_nabs = _ptr(self.d_cell_nabs)
        b.d_run_status = _ptr(self.d_run_status)
        b.d_cell_nka = _ptr(self.d_cell_nka)
        return b

    def _bin(self):
        self._alloc_slabs(0, 0)
        parts = self._particles()
        b = self.struct()
        B.bin_particles(self.ctx.h, parts, b, self.capacity, self.d_need.data_ptr(), _stream())
        need = self.d_need.cpu().numpy()
        self._alloc_slabs(need[0], need[1])
        self.d_status.zero_()
        b = self.struct()
        B.bin_particles(self.ctx.h, parts, b, self.capacity, self.d_need.data_ptr(), _stream())
        need = self.d_need.cpu().numpy()
        self.e_cap_max, self.i_cap_max = int(need[2]), int(need[3])
        st = int(self.d_status.item())
        if st & B.XP_ST_BIN_SIZE:
            raise B.XpError("bin_particles: slab arrays too small after sizing")
        if self.big == "all":
            self.big_cells_max, self.big_e_slots, self.big_i_slots = (
                self.n_cells, self.e_slots, self.i_slots)
        else:
            self.big_cells_max, self.big_e_slots, self.big_i_slots = (
                int(need[4]), int(need[5]), int(need[6]))
        step_bytes = B.xp_step_work_bytes(self.struct())
        if step_bytes > self.work_bytes:
            self.work_bytes = step_bytes
            self.d_work = torch.empty(self.work_bytes, dtype=torch.uint8, device=self.device)
        # the first step plans for the binned counts
        self.mirror = StatsMirror(self.d_stats, count_stats(self.d_e_cnt[:self.n_cells].cpu().numpy()))

    # -- the method ---------------------------------------------------------------
    def plan_hint(self, quantile=0.9):
        """LDS plan hint from the newest stats that reached the host."""
        return self.mirror.hint(quantile)

    def _hint(self, use_hint, quantile=0.9):
        if not use_hint:
            return 0
        return self.plan_hint(quantile)

    def _after(self):
        self.mirror.after_step()

    def _params(self, step, flags, schedule, d_step, use_hint, e_hint, big_grid):
        hint = int(e_hint) if e_hint is not None else self._hint(use_hint)
        return B.XpStepParams(int(flags), int(step), _ptr(d_step), int(schedule), hint,
                              int(big_grid), 0)

    def step(self, step, flags=B.XP_ALL, schedule=0, d_step=None, use_hint=True, e_hint=None,
             big_grid=0, record_stats=True):
        """One step of every run.  d_step: optional int32 [n_runs] device step
        index per run (overrides step).  e_hint / big_grid / schedule change
        speed only.  record_stats=False skips the stats read-back (graph capture)."""
        p = self._params(step, flags, schedule, d_step, use_hint, e_hint, big_grid)
        B.collide_ionize_step(self.ctx.h, self.struct(), p, _stream())
        if record_stats:
            self._after()

    def photo_auger(self, step, flags=B.XP_PHOTO | B.XP_DECAY, schedule=0, d_step=None,
                    use_hint=True, e_hint=None, big_grid=0, record_stats=True):
        p = self._params(step, flags, schedule, d_step, use_hint, e_hint, big_grid)
        B.photo_auger_step(self.ctx.h, self.struct(), p, _stream())
        if record_stats:
            self._after()

    def transport(self):
        """Reduced radiation transport after a step (transport_photons): the
        per-cell field is rebuilt from the runs' incident densities and the
        step's photon events.  Returns the device array of run transmissions
        [n_runs][XP_MAX_BINS] (no host sync)."""
        if self.d_cell_nhv is None:
            raise ValueError("transport needs a batch created with cell_nhv")
        B.transport_photons(self.ctx.h, self.struct(), _ptr(self.d_trans), _stream())
        return self.d_trans

    def cell_field(self, run=0):
        c0 = self.cell_begin[run]
        nc = self.specs[run].nx * self.specs[run].ny
        nb = len(self.specs[run].photon_hv)
        return self.d_cell_nhv[c0:c0 + nc, :nb].cpu().numpy()

    def absorbed(self, run=0):
        c0 = self.cell_begin[run]
        nc = self.specs[run].nx * self.specs[run].ny
        return self.d_cell_nabs[c0:c0 + nc].cpu().numpy()

    def kalpha_field(self, run=0):
        """K-alpha macro-photons returned per bin by the last step, [cells][XP_MAX_BINS]."""
        c0 = self.cell_begin[run]
        nc = self.specs[run].nx * self.specs[run].ny
        return self.d_cell_nka[c0:c0 + nc].cpu().numpy()

    def diagnostics(self, reset=False):
        out = torch.zeros(self.n_runs * C.sizeof(B.XpDiag), dtype=torch.uint8, device=self.device)
        B.diagnostics(self.ctx.h, self.struct(), out.data_ptr(),
                      B.XP_DIAG_RESET if reset else 0, _stream())
        raw = out.cpu().numpy().tobytes()
        sz = C.sizeof(B.XpDiag)
        return [B.XpDiag.from_buffer_copy(raw[r * sz:(r + 1) * sz]) for r in range(self.n_runs)]

    def status(self):
        return int(self.d_status.item())

    def run_status(self):
        """XP_ST_* bits of each run since the batch was built."""
        return self.d_run_status.cpu().numpy().view(np.uint32).copy()

    def stats(self):
        """Of the last step: [0] largest electron count of an LDS cell, [1] LDS
        re-plans, [2] cells on the global-memory path, [3] largest electron
        count among those, [4 + b] LDS cells with 16(b-1) < n_e <= 16 b."""
        return self.d_stats.cpu().numpy().copy()

    # -- read-back for checks ---------------------------------------------------
    def _cells_state(self, c0, nc) -> CompactState:
        """Live particles of cells [c0, c0 + nc) in slot order, gathered on the
        device and copied once."""
        dev = self.device

        def live(off, cnt):
            o = off[c0:c0 + nc]
            n = cnt[c0:c0 + nc].to(torch.int64)
            tot = int(n.sum().item())
            if tot == 0:
                return n, torch.zeros(0, dtype=torch.int64, device=dev)
            first = torch.cumsum(n, 0) - n
            rank = torch.arange(tot, dtype=torch.int64, device=dev) - torch.repeat_interleave(first, n)
            return n, torch.repeat_interleave(o, n) + rank

        en, eidx = live(self.d_e_off, self.d_e_cnt)
        inn, iidx = live(self.d_i_off, self.d_i_cnt)
        g = lambda t, idx: t.index_select(0, idx).cpu().numpy()
        ey = g(self.ey, eidx) if self.two_d else np.zeros(eidx.numel())
        iy = g(self.iy, iidx) if self.two_d else np.zeros(iidx.numel())
        en, inn = en.cpu().numpy(), inn.cpu().numpy()
        return CompactState(
            e_start=np.concatenate([[0], np.cumsum(en)]), ex=g(self.ex, eidx), ey=ey,
            evx=g(self.evx, eidx), evy=g(self.evy, eidx), evz=g(self.evz, eidx),
            ew=g(self.ew, eidx).view(np.uint32),
            i_start=np.concatenate([[0], np.cumsum(inn)]), ix=g(self.ix, iidx), iy=iy,
            ivx=g(self.ivx, iidx), ivy=g(self.ivy, iidx), ivz=g(self.ivz, iidx),
            iz=g(self.iz, iidx), ik=g(self.ik, iidx))

    def state(self, run=0) -> CompactState:
        c0 = self.cell_begin[run]
        return self._cells_state(c0, self.specs[run].nx * self.specs[run].ny)

    def states(self):
        """state(r) of every run, from one gather and one copy of the batch."""
        whole = self._cells_state(0, self.n_cells)
        out = []
        for r, spec in enumerate(self.specs):
            c0, nc = self.cell_begin[r], spec.nx * spec.ny
            es, is_ = whole.e_start, whole.i_start
            e0, e1, i0, i1 = es[c0], es[c0 + nc], is_[c0], is_[c0 + nc]
            out.append(CompactState(
                e_start=es[c0:c0 + nc + 1] - e0, ex=whole.ex[e0:e1], ey=whole.ey[e0:e1],
                evx=whole.evx[e0:e1], evy=whole.evy[e0:e1], evz=whole.evz[e0:e1], ew=whole.ew[e0:e1],
                i_start=is_[c0:c0 + nc + 1] - i0, ix=whole.ix[i0:i1], iy=whole.iy[i0:i1],
                ivx=whole.ivx[i0:i1], ivy=whole.ivy[i0:i1], ivz=whole.ivz[i0:i1],
                iz=whole.iz[i0:i1], ik=whole.ik[i0:i1]))
        return out

    def cell_records_of(self, run=0):
        c0 = self.cell_begin[run]
        nc = self.specs[run].nx * self.specs[run].ny
        return (self.d_cell_cnt[c0:c0 + nc].cpu().numpy(),
                self.d_cell_led[c0:c0 + nc].cpu().numpy(),
                self.d_cell_mom[c0:c0 + nc].cpu().numpy())

    def run_counters(self):
        return self.d_run_cnt.cpu().numpy().view(np.uint64)
