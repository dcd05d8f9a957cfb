"""Serving: continuous batching of independent runs on one GPU.

A Pool holds particle slabs for many runs in device memory, sized by an HBM
budget.  A request (one run: its cells, particles and step count) is admitted
as soon as its footprint fits: its cells are appended to the pool's compact
cell table, its slabs are carved out of the free electron and ion ranges, and
its particles are binned straight into them.  Every pool step advances all
resident runs together in one collide_ionize_step call.  Each run keeps its
own step index in device memory, so runs admitted at different times share
every launch.  A finished run is read back and retired: its slab ranges
return to the free lists and the cell and run tables are compacted.

Slabs never move, and a run's random streams are keyed by its seed and its
run-local cell index, so a run's result does not depend on what else is
resident or when it was admitted.

`serve` drives a pool from a timed request trace (arrivals in wall-clock
seconds) and reports each request's time-to-result.  `sequential` is the
plain baseline: the same trace served one run at a time, first come first
served, each run alone in its own batch.
"""

from __future__ import annotations

import ctypes as C
import time
from collections import deque

import numpy as np
import torch

from . import binding as B
from . import runtime as RT

# device bytes per slot of the particle arrays (the step's workspace for the
# same slots is sized by the library and counted in the budget as well)
E_SLOT_BYTES = 44
I_SLOT_BYTES = 42


class RangeAlloc:
    """First-fit allocator of contiguous ranges of [0, size)."""

    def __init__(self, size):
        self.size = int(size)
        self.free = [(0, self.size)] if size > 0 else []

    def alloc(self, n):
        n = int(n)
        if n == 0:
            return 0
        for k, (s, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (s + n, l - n)
                return s
        return None

    def release(self, start, n):
        if n == 0:
            return
        self.free.append((int(start), int(n)))
        self.free.sort()
        merged = []
        for s, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((s, l))
        self.free = merged

    def used(self):
        return self.size - sum(l for _, l in self.free)


class Resident:
    """A run in the pool."""

    def __init__(self, req, cell_lo, e_lo, e_n, i_lo, i_n, big, caps):
        self.req = req
        self.caps = caps                # largest (e_cap, i_cap) of its cells
        self.cell_lo = cell_lo
        self.e_lo, self.e_n = e_lo, e_n
        self.i_lo, self.i_n = i_lo, i_n
        self.big = big                  # (cells, summed e_cap, summed i_cap) beyond the LDS plans
        self.steps_done = 0
        self.t_admit = None
        self.t_done = None

    @property
    def ncells(self):
        return self.req.spec.ncells


class Pool:
    def __init__(self, ctx: RT.Context, budget_bytes, max_cells=1 << 17, max_runs=1024,
                 capacity=(7, 16), e_share=0.88):
        self.ctx = ctx
        dev = ctx.device
        self.device = dev
        self.capacity = B.XpCapacity(int(capacity[0]), int(capacity[1]))
        self.max_cells, self.max_runs = int(max_cells), int(max_runs)
        # the budget covers the slabs and the step's workspace for any set of
        # resident runs (every slot possibly on the global-memory path)
        scale = 1.0
        for _ in range(6):
            self.E = int(budget_bytes * scale * e_share) // E_SLOT_BYTES
            self.I = int(budget_bytes * scale * (1.0 - e_share)) // I_SLOT_BYTES
            sizing = B.XpBatch()
            sizing.n_runs, sizing.n_cells = self.max_runs, self.max_cells
            sizing.big_cells_max = self.max_cells
            sizing.big_e_slots, sizing.big_i_slots = self.E, self.I
            work = B.xp_step_work_bytes(sizing)
            total = self.E * E_SLOT_BYTES + self.I * I_SLOT_BYTES + work
            if total <= budget_bytes:
                break
            scale *= 0.995 * budget_bytes / total
        f64 = lambda n: torch.empty(n, dtype=torch.float64, device=dev)
        E, I = max(self.E, 1), max(self.I, 1)
        self.ex, self.ey, self.evx, self.evy, self.evz = (f64(E) for _ in range(5))
        self.ew = torch.zeros(E, dtype=torch.int32, device=dev)
        self.ix, self.iy, self.ivx, self.ivy, self.ivz = (f64(I) for _ in range(5))
        self.iz = torch.zeros(I, dtype=torch.uint8, device=dev)
        self.ik = torch.zeros(I, dtype=torch.uint8, device=dev)
        nc = self.max_cells
        self.e_off = torch.zeros(nc, dtype=torch.int64, device=dev)
        self.i_off = torch.zeros(nc, dtype=torch.int64, device=dev)
        self.e_cap = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.i_cap = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.e_cnt = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.i_cnt = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.cell_run = torch.zeros(nc, dtype=torch.int32, device=dev)
        self.d_runs = torch.zeros(self.max_runs * C.sizeof(B.XpRun), dtype=torch.uint8, device=dev)
        self.d_step = torch.zeros(self.max_runs, dtype=torch.int32, device=dev)
        self.run_cnt = torch.zeros((self.max_runs, B.XP_NCOUNT), dtype=torch.int64, device=dev)
        self.run_led = torch.zeros((self.max_runs, B.XP_NLEDGER), dtype=torch.float64, device=dev)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=dev)
        # XP_ST_* bits per resident run (cleared on admission, read on retirement)
        self.d_run_status = torch.zeros(self.max_runs, dtype=torch.int32, device=dev)
        self.d_stats = torch.zeros(B.XP_NSTATS, dtype=torch.int32, device=dev)
        self.mirror = RT.StatsMirror(self.d_stats, np.zeros(B.XP_NSTATS, dtype=np.int32))
        self.ealloc, self.ialloc = RangeAlloc(self.E), RangeAlloc(self.I)
        self.active: list[Resident] = []
        self.cells_used = 0
        self.e_cap_max = self.i_cap_max = 0
        # workspace of the step for any set of resident runs
        probe = self._struct(self.max_cells, self.max_runs, (self.max_cells, self.E, self.I))
        self.work_bytes = B.xp_step_work_bytes(probe)
        self.d_work = torch.empty(self.work_bytes, dtype=torch.uint8, device=dev)
        self.peak_active = 0

    # -- device views ----------------------------------------------------------
    def _struct(self, n_cells, n_runs, big, cell_lo=0, slabs=None, runs_ptr=None,
                cell_run_ptr=None, status_ptr=None, work=None):
        p = RT._ptr
        b = B.XpBatch()
        b.n_runs, b.n_cells = n_runs, n_cells
        b.d_runs = runs_ptr if runs_ptr is not None else p(self.d_runs)
        b.d_cell_run = cell_run_ptr if cell_run_ptr is not None else p(self.cell_run)
        b.d_e_off = p(self.e_off) + 8 * cell_lo
        b.d_e_cap = p(self.e_cap) + 4 * cell_lo
        b.d_e_cnt = p(self.e_cnt) + 4 * cell_lo
        b.d_i_off = p(self.i_off) + 8 * cell_lo
        b.d_i_cap = p(self.i_cap) + 4 * cell_lo
        b.d_i_cnt = p(self.i_cnt) + 4 * cell_lo
        e_lo, e_n, i_lo, i_n = slabs if slabs is not None else (0, self.E, 0, self.I)
        b.e_slots, b.i_slots = e_n, i_n
        b.d_ex, b.d_ey = p(self.ex) + 8 * e_lo, p(self.ey) + 8 * e_lo
        b.d_evx, b.d_evy, b.d_evz = (p(t) + 8 * e_lo for t in (self.evx, self.evy, self.evz))
        b.d_ew = p(self.ew) + 4 * e_lo
        b.d_ix, b.d_iy = p(self.ix) + 8 * i_lo, p(self.iy) + 8 * i_lo
        b.d_ivx, b.d_ivy, b.d_ivz = (p(t) + 8 * i_lo for t in (self.ivx, self.ivy, self.ivz))
        b.d_iz, b.d_ik = p(self.iz) + i_lo, p(self.ik) + i_lo
        b.d_run_counters, b.d_run_ledger = p(self.run_cnt), p(self.run_led)
        b.d_status = status_ptr if status_ptr is not None else p(self.d_status)
        # admission views carry a run table of their own: no per-run words there
        b.d_run_status = p(self.d_run_status) if runs_ptr is None and hasattr(self, "d_run_status") \
            else None
        if work is None:
            b.d_work, b.work_bytes = p(self.d_work) if hasattr(self, "d_work") else None, \
                getattr(self, "work_bytes", 0)
        else:
            b.d_work, b.work_bytes = p(work), work.numel()
        b.e_cap_max, b.i_cap_max = max(self.e_cap_max, 1), self.i_cap_max
        b.d_stats = p(self.d_stats)
        b.big_cells_max, b.big_e_slots, b.big_i_slots = big
        return b

    def _caps(self):
        self.e_cap_max = max((r.caps[0] for r in self.active), default=0)
        self.i_cap_max = max((r.caps[1] for r in self.active), default=0)

    def _run_bytes(self):
        structs = []
        for k, r in enumerate(self.active):
            structs.append(B.make_run(r.req.spec, r.cell_lo))
        arr = (B.XpRun * max(len(structs), 1))(*structs) if structs else (B.XpRun * 1)()
        return bytes(arr)

    def _upload_runs(self):
        raw = self._run_bytes()
        t = torch.frombuffer(bytearray(raw), dtype=torch.uint8)
        self.d_runs[:t.numel()].copy_(t.to(self.device))

    # -- admission ---------------------------------------------------------------
    def try_admit(self, req):
        """Admit a request if its cells, slabs and run slot fit; False otherwise."""
        spec, parts = req.spec, req.parts
        nc = spec.ncells
        if len(self.active) >= self.max_runs or self.cells_used + nc > self.max_cells:
            return False
        dev = self.device
        cell_lo = self.cells_used
        run = torch.frombuffer(bytearray(bytes(B.make_run(spec, 0))), dtype=torch.uint8).to(dev)
        cell_run = torch.zeros(nc, dtype=torch.int32, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        need = torch.zeros(8, dtype=torch.int64, device=dev)
        two_d = spec.ny > 1
        inp = {f: RT._dev(getattr(parts, f), dev) for f in ("ex", "ey", "evx", "evy", "evz",
                                                            "ix", "iy", "ivx", "ivy", "ivz")}
        inp["ew"] = RT._dev(parts.ew.astype(np.uint32).view(np.int32), dev)
        inp["iz"] = RT._dev(parts.iz.astype(np.uint8), dev)
        inp["ik"] = RT._dev(parts.ik.astype(np.uint8), dev)
        p = B.XpParticles()
        p.ne, p.ni = parts.ne, parts.ni
        p.d_ex, p.d_ey = RT._ptr(inp["ex"]), RT._ptr(inp["ey"]) if two_d else None
        p.d_evx, p.d_evy, p.d_evz = (RT._ptr(inp[k]) for k in ("evx", "evy", "evz"))
        p.d_ew = RT._ptr(inp["ew"])
        p.d_ix, p.d_iy = RT._ptr(inp["ix"]), RT._ptr(inp["iy"]) if two_d else None
        p.d_ivx, p.d_ivy, p.d_ivz = (RT._ptr(inp[k]) for k in ("ivx", "ivy", "ivz"))
        p.d_iz, p.d_ik = RT._ptr(inp["iz"]), RT._ptr(inp["ik"])
        work = torch.empty(B.xp_work_bytes(parts.ne, parts.ni, nc, 1), dtype=torch.uint8, device=dev)
        # sizing pass: no slab is written (XP_ST_BIN_SIZE), the cell range gets counts and caps
        view = self._struct(nc, 1, (0, 0, 0), cell_lo=cell_lo, slabs=(0, 0, 0, 0),
                            runs_ptr=RT._ptr(run), cell_run_ptr=RT._ptr(cell_run),
                            status_ptr=RT._ptr(status), work=work)
        B.bin_particles(self.ctx.h, p, view, self.capacity, RT._ptr(need), RT._stream())
        n = need.cpu().numpy()
        e_n, i_n = int(n[0]), int(n[1])
        e_lo = self.ealloc.alloc(e_n)
        if e_lo is None:
            return False
        i_lo = self.ialloc.alloc(i_n)
        if i_lo is None:
            self.ealloc.release(e_lo, e_n)
            return False
        status.zero_()
        view = self._struct(nc, 1, (0, 0, 0), cell_lo=cell_lo, slabs=(e_lo, e_n, i_lo, i_n),
                            runs_ptr=RT._ptr(run), cell_run_ptr=RT._ptr(cell_run),
                            status_ptr=RT._ptr(status), work=work)
        B.bin_particles(self.ctx.h, p, view, self.capacity, RT._ptr(need), RT._stream())
        if int(status.item()) & B.XP_ST_BIN_SIZE:
            raise B.XpError("admission: slab range smaller than the binning needs")
        # offsets of the view are relative to its slab range
        self.e_off[cell_lo:cell_lo + nc] += e_lo
        self.i_off[cell_lo:cell_lo + nc] += i_lo
        k = len(self.active)
        self.cell_run[cell_lo:cell_lo + nc] = k
        self.d_step[k] = 0
        self.d_run_status[k] = 0
        self.run_cnt[k].zero_()
        self.run_led[k].zero_()
        n = need.cpu().numpy()
        r = Resident(req, cell_lo, e_lo, e_n, i_lo, i_n, (int(n[4]), int(n[5]), int(n[6])),
                     (int(n[2]), int(n[3])))
        self.active.append(r)
        self.cells_used += nc
        self._caps()
        self._upload_runs()
        self.peak_active = max(self.peak_active, len(self.active))
        return True

    # -- stepping ------------------------------------------------------------------
    def _big_bounds(self):
        nb = sum(r.big[0] for r in self.active)
        if nb == 0:
            return (0, 0, 0)
        return (nb, sum(r.big[1] for r in self.active), sum(r.big[2] for r in self.active))

    def step(self, k=1, schedule=0):
        """k steps of every resident run (enqueued, no synchronization)."""
        if not self.active:
            return
        b = self._struct(self.cells_used, len(self.active), self._big_bounds())
        hint = self.mirror.hint(0.9)
        nr = len(self.active)
        for _ in range(k):
            prm = B.XpStepParams(B.XP_ALL, 0, RT._ptr(self.d_step), int(schedule), hint, 0, 0)
            B.collide_ionize_step(self.ctx.h, b, prm, RT._stream())
            self.d_step[:nr].add_(1)
        self.mirror.after_step()
        for r in self.active:
            r.steps_done += k

    def status(self):
        return int(self.d_status.item())

    # -- read-back and retirement --------------------------------------------------
    def state(self, r: Resident) -> RT.CompactState:
        """Particle state of a resident run (canonical cell order)."""
        c0, nc = r.cell_lo, r.ncells
        eo = self.e_off[c0:c0 + nc].cpu().numpy()
        en = self.e_cnt[c0:c0 + nc].cpu().numpy().astype(np.int64)
        io = self.i_off[c0:c0 + nc].cpu().numpy()
        inn = self.i_cnt[c0:c0 + nc].cpu().numpy().astype(np.int64)
        cat = lambda o, n: np.concatenate([np.arange(a, a + m) for a, m in zip(o, n)]) if n.sum() \
            else np.zeros(0, np.int64)
        ei, ii = cat(eo, en), cat(io, inn)
        et = torch.from_numpy(ei).to(self.device)
        it = torch.from_numpy(ii).to(self.device)
        g = lambda t, idx: t[idx].cpu().numpy()
        two_d = r.req.spec.ny > 1
        return RT.CompactState(
            e_start=np.concatenate([[0], np.cumsum(en)]), ex=g(self.ex, et),
            ey=g(self.ey, et) if two_d else np.zeros(ei.size),
            evx=g(self.evx, et), evy=g(self.evy, et), evz=g(self.evz, et),
            ew=g(self.ew, et).view(np.uint32),
            i_start=np.concatenate([[0], np.cumsum(inn)]), ix=g(self.ix, it),
            iy=g(self.iy, it) if two_d else np.zeros(ii.size),
            ivx=g(self.ivx, it), ivy=g(self.ivy, it), ivz=g(self.ivz, it),
            iz=g(self.iz, it), ik=g(self.ik, it))

    def counters(self, r: Resident):
        k = self.active.index(r)
        return self.run_cnt[k].cpu().numpy().view(np.uint64)

    def run_status(self, r: Resident):
        """XP_ST_* bits raised by the run's own cells since its admission."""
        k = self.active.index(r)
        return int(self.d_run_status[k].item()) & 0xFFFFFFFF

    def retire(self, done):
        """Drop finished runs: free their slabs, compact the cell and run tables."""
        if not done:
            return
        done_ids = {id(r) for r in done}
        keep = [r for r in self.active if id(r) not in done_ids]
        for r in done:
            self.ealloc.release(r.e_lo, r.e_n)
            self.ialloc.release(r.i_lo, r.i_n)
        old_idx = [self.active.index(r) for r in keep]
        slices = [(r.cell_lo, r.ncells) for r in keep]
        arrays = (self.e_off, self.i_off, self.e_cap, self.i_cap, self.e_cnt, self.i_cnt)
        if keep:
            new = [torch.cat([a[c:c + n] for c, n in slices]) for a in arrays]
            total = sum(n for _, n in slices)
            for a, v in zip(arrays, new):
                a[:total].copy_(v)
            lo = 0
            for k, r in enumerate(keep):
                r.cell_lo = lo
                self.cell_run[lo:lo + r.ncells] = k
                lo += r.ncells
            idx = torch.tensor(old_idx, dtype=torch.int64, device=self.device)
            self.d_step[:len(keep)] = self.d_step[idx].clone()
            self.d_run_status[:len(keep)] = self.d_run_status[idx].clone()
            self.run_cnt[:len(keep)] = self.run_cnt[idx].clone()
            self.run_led[:len(keep)] = self.run_led[idx].clone()
        self.active = keep
        self.cells_used = sum(r.ncells for r in keep)
        self._caps()
        self._upload_runs()


def serve(pool: Pool, trace, k=8, on_done=None, clock=time.perf_counter):
    """Serve a request trace (arrival times in seconds from the start) with
    continuous batching.  Returns per-request records: arrival, admission and
    completion times (s) and the run's accumulated counters."""
    pending = deque(sorted(trace, key=lambda q: q.arrival))
    queue = deque()
    out = {}
    t0 = clock()
    waited = 0
    while pending or queue or pool.active:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        while queue:
            if not pool.try_admit(queue[0]):
                break
            pool.active[-1].t_admit = clock() - t0
            queue.popleft()
        if queue and pool.active:
            waited = max(waited, len(queue))
        if not pool.active:
            if queue:
                raise B.XpError("request %d does not fit an empty pool" % queue[0].rid)
            if pending:
                time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
            continue
        kk = min(k, min(r.req.nsteps - r.steps_done for r in pool.active))
        pool.step(kk)
        done = [r for r in pool.active if r.steps_done >= r.req.nsteps]
        if done:
            torch.cuda.synchronize()
            t = clock() - t0
            for r in done:
                r.t_done = t
                rec = {"rid": r.req.rid, "arrival": r.req.arrival, "admit": r.t_admit,
                       "done": t, "ttr": t - r.req.arrival, "steps": r.req.nsteps,
                       "counters": pool.counters(r).copy(), "status": pool.run_status(r)}
                if on_done is not None:
                    on_done(pool, r, rec)
                out[r.req.rid] = rec
            pool.retire(done)
    return out, waited


def sequential(ctx: RT.Context, trace, capacity=(7, 16), clock=time.perf_counter, on_done=None):
    """The plain baseline: first come, first served, one run at a time, each
    alone in its own batch with eager steps.  on_done(record) after each run."""
    out = {}
    t0 = clock()
    for q in sorted(trace, key=lambda q: q.arrival):
        now = clock() - t0
        if q.arrival > now:
            time.sleep(q.arrival - now)
        start = clock() - t0
        bat = RT.Batch(ctx, [(q.spec, q.parts)], capacity=capacity)
        for s in range(q.nsteps):
            bat.step(s)
        torch.cuda.synchronize()
        t = clock() - t0
        out[q.rid] = {"rid": q.rid, "arrival": q.arrival, "admit": start, "done": t,
                      "ttr": t - q.arrival, "steps": q.nsteps,
                      "counters": bat.run_counters()[0].copy(), "status": bat.status()}
        if on_done is not None:
            on_done(out[q.rid])
        del bat
    return out


def latency_summary(records, elapsed=None):
    ttr = np.array([r["ttr"] for r in records.values()])
    done = max(r["done"] for r in records.values())
    span = elapsed if elapsed is not None else done
    return {"p50_s": float(np.percentile(ttr, 50)), "p99_s": float(np.percentile(ttr, 99)),
            "mean_s": float(ttr.mean()), "runs": len(ttr),
            "runs_per_hour": len(ttr) * 3600.0 / span, "makespan_s": float(done)}
