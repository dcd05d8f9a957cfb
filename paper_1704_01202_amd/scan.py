"""Batched scans: many independent runs stepped together on one GPU.

All runs of a scan (for example an intensity or photon-energy scan of 0D
runs) live in one batch.  Every step is one call of collide_ionize_step over
all of them.  Cells that fit one workgroup's LDS take the LDS path; larger
cells take the global-memory path, which spreads each cell over many
workgroups.  Together these split the work by per-cell size.  Each run keeps
its own step index in device memory (d_step), so a HIP graph captured over k
steps advances every run by k on each replay.

Knobs that change speed but never results (schedule, the quantile of cell
sizes the first LDS plan covers, global-path grid) are picked by timing real steps: the physics of the step
does not depend on them, so a tuning step is an ordinary step of the scan.

The sequential baseline steps every run alone, one after the other, with
eager launches: what a plain loop over the runs would do.
"""

from __future__ import annotations

import time

import torch

from . import binding as B
from . import runtime as RT


class Scan:
    def __init__(self, ctx: RT.Context, runs, capacity=(7, 16), flags=B.XP_ALL):
        self.ctx = ctx
        self.flags = int(flags)
        self.bat = RT.Batch(ctx, runs, capacity=capacity)
        self.n_runs = len(runs)
        self.d_step = torch.zeros(self.n_runs, dtype=torch.int32, device=ctx.device)
        self.steps_done = 0
        self.config = {"schedule": 0, "quantile": 0.9, "big_grid": 0}
        self.graph = None
        self.graph_k = 0
        self.tuning = []

    # -- stepping ---------------------------------------------------------
    def _hint(self):
        return self.bat.plan_hint(self.config["quantile"])

    def eager_step(self):
        c = self.config
        self.bat.step(0, self.flags, schedule=c["schedule"], d_step=self.d_step,
                      e_hint=self._hint(), big_grid=c["big_grid"])
        self.d_step.add_(1)
        self.steps_done += 1

    def autotune(self, candidates=None, reps=2):
        """Time `reps` real steps per candidate; keep the fastest."""
        if candidates is None:
            candidates = [{"schedule": s, "quantile": q, "big_grid": g}
                          for s in (0, 1, 5) for q in (0.75, 0.9, 0.99) for g in (0, 1024, 8192)]
        stream = torch.cuda.current_stream()
        best, best_ms = None, float("inf")
        self.tuning = []
        for cand in candidates:
            self.config = dict(cand)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                self.eager_step()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            self.tuning.append((dict(cand), ms))
            if ms < best_ms:
                best, best_ms = dict(cand), ms
        self.config = best
        return best, best_ms

    def capture(self, k):
        """HIP graph of k steps of every run with the current configuration;
        the LDS plan is fixed at capture (cells that outgrow it are re-planned
        inside the same launch sequence, so results do not change)."""
        c = self.config
        hint = self._hint()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            for _ in range(k):
                self.bat.step(0, self.flags, schedule=c["schedule"], d_step=self.d_step,
                              e_hint=hint, big_grid=c["big_grid"], record_stats=False)
                self.d_step.add_(1)
        torch.cuda.current_stream().wait_stream(side)
        self.graph, self.graph_k = g, k
        return g

    def replay(self):
        self.graph.replay()
        self.steps_done += self.graph_k

    def run(self, nsteps, k=10):
        """Advance every run by nsteps: eager until a graph exists, then
        replays of k-step graphs, eager for the remainder."""
        done = 0
        if self.graph is None or self.graph_k != k:
            if nsteps >= k:
                self.capture(k)
        while self.graph is not None and nsteps - done >= self.graph_k:
            self.replay()
            done += self.graph_k
        while done < nsteps:
            self.eager_step()
            done += 1

    def status(self):
        return self.bat.status()


def sequential(ctx: RT.Context, runs, nsteps, capacity=(7, 16), flags=B.XP_ALL, keep=False,
               per_run=None, on_run=None):
    """Every run alone in its own batch, stepped eagerly one after another.
    Returns (seconds spent stepping, seconds including each run's set-up,
    list of batches if keep); per_run (a list) receives each run's stepping
    seconds in order; on_run(index, seconds) is called after each run."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stepping = 0.0
    kept = []
    for spec, parts in runs:
        bat = RT.Batch(ctx, [(spec, parts)], capacity=capacity)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for s in range(nsteps):
            bat.step(s, flags)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        stepping += dt
        if per_run is not None:
            per_run.append(dt)
        if on_run is not None:
            on_run(len(per_run) - 1 if per_run is not None else -1, dt)
        if keep:
            kept.append(bat)
        else:
            del bat
    return stepping, time.perf_counter() - t0, kept
