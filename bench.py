"""Throughput of the per-cell Monte-Carlo collision / ionization step on one MI355X.

Workload: 2D uniform solid-Al target, 512 x 512 PIC cells x (64 electrons +
64 Al3+ ions) = 33.5 M particles, FP64, Ecker-Kroll continuum lowering,
dt = 0.05 fs, photoionization by a uniform 1.7e17 W/cm^2, 1.85 keV flux fused
into every step (synthetic inputs, seeded).

A step is one pass of the whole hot path over every cell: moments and
continuum lowering, e-e and e-i binary collisions, collisional ionization,
three-body recombination, K-vacancy decay and photoionization, with appends
and removals, through `collide_ionize_step` (the slabs were filled by
`bin_particles` before the timed region, outside the step).

Prints one JSON line: binary collisions per second (whole job), the roofline
of the step kernel (algorithmic HBM bytes / its average duration from HIP
events on its stream), and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
E_BYTES = 52      # electron per step: v read + write (48 B), weight read (4 B)
I_BYTES = 52      # ion per step: v read + write (48 B), Z and k read + write (4 B)
NEW_BYTES = 44    # appended electron: x, y, v (40 B) and weight (4 B) written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_threads():
    """Threads the oracle may use: OMP_NUM_THREADS when set (the host's share),
    else the visible cores."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    n = int(env) if env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    return max(1, min(n, os.cpu_count() or n))


def cpu_baseline(spec, parts, budget_s=15.0, max_steps=40, therm=False, ion_z=False, nanbu=False,
                 rel=False, rec_xs=False, photo_frac=False, single=True):
    """The oracle on a bounded sample of the same workload: every cell of the
    same initial state, stepped from step 0 until about budget_s of work on the
    host's threads; then (single) step 0 again on one thread."""
    from oracle import oracle as O
    from paper_1704_01202_amd import workloads as W
    tab = W.make_tables()
    sim = O.Sim(tab, spec)
    sim.bin(parts)
    threads = cpu_threads()
    coll = 0
    steps = 0
    t0 = time.perf_counter()
    flags = (O.ALL | (O.THERM if therm else 0) | (O.ION_Z if ion_z else 0) | (O.NANBU if nanbu else 0)
             | (O.REL if rel else 0) | (O.REC_XS if rec_xs else 0) | (O.PHOTO_FRAC if photo_frac else 0))
    while steps < max_steps:
        sim.step(steps, flags, threads)
        cnt, _ = sim.counters()
        coll += int(cnt[:, 0].sum() + cnt[:, 1].sum() + cnt[:, 2].sum())
        steps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    out = {"value": coll / dt, "unit": "collisions/s", "cores": threads, "kind": "oracle",
           "sample": "all %d cells of the same workload, steps 0-%d (%d collisions) in %.1f s"
                     % (spec.ncells, steps - 1, coll, dt)}
    if single and threads > 1:
        # one host thread on the first step of the same state, for scale
        del sim
        sim = O.Sim(tab, spec)
        sim.bin(parts)
        t1 = time.perf_counter()
        sim.step(0, flags, 1)
        d1 = time.perf_counter() - t1
        cnt, _ = sim.counters()
        c1 = int(cnt[:, 0].sum() + cnt[:, 1].sum() + cnt[:, 2].sum())
        out["single_thread_value"] = c1 / d1
        out["single_thread_sample"] = "step 0 of all %d cells on 1 thread (%d collisions) in %.1f s" \
            % (spec.ncells, c1, d1)
    return out


def source_digest():
    """sha256 over the device sources and build flags: counter figures taken
    from a profile are only valid for the kernel they were taken on."""
    import hashlib
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1704_01202_amd")
    files = [os.path.join(ROOT, "include", "xpic.h"), os.path.join(pkg, "build.py")]
    csrc = os.path.join(pkg, "csrc")
    files += [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))
              if f.endswith((".hip", ".h"))]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_step_c2_512x512_hbm_traffic.md")


def measured_traffic():
    """HBM bytes per k_step launch from the committed FETCH_SIZE / WRITE_SIZE
    summary (already scaled by the copy-kernel calibration), or None when the
    summary is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"^source_digest:\s*(\w+)", text, re.M)
    b = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m or not b or m.group(1) != source_digest():
        return None
    return float(b.group(1))


SQ_PROFILE = os.path.join(ROOT, "profiles", "k_step_c2_512x512_sq_counters.md")
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per 4 cycles
VALU_PEAK = 256 * 4 * 2.4e9 / 4


def measured_valu():
    """VALU wave-instructions per tier-0 k_step launch from the committed SQ
    counter summary, or None when it is missing or was taken on other sources."""
    try:
        with open(SQ_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"^source_digest:\s*(\w+)", text, re.M)
    b = re.search(r"^valu_insts_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not m or not b or m.group(1) != source_digest():
        return None
    return float(b.group(1))


def copy_reference(mib):
    """A plain device-to-device copy of known size (mib MiB read, mib MiB
    written), three times: the reference the HBM counters are scaled by."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy reference: 3 x %d MiB device copies" % mib)


def measure_scan(nruns=256, run_steps=500, seq=True, k=5):
    """Batched scan of the C4 runs at their full length: every run stepped
    run_steps times in one batch (two eager steps, then graph replays of k
    steps), autotuned knobs, against a sequential plain loop over the same runs
    for the same steps.  No extrapolation: both legs step every run run_steps
    times.  Returns a dict of the measurements."""
    import numpy as np
    import torch
    from paper_1704_01202_amd import runtime as RT
    from paper_1704_01202_amd import scan as SC
    from paper_1704_01202_amd import workloads as W

    t0 = time.perf_counter()
    tab = W.make_tables()
    runs = W.config_c4_runs(nruns=nruns, nsteps=run_steps)
    n_part = sum(p.ne + p.ni for _, p in runs)
    log("scan generated (%.1f s): %d runs, %d particles" % (time.perf_counter() - t0, len(runs), n_part))
    ctx = RT.Context(tab)
    # slabs for any state the runs can reach: weight units are conserved with
    # the charge (sum w_e = sum Z <= 13 units per ion) and every electron holds
    # at least one unit, so n_e + 12 n_i + 16 slots (n_e = n_i here) never overflow
    cap = (12, 16)
    # autotune on a throw-away copy: the knobs change speed, never results
    tuner = SC.Scan(ctx, runs, capacity=cap)
    for _ in range(2):
        tuner.eager_step()
    best, best_ms = tuner.autotune(reps=1)
    log("autotuned on steps 2-%d: %s (%.3f ms/step)" % (tuner.steps_done - 1, best, best_ms))
    del tuner
    torch.cuda.empty_cache()
    sc = SC.Scan(ctx, runs, capacity=cap)
    sc.config = dict(best)
    torch.cuda.synchronize()
    log("batched: %d cells, e_slots %d, global-path cells %d (%.1f s)"
        % (sc.bat.n_cells, sc.bat.e_slots, sc.bat.big_cells_max, time.perf_counter() - t0))
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    reps = max(0, (run_steps - 2) // k)
    tail = run_steps - 2 - reps * k
    marks = [ev() for _ in range(reps + 1)]
    e0, e1 = ev(), ev()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    sc.eager_step()
    sc.eager_step()
    if reps:
        sc.capture(k)
    marks[0].record(stream)
    for q in range(reps):
        sc.replay()
        marks[q + 1].record(stream)
        if (q + 1) % 20 == 0:
            # a progress line every 100 steps (the wait adds no GPU work)
            torch.cuda.synchronize()
            log("batched: %d of %d steps, %.1f s" % (2 + (q + 1) * k, run_steps, time.perf_counter() - w0))
    for _ in range(tail):
        sc.eager_step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    assert sc.steps_done == run_steps
    ms_step = e0.elapsed_time(e1) / run_steps
    step_ms = np.array([marks[q].elapsed_time(marks[q + 1]) / k for q in range(reps)]) if reps \
        else np.array([ms_step])
    cnt = sc.bat.run_counters().sum(axis=0)
    coll = int(cnt[0] + cnt[1] + cnt[2])
    status = sc.status()
    run_status = sc.bat.run_status()
    rph = len(runs) * 3600.0 / wall
    log("batched: %d steps of %d runs in %.2f s (%.3f ms/step), status %d"
        % (run_steps, len(runs), wall, ms_step, status))
    del sc
    torch.cuda.empty_cache()
    out = {
        "workload": "%d independent 0D runs, 1e4-2e6 particles log-uniform, 1e16-1e18 W/cm^2, "
                    "1.55-1.9 keV, SP/EK alternating, dt 0.1 fs, %d steps per run, one batch, "
                    "HIP-graph replays of %d steps" % (len(runs), run_steps, k),
        "runs": len(runs), "steps_per_run": run_steps, "particles": n_part,
        "autotuned": best, "wall_s": wall, "ms_per_step": ms_step,
        "runs_per_hour": rph, "collisions_per_s": coll / wall,
        # every run of the batch completes with its last step
        "time_to_result_s": {"p50": wall, "p99": wall},
        "step_latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                            "p99": float(np.percentile(step_ms, 99))},
        "status": status, "runs_flagged": int((run_status != 0).sum()),
    }
    if seq:
        per_run = []
        def one(i, dt):
            if i % 16 == 15:
                log("sequential: %d of %d runs, %.1f s stepping so far" % (i + 1, len(runs), sum(per_run)))
        stepping, total, _ = SC.sequential(ctx, runs, run_steps, capacity=cap, per_run=per_run,
                                           on_run=one)
        done = np.cumsum(per_run)
        out["sequential"] = {
            "runs_per_hour": len(runs) * 3600.0 / stepping, "stepping_s": stepping,
            "with_setup_s": total,
            "time_to_result_s": {"p50": float(np.percentile(done, 50)),
                                 "p99": float(np.percentile(done, 99))},
        }
        out["vs_sequential"] = rph / out["sequential"]["runs_per_hour"]
        log("sequential: %.2f s stepping (%.2f s with set-up) for %d steps of every run"
            % (stepping, total, run_steps))
    return out


def bench_c4(args):
    """Batched scan as its own JSON line (runs/hour), every run stepped
    --run-steps times in both legs."""
    m = measure_scan(nruns=args.runs, run_steps=args.run_steps, seq=not args.no_seq)
    out = {
        "metric": "runs/hour (batched scan)",
        "value": m["runs_per_hour"],
        "unit": "runs/h",
        "n_gpus": 1,
        "steps": m["steps_per_run"],
        "warmup": 0,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": m["workload"], "particles": m["particles"],
                   "autotuned": m["autotuned"], "status": m["status"]},
        "scan": m,
    }
    print(json.dumps(out), flush=True)


def bench_c3(args):
    """Uneven occupancy: 1024 x 256 cells on a density ramp (4 to ~1024
    particles per cell).  The autotuner picks among one wave per cell, one
    block per cell and the automatic choice (and the quantile of cell sizes the
    first LDS plan covers); the tuned
    configuration is then timed over graph-replayed steps.  One JSON line."""
    import torch
    from paper_1704_01202_amd import runtime as RT
    from paper_1704_01202_amd import scan as SC
    from paper_1704_01202_amd import workloads as W

    t0 = time.perf_counter()
    tab = W.make_tables()
    spec, parts = W.config_c3()
    log("C3 generated (%.1f s): %d electrons, %d ions" % (time.perf_counter() - t0, parts.ne, parts.ni))
    ctx = RT.Context(tab)
    # slabs of n_e + 3 n_i + 16 electron slots: room for the electrons to grow
    # fourfold in the densest cells (a capacity overflow is flagged in the
    # status), and every slab fits one workgroup's LDS, so the global-memory
    # path is never launched
    sc = SC.Scan(ctx, [(spec, parts)], capacity=(3, 16))
    for _ in range(2):
        sc.eager_step()
    cands = [{"schedule": s_, "quantile": q, "big_grid": 0} for s_ in (0, 1, 5)
             for q in (0.5, 0.75, 0.9, 0.99, 1.0)]
    best, best_ms = sc.autotune(cands, reps=2)
    log("autotune: " + ", ".join("%s/%.2f: %.3f ms" % (c["schedule"], c["quantile"], ms) for c, ms in sc.tuning))
    k = 5
    sc.capture(k)
    sc.bat.d_run_cnt.zero_()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    reps = max(1, args.steps // k)
    for _ in range(reps):
        sc.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    timed = reps * k
    cnt = sc.bat.run_counters()[0]
    coll = int(cnt[0] + cnt[1] + cnt[2])
    st = sc.bat.stats()
    out = {
        "metric": "binary collisions/sec",
        "value": coll / wall,
        "unit": "collisions/s",
        "n_gpus": 1,
        "steps": timed,
        "warmup": sc.steps_done - timed,
        "ms_per_step": e0.elapsed_time(e1) / timed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D 1024x256 cells, density ramp 0.01-1x solid (20-cell scale), "
                               "Poisson 4-1024 particles per cell, T_e 5-50 eV per column, EK, dt 0.05 fs",
                   "cells": spec.ncells, "electrons_start": parts.ne, "ions": parts.ni,
                   "autotuned": best, "status": sc.status(),
                   "global_path_cells_last_step": int(st[2])},
        "autotune_ms": [[c["schedule"], c["quantile"], ms] for c, ms in sc.tuning],
    }
    print(json.dumps(out), flush=True)


def bench_c5(args):
    """Served stream: Poisson arrivals of 0D and 1D runs served with continuous
    batching from a resident pool, against a sequential plain loop over the
    same trace.  Prints one JSON line (runs/hour, p50/p99 time-to-result)."""
    import torch
    from paper_1704_01202_amd import runtime as RT
    from paper_1704_01202_amd import serve as SV
    from paper_1704_01202_amd import workloads as W

    t0 = time.perf_counter()
    tab = W.make_tables()
    trace = W.config_c5_trace(n_requests=args.requests, rate=args.rate, size_hi=args.size_hi,
                              steps_lo=args.steps_lo, steps_hi=args.steps_hi)
    n_part = sum(q.parts.ne + q.parts.ni for q in trace)
    n_steps = sum(q.nsteps for q in trace)
    log("trace generated (%.1f s): %d requests, %d particles, %d run-steps"
        % (time.perf_counter() - t0, len(trace), n_part, n_steps))
    ctx = RT.Context(tab)
    # slabs for any reachable state (see measure_scan)
    cap = (12, 16)
    pool = SV.Pool(ctx, budget_bytes=int(args.budget_gb * 2**30), max_cells=1 << 16, max_runs=512,
                   capacity=cap)
    torch.cuda.synchronize()
    log("pool: %d electron slots, %d ion slots, workspace %.1f GB"
        % (pool.E, pool.I, pool.work_bytes / 2**30))
    def served_one(pool_, r, rec):
        log("served request %d (%d steps) done at %.1f s" % (rec["rid"], rec["steps"], rec["done"]))
    recs, waited = SV.serve(pool, trace, k=args.serve_k, on_done=served_one)
    served = SV.latency_summary(recs)
    status = pool.status()
    log("served: %s; peak resident %d, longest queue %d, status %d"
        % (served, pool.peak_active, waited, status))
    peak = pool.peak_active
    coll = sum(int(r["counters"][0] + r["counters"][1] + r["counters"][2]) for r in recs.values())
    del pool
    torch.cuda.empty_cache()
    seq = None
    if not args.no_seq:
        seq_recs = SV.sequential(ctx, trace, capacity=cap, on_done=lambda rec: log(
            "sequential request %d (%d steps) done at %.1f s" % (rec["rid"], rec["steps"], rec["done"])))
        seq = SV.latency_summary(seq_recs)
        seq["status"] = max(r.get("status", 0) for r in seq_recs.values())
        log("sequential: %s" % seq)
    out = {
        "metric": "runs/hour (served stream)",
        "value": served["runs_per_hour"],
        "unit": "runs/h",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%d requests, Poisson %.0f/s, half 0D half 1D (64-4096 cells), "
                               "1e4-%.0e particles, %d-%d steps, 1e16-1e18 W/cm^2, SP/EK"
                               % (len(trace), args.rate, args.size_hi, args.steps_lo, args.steps_hi),
                   "budget_gb": args.budget_gb, "particles": n_part, "status": status},
        "p50_s": served["p50_s"],
        "p99_s": served["p99_s"],
        "collisions_per_s": coll / served["makespan_s"],
        "peak_resident_runs": peak,
        "longest_queue": waited,
        "sequential": seq,
        "vs_sequential": served["runs_per_hour"] / seq["runs_per_hour"] if seq else None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--therm", action="store_true",
                    help="c2: add the forced thermalization variant (Sec. VI.C) after S5")
    ap.add_argument("--ion-z", action="store_true",
                    help="c2: collisional ionization per ion charge state (variant of Sec. IV)")
    ap.add_argument("--nanbu", action="store_true",
                    help="c2: Nanbu's cumulative scattering law in the e-e and e-i collisions")
    ap.add_argument("--rel", action="store_true",
                    help="c2: relativistic binary collisions (centre-of-momentum frame)")
    ap.add_argument("--rec-xs", action="store_true",
                    help="c2: three-body recombination from cross sections by detailed balance")
    ap.add_argument("--photo-frac", action="store_true",
                    help="c2: photo events limited by the bin's photons in the cell (partial photoionization)")
    ap.add_argument("--ka-field", action="store_true",
                    help="c2: K-alpha photons returned to the per-cell photon field (with --transport)")
    ap.add_argument("--transport", action="store_true",
                    help="c2: per-cell photon field rebuilt after every step by the reduced "
                         "radiation transport (transport_photons)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run a plain device copy of MIB MiB "
                         "(calibrates the HBM byte counters under a profiler)")
    ap.add_argument("--workload", choices=("c2", "c3", "c4", "c5"), default="c2",
                    help="c2: the 512x512-cell step (default); c3: uneven occupancy with the "
                         "autotuned schedule; c4: the batched scan; c5: the served stream")
    ap.add_argument("--requests", type=int, default=48, help="c5: requests in the trace")
    ap.add_argument("--rate", type=float, default=20.0, help="c5: arrivals per second")
    ap.add_argument("--size-hi", type=float, default=2e6, help="c5: largest run, particles")
    ap.add_argument("--steps-lo", type=int, default=100, help="c5: fewest steps of a run")
    ap.add_argument("--steps-hi", type=int, default=600, help="c5: most steps of a run")
    ap.add_argument("--budget-gb", type=float, default=200.0,
                    help="c5: pool budget (slabs and workspace), GiB")
    ap.add_argument("--serve-k", type=int, default=8, help="c5: steps between admission checks")
    ap.add_argument("--runs", type=int, default=256, help="c4: runs in the scan")
    ap.add_argument("--run-steps", type=int, default=500, help="c4: steps of every run")
    ap.add_argument("--no-seq", action="store_true", help="c4, c5: skip the sequential leg")
    ap.add_argument("--no-scan", action="store_true",
                    help="c2: leave out the batched-scan measurement (C4 runs at full length)")
    ap.add_argument("--no-full-run", action="store_true",
                    help="c2: leave out the whole configured run (200 steps from the initial state)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the step has no cross-GPU work and only --gpus 1 "
              "is supported (cells and runs are independent within a step; a multi-GPU run "
              "would shard them by cell slab or by run)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        bench_c3(args)
        return
    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload == "c5":
        bench_c5(args)
        return

    import torch
    from paper_1704_01202_amd import binding as B
    from paper_1704_01202_amd import runtime as RT
    from paper_1704_01202_amd import workloads as W

    t0 = time.perf_counter()
    tab = W.make_tables()
    spec, parts = W.config_c2(nx=args.nx, ny=args.ny)
    log("workload generated (%.1f s): %d electrons, %d ions, %d cells"
        % (time.perf_counter() - t0, parts.ne, parts.ni, spec.ncells))
    ctx = RT.Context(tab)
    field = None
    if args.transport:
        import numpy as np
        field = np.tile(np.asarray(spec.photon_n, dtype=np.float64), (spec.ncells, 1))
    bat = RT.Batch(ctx, [(spec, parts)], capacity=(7, 16), cell_nhv=field,
                   kalpha_return=args.ka_field and args.transport)
    torch.cuda.synchronize()
    log("binned into slabs: e_slots %d, max cap %d (%.1f s)"
        % (bat.e_slots, bat.e_cap_max, time.perf_counter() - t0))
    stream = torch.cuda.current_stream()
    flags = (B.XP_ALL | (B.XP_THERM if args.therm else 0) | (B.XP_ION_Z if args.ion_z else 0)
             | (B.XP_NANBU if args.nanbu else 0) | (B.XP_REL if args.rel else 0)
             | (B.XP_REC_XS if args.rec_xs else 0) | (B.XP_PHOTO_FRAC if args.photo_frac else 0)
             | (B.XP_KA_FIELD if args.ka_field else 0))
    for s in range(args.warmup):
        bat.step(s, flags, schedule=args.schedule)
        if args.transport:
            bat.transport()
    torch.cuda.synchronize()
    bat.d_run_cnt.zero_()
    ne_before = int(bat.d_e_cnt.sum().item())
    ni = int(bat.d_i_cnt.sum().item())
    log("warmup done, %d electrons resident" % ne_before)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    ne_steps = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    tev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps if args.transport else 0)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        bat.step(args.warmup + k, flags, schedule=args.schedule)
        ev[k][1].record(stream)
        if args.transport:
            tev[k][0].record(stream)
            bat.transport()
            tev[k][1].record(stream)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    wall = t_end - t_start
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    cnt = bat.run_counters()[0]
    status = bat.status()
    ne_after = int(bat.d_e_cnt.sum().item())
    coll = int(cnt[0] + cnt[1] + cnt[2])
    new_e = int(cnt[21])
    # algorithmic bytes of all timed launches: electrons present at each step
    # start (interpolated between the measured ends) + ions + appended electrons
    e_avg = 0.5 * (ne_before + ne_after)
    bytes_total = args.steps * (E_BYTES * e_avg + I_BYTES * ni) + NEW_BYTES * new_e
    avg_ms = sum(kernel_ms) / len(kernel_ms)
    achieved = bytes_total / args.steps / (avg_ms * 1e-3) / 1e9
    if status != 0:
        log("WARNING: device status %d" % status)
    out = {
        "metric": "binary collisions/sec",
        "value": coll / wall,
        "unit": "collisions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D uniform solid Al, %dx%d cells x (64 e + 64 Al3+), EK IPD, "
                               "dt 0.05 fs, 1.7e17 W/cm^2 1.85 keV photoionization fused%s"
                               % (args.nx, args.ny,
                                  (", forced thermalization after S5" if args.therm else "")
                                  + (", ionization per ion charge state" if args.ion_z else "")
                                  + (", Nanbu scattering law" if args.nanbu else "")
                                  + (", relativistic collisions" if args.rel else "")
                                  + (", recombination from cross sections" if args.rec_xs else "")
                                  + (", photon budget with partial photoionization" if args.photo_frac else "")
                                  + (", K-alpha return to the field" if args.ka_field else "")
                                  + (", reduced radiation transport after every step"
                                     if args.transport else "")),
                   "cells": spec.ncells, "electrons_start": parts.ne, "ions": ni,
                   "electrons_timed": [ne_before, ne_after], "status": status},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_step", "kernel_avg_ms": avg_ms,
                     "bytes_per_launch": bytes_total / args.steps},
        "collisions_total": coll,
    }
    valu = measured_valu()
    plain = not (args.therm or args.ion_z or args.nanbu or args.rel or args.transport or args.rec_xs
                 or args.photo_frac or args.ka_field)
    if valu is not None and args.nx == 512 and args.ny == 512 and plain:
        # the step is bound by instruction issue, not by HBM: VALU instructions
        # of a launch (profiled) over the launch time measured here
        rate = valu / (avg_ms * 1e-3)
        out["valu_issue"] = {"bound": "alu", "achieved": rate, "peak": VALU_PEAK,
                             "unit": "wave-instructions/s", "frac": rate / VALU_PEAK,
                             "insts_per_launch": valu}
    if args.transport:
        # the step's time covers collide_ionize_step; the transport is timed apart
        tr_ms = [a.elapsed_time(b) for a, b in tev]
        out["transport"] = {"kernel": "k_tr_rows + k_tr_sum", "avg_ms": sum(tr_ms) / len(tr_ms),
                            "transmission": float(bat.d_trans[0, 0].item())}
    if args.copy_ref > 0:
        copy_reference(args.copy_ref)
    del bat
    torch.cuda.empty_cache()
    if not args.no_full_run:
        # the whole configured run: a fresh batch from the same initial state,
        # every one of its steps timed by events on the step's stream
        fb = RT.Batch(ctx, [(spec, parts)], capacity=(7, 16), cell_nhv=field)
        torch.cuda.synchronize()
        nfull = int(spec.nsteps)
        fev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(nfull)]
        ne0 = int(fb.d_e_cnt.sum().item())
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for k in range(nfull):
            fev[k][0].record(stream)
            fb.step(k, flags, schedule=args.schedule)
            fev[k][1].record(stream)
            if args.transport:
                fb.transport()
        torch.cuda.synchronize()
        fwall = time.perf_counter() - f0
        fms = [a.elapsed_time(b) for a, b in fev]
        fc = fb.run_counters()[0]
        fcoll = int(fc[0] + fc[1] + fc[2])
        ne1 = int(fb.d_e_cnt.sum().item())
        fbytes = E_BYTES * 0.5 * (ne0 + ne1) * nfull + I_BYTES * ni * nfull + NEW_BYTES * int(fc[21])
        out["full_run"] = {"steps": nfull, "wall_s": fwall, "ms_per_step": fwall * 1e3 / nfull,
                           "collisions_per_s": fcoll / fwall, "collisions": fcoll,
                           "step_kernels_ms": {"first": fms[0], "last": fms[-1],
                                               "mean": sum(fms) / nfull},
                           "hbm_frac": fbytes / (sum(fms) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "electrons": [ne0, ne1], "status": fb.status()}
        log("full run: %d steps in %.3f s, %.3e collisions/s" % (nfull, fwall, fcoll / fwall))
        del fb
        torch.cuda.empty_cache()
    if not args.no_scan:
        out["batched_scan"] = measure_scan()
    if not args.no_cpu:
        log("timing the CPU oracle on a sample ...")
        out["cpu_baseline"] = cpu_baseline(spec, parts, therm=args.therm, ion_z=args.ion_z,
                                           nanbu=args.nanbu, rel=args.rel, rec_xs=args.rec_xs,
                                           photo_frac=args.photo_frac)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
