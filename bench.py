"""Benchmark of the MI355X FDTD hot path.

Headline workload (the large plain + batched form): the synthetic dicot
cross-section at dx = 12.5 nm, 8192 x 16384 cells, at 4 wavelengths (450, 550,
680, 850 nm) x {healthy, diseased} geometries: 8 instances, 1.07e9 cells, in
one context (one launch per step block over all of them), 40000 FP32 steps,
32-cell CPML, compensated (Kahan) monitor sums over the last 20000 steps.  One
bench "step" is one whole run of the path on that batch: reset, all 40000
time steps (field updates, CPML, TF/SF source, running-DFT monitors), then the
spectra of all 8 instances (Bloch projection, tone fit, R/T/A).  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line with the throughput in cell-updates per second, the
roofline of the dominant kernel (HIP-event timed live, on the stream it runs
on), and the FP64 oracle timed on a bounded sample on the host cores.

The oracle's host sample is timed right after the headline.  Extra legs (off
with --no-extras; each starts only if it is expected to end before --deadline-s
of wall time), reported in the same line:
  large_one - one instance of the headline batch run alone (batched vs plain);
  dicot     - the plain form: 4096 x 8192 cells at 25 nm, lambda = 550 nm,
              20000 steps, whole runs, with its own bulk-kernel roofline;
  batched   - 61 wavelengths (400-1000 nm) x {healthy, diseased} of one
              24 x 48 um domain, each at dx = lambda/(20 n_max), so grid sizes
              are uneven (732 x 1465 to 2048 x 4096); 20000 steps; one context
              (one launch per step block over all instances), also replayed as
              one captured HIP graph, against the same instances run one
              context at a time;
  adjoint   - the 1024 x 2048 monocot at 20 nm, 8000 steps: recorded forward
              (checkpoints every ~sqrt(T) steps) and the discrete adjoint for
              dR/d(n,k) and dR/d eps_r per pixel, against the plain forward;
              with GPU central differences (h = 1e-4) of R in every label's
              n and k beside the adjoint's gradient;
  te        - the dicot workload in TEz (P polarisation): throughput and
              spectra, and the unpolarised R, T, A (mean of TMz and TEz);
  broadband - the batched leg's two geometries as two pulsed broadband runs;
  sweep     - a sample of the paper-scale sweep (5 slices x 2 polarisations)
              at the paper's 55000 steps per run.
The roofline object also carries the bandwidth of a 4 GiB device copy
measured in the same process, as a second, attainable denominator.

Profiling helpers (not part of the default run):
  --leg te|adjoint|broadband|dicot  run that extra leg alone and print its JSON;
  --profile-pass      a short run of a bulk kernel followed by a copy of known
                      size, for rocprofv3 counter collection (workload by
                      --profile-workload: large (the headline batch), dicot,
                      broadband; with --profile-pol 1 the dicot in TEz);
  --derive-traffic F W  turn two rocprofv3 --pmc result databases (FETCH_SIZE,
                      WRITE_SIZE) of --profile-pass into profiles/traffic.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_LAUNCH = 25   # Ez, Hx, Hy read + written (FP32) and one uint8 label, per launch
COPY_BYTES = 1 << 30         # size of the reference copy for counter scaling
LARGE_NAME = "large_dicot8192x16384_x8"   # the headline batch, in profiles/traffic.json


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash(workload: str = "") -> str:
    """Hash of the sources of the kernels a workload's counters measure: the
    monochromatic kernels (fdtd_device.h, fdtd_kernels.hip) and, for broadband
    workloads, fdtd_broadband.hip as well."""
    h = hashlib.sha256()
    files = ["fdtd_device.h", "fdtd_kernels.hip"]
    if workload.startswith("broadband"):
        files.append("fdtd_broadband.hip")
    for f in files:
        with open(os.path.join(ROOT, "paper_2512_17132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def broadband_launch_bytes(insts, lean_cells: int) -> int:
    """Algorithmic HBM bytes of one launch of a broadband bulk kernel over
    lean_cells owned cells: the fields and the label (25 B per cell) and the
    states of driven poles only (those whose label's oscillator strength is
    non-zero; 8 B read and 8 B written per pole): TMz, each cell's own; TEz,
    for each of its Ex and Ey edges the cell's and, where the cell across the
    edge (below for Ex, to the left for Ey) carries another label, that
    cell's.  The items that own the absorbing layers, the source and the
    monitor rows lie in air in the leaves measured here, so every driven pole
    sits in a bulk cell."""
    total = 25 * int(lean_cells)
    for b in insts:
        drv = np.array([sum(1 for p in range(b.n_poles) if b.model[L, 2 + 3 * p] != 0.0)
                        for L in range(b.model.shape[0])])
        lab = b.labels
        n = drv[lab]
        if getattr(b, "polarization", 0):
            below = np.vstack([lab[:1], lab[:-1]])
            left = np.roll(lab, 1, axis=1)
            n = 2 * n + np.where(below != lab, drv[below], 0) + np.where(left != lab, drv[left], 0)
        total += 16 * int(n.sum())
    return total


def broadband_te_launch_bytes(inst) -> int:
    """Algorithmic HBM bytes of one launch of the broadband TEz streaming
    kernel, whose launch holds the instance's special items beside its lean
    ones: broadband_launch_bytes over every cell, plus the absorbing layers'
    two CPML states per cell (8 B read and 8 B written)."""
    cells = inst.nx * inst.ny
    return broadband_launch_bytes([inst], cells) + 16 * 2 * inst.n_pml * inst.nx


def shape_key(K: int, B: int, W: int = 64) -> str:
    """Key of a launch shape in profiles/traffic.json: steps per launch, band
    rows, and the bulk TMz items' columns when they are a workgroup's."""
    return "K%d_B%d" % (K, B) + ("_W%d" % W if W and W != 64 else "")


def bulk_kernel_name(K: int, W: int = 64) -> str:
    """The TMz bulk kernel of launch shape (K, W)."""
    return "k_tblock_wg<%d,false>" % K if W == 256 else "k_tblock<%d,false,false>" % K


def traffic_record(workload: str, K: int, B: int, W: int = 64):
    """HBM bytes per launch of the dominant kernel at launch shape (K, B, W)
    from committed rocprofv3 counter summaries, or None if absent or taken on a
    different kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload, {}).get(shape_key(K, B, W))
    except Exception:
        return None
    if not rec or rec.get("kernel_hash") != kernel_source_hash(workload):
        return None
    return rec.get("bytes_per_launch")


def run_oracle_sample(inst, n_begin: int, n_end: int, threads: int = 0):
    """The oracle on steps [n_begin, n_end) of inst from a zero state, with the
    instance's own monitor window (steps from n_steps - n_steps/2 enter the
    monitor sums): (cell-updates/s, seconds, threads used).  threads = 0: the
    oracle's default (all host threads)."""
    import oracle as O
    if threads:
        O.set_num_threads(threads)
    prob = O.Problem(nx=inst.nx, ny=inst.ny, h=inst.dx, lambda0=inst.lambda0, n_steps=inst.n_steps,
                     n_pml=inst.n_pml, j_src=inst.j_src, j_ref=inst.j_ref, j_trn=inst.j_trn,
                     courant=inst.courant, ramp_periods=inst.ramp_periods)
    ce, cb = O.pixel_coefficients(prob, inst.labels, inst.nk)
    e_inc, h_inc = O.incident(prob)
    t0 = time.perf_counter()
    O.run(prob, ce, cb, e_inc, h_inc, n_begin=n_begin, n_end=n_end)
    dt = time.perf_counter() - t0
    return inst.cells * (n_end - n_begin) / dt, dt, O.num_threads()


def host_cpu():
    """CPU model and the counts of logical CPUs (os.cpu_count) and of CPUs this
    process may run on (nproc)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc, "logical_cpus": os.cpu_count()}


def copy_bandwidth_gbs(nbytes: int = 4 << 30, reps: int = 5) -> float:
    """Attainable HBM bandwidth: a device-to-device copy of nbytes, best of
    reps, counting the bytes read plus the bytes written."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / best / 1e9


def batched_instances(steps: int):
    """The 122 batched instances, rasterised in parallel on the host."""
    import leafgen as LG
    return LG.configs.batched_config_parallel(steps, workers=min(16, os.cpu_count() or 1))


# The bulk kernel's launch duration is measured with HIP events on every
# PROFILE_EVERY-th launch of the timed region: each event pair adds marker
# packets to the stream, which cost 2-4 % of the step time when every launch
# is bracketed.
PROFILE_EVERY = 8


def timed_runs(sim, n_runs: int):
    """Whole runs (reset, all steps, spectra), wall time and bulk-kernel time
    (summed over the timed launches, and their count)."""
    import torch
    torch.cuda.synchronize()
    sim.set_profiling(True, every=PROFILE_EVERY)
    t0 = time.perf_counter()
    for k in range(n_runs):
        if k:
            sim.reset()
        sim.run()
        out = sim.spectra()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = sim.kernel_time()
    sim.set_profiling(False)
    return wall, kms, launches, out


def leg_batched(insts, steps: int):
    import torch
    from paper_2512_17132_amd import fdtd
    cells = sum(i.cells for i in insts)
    sim = fdtd.Simulation(insts, fdtd.Options(n_steps=steps, use_graph=0))
    sim.autotune()
    cfg = sim.config()
    sim.run()
    R, T, A = sim.spectra()
    sim.reset()
    wall, kms, launches, _ = timed_runs(sim, 1)
    sim.close()
    batched_rate = cells * steps / wall
    log("batched: %.2f s -> %.1f Gcell/s (K=%d, band %d)" % (wall, batched_rate / 1e9, cfg["t_block"], cfg["band_rows"]))
    # the same run replayed from a captured HIP graph (no timing events: the
    # whole run is one graph launch)
    gsim = fdtd.Simulation(insts, fdtd.Options(n_steps=steps, use_graph=1))
    gsim.autotune()
    gsim.run()                      # captures the graph
    gsim.spectra()
    gsim.reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gsim.run()
    gsim.spectra()
    torch.cuda.synchronize()
    graph_wall = time.perf_counter() - t1
    gcfg = gsim.config()
    gsim.close()
    log("batched, graph replay: %.2f s -> %.1f Gcell/s (K=%d, band %d)"
        % (graph_wall, cells * steps / graph_wall / 1e9, gcfg["t_block"], gcfg["band_rows"]))
    # the same instances, one context at a time
    t_plain = 0.0
    for inst in insts:
        s = fdtd.Simulation([inst], fdtd.Options(n_steps=steps, t_block=cfg["t_block"], band_rows=cfg["band_rows"],
                                                 special_rows=cfg["special_rows"], use_graph=0))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.run()
        s.spectra()
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t1
        s.close()
    plain_rate = cells * steps / t_plain
    log("one at a time: %.2f s -> %.1f Gcell/s" % (t_plain, plain_rate / 1e9))
    return {"workload": "61 wavelengths 400-1000 nm x {healthy, diseased}, 24.09 x 48.19 um at dx = lambda/(20 n_max), "
                        "%d steps, %d instances, %d cells" % (steps, len(insts), cells),
            "value": batched_rate / 1e9, "unit": "Gcell-updates/s", "seconds": wall,
            "graph_replay": cells * steps / graph_wall / 1e9, "graph_replay_seconds": graph_wall,
            "one_at_a_time": plain_rate / 1e9, "one_at_a_time_seconds": t_plain,
            "speedup": batched_rate / plain_rate, "t_block": cfg["t_block"], "band_rows": cfg["band_rows"],
            "R_400nm_healthy": float(R[0]), "T_400nm_healthy": float(T[0])}


def leg_te(inst, tm_rta, use_graph: int = 0, shape=(10, 192)):
    """The dicot in TEz, one whole timed run after a warm-up.  use_graph = 1
    replays the run from its captured graph at the fixed launch shape `shape`
    (no autotuning, no kernel timing: both would switch replay off), for
    comparing graph replay with direct launches."""
    import copy
    import torch
    from paper_2512_17132_amd import fdtd
    te = copy.copy(inst)
    te.polarization = 1
    if use_graph:
        sim = fdtd.Simulation([te], fdtd.Options(n_steps=te.n_steps, use_graph=1, t_block=shape[0], band_rows=shape[1]))
        sim.run()
        sim.spectra()
        sim.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run()
        R, T, A = sim.spectra()
        torch.cuda.synchronize()
        wall, kms, launches = time.perf_counter() - t0, 0.0, 0
    else:
        sim = fdtd.Simulation([te], fdtd.Options(n_steps=te.n_steps, use_graph=0))
        sim.autotune()
        sim.run()
        sim.spectra()
        sim.reset()
        wall, kms, launches, (R, T, A) = timed_runs(sim, 1)
    cfg = sim.config()
    sim.close()
    rate = te.cells * te.n_steps / wall
    log("TEz: %.3f s -> %.1f Gcell/s (K=%d, band %d); R %.5f T %.5f A %.5f"
        % (wall, rate / 1e9, cfg["t_block"], cfg["band_rows"], R[0], T[0], A[0]))
    launch_s = kms * 1e-3 / max(1, launches)
    achieved = BYTES_PER_CELL_LAUNCH * cfg["lean_cells"] / launch_s / 1e9 if launch_s > 0 else None
    # the committed counters describe the one-wave TEz bulk kernel; a record
    # under the workgroup layout's key would describe that kernel
    traffic = traffic_record(inst.name + "_te", cfg["t_block"], cfg["band_rows"], cfg["bulk_columns"])
    out = {"workload": "the dicot workload in TEz (P polarisation, Hz/Ex/Ey, edge-averaged materials)%s"
                       % (", replayed from its captured graph" if use_graph else ""),
           "value": rate / 1e9, "unit": "Gcell-updates/s", "seconds": wall, "t_block": cfg["t_block"],
           "band_rows": cfg["band_rows"], "bulk_columns": cfg["bulk_columns"],
           "bulk_kernel_avg_launch_ms": kms / max(1, launches),
           "bulk_kernel_hbm_gbs": achieved,
           "bulk_kernel_hbm_frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
           "bulk_kernel_traffic_bytes": traffic,
           "R": float(R[0]), "T": float(T[0]), "A": float(A[0])}
    if tm_rta is not None:
        Ru, Tu, Au = fdtd.unpolarized(tm_rta, (R, T, A))
        log("unpolarised R %.5f T %.5f A %.5f" % (Ru[0], Tu[0], Au[0]))
        out["unpolarized"] = {"R": float(Ru[0]), "T": float(Tu[0]), "A": float(Au[0])}
    return out


def leg_large_one(inst):
    """One instance of the headline batch in a context of its own, one whole
    run after a warm-up run (the plain side of batched vs plain)."""
    import torch
    from paper_2512_17132_amd import fdtd
    s = fdtd.Simulation([inst], fdtd.Options(n_steps=inst.n_steps, use_graph=0))
    s.autotune()
    cfg = s.config()
    s.step(cfg["t_block"])
    s.reset()
    wall, kms, launches, (R, T, A) = timed_runs(s, 1)
    s.close()
    rate = inst.cells * inst.n_steps / wall
    log("large, one instance alone (%s): %.2f s -> %.1f Gcell/s (K=%d, band %d, bulk items of %d columns)"
        % (inst.name, wall, rate / 1e9, cfg["t_block"], cfg["band_rows"], cfg["bulk_columns"]))
    return {"workload": "one instance of the headline batch (%s, %d x %d cells, %d steps) in a context of its own"
                        % (inst.name, inst.nx, inst.ny, inst.n_steps),
            "value": rate / 1e9, "unit": "Gcell-updates/s", "seconds": wall, "t_block": cfg["t_block"],
            "bulk_columns": cfg["bulk_columns"],
            "band_rows": cfg["band_rows"], "R": float(R[0]), "T": float(T[0])}


def leg_dicot(inst, n_runs: int = 3):
    """The plain form: the 4096 x 8192 dicot, whole runs (reset, 20000 steps,
    spectra) after a warm-up run, with the bulk kernel's roofline."""
    from paper_2512_17132_amd import fdtd
    sim = fdtd.Simulation([inst], fdtd.Options(n_steps=inst.n_steps, use_graph=0))
    sim.autotune()
    sim.run()
    sim.spectra()
    sim.reset()
    wall, kms, launches, (R, T, A) = timed_runs(sim, n_runs)
    cfg = sim.config()
    sim.close()
    rate = inst.cells * inst.n_steps * n_runs / wall
    K, B, W = cfg["t_block"], cfg["band_rows"], cfg["bulk_columns"]
    avg_s = kms * 1e-3 / max(1, launches)
    achieved = BYTES_PER_CELL_LAUNCH * cfg["lean_cells"] / avg_s / 1e9
    log("dicot: %d runs in %.3f s -> %.1f Gcell/s (K=%d, band %d, bulk items of %d columns); bulk kernel %.3f ms, "
        "%.0f GB/s" % (n_runs, wall, rate / 1e9, K, B, W, avg_s * 1e3, achieved))
    return {"workload": "synthetic dicot cross-section, plain method: %d x %d cells, dx = 25 nm, lambda = 550 nm, "
                        "%d FP32 steps, 32-cell CPML; %d whole runs" % (inst.nx, inst.ny, inst.n_steps, n_runs),
            "value": rate / 1e9, "unit": "Gcell-updates/s", "seconds": wall, "t_block": K, "band_rows": B,
            "bulk_columns": W, "bulk_kernel": bulk_kernel_name(K, W), "bulk_kernel_avg_launch_ms": avg_s * 1e3,
            "bulk_kernel_algorithmic_bytes_per_launch": BYTES_PER_CELL_LAUNCH * cfg["lean_cells"],
            "bulk_kernel_hbm_gbs": achieved, "bulk_kernel_hbm_frac": achieved / HBM_PEAK_GBS,
            "bulk_kernel_traffic_bytes": traffic_record(inst.name, K, B, W),
            "R": float(R[0]), "T": float(T[0]), "A": float(A[0])}


PAPER_SWEEP_LAMS_NM = list(range(400, 2501, 10))   # 211 wavelengths
PAPER_SWEEP_STEPS = 55000


def leg_sweep(labels, lams_nm=(550, 1450), steps: int = 55000):
    """A bounded sample of the paper-scale sweep: the 8511 x 6689 dicot grid
    cut into 5 periodic slices, 2 polarisations, two wavelengths, each run at
    the paper's 55000 steps; timed whole (context set-up, tuning, run,
    spectra), its spectrum averaged over slices and polarisations by the
    library, and extrapolated to 211 wavelengths: the running time at the
    sample's running rate, plus set-up and tuning for the full sweep's runs
    and contexts at the sample's cost per run and per context."""
    import leafgen as LG
    from paper_2512_17132_amd import sweep as SW
    g = LG.configs.PAPER_DICOT_GRID
    j_src, j_ref, j_trn = LG.configs.rows(g["ny"], g["n_pml"])
    runs = SW.plan(labels, LG.materials.dicot_nk, [l * 1e-9 for l in lams_nm], g["dx_nm"] * 1e-9, g["n_pml"],
                   j_src, j_ref, j_trn, steps, n_slices=5)
    res = SW.run_sweep(runs)
    rate = res.cell_updates / res.seconds
    run_rate = res.cell_updates / res.run_seconds
    slice_cells = sum(r.cells for r in runs) / len(runs)
    full = len(PAPER_SWEEP_LAMS_NM) * 2 * 5 * slice_cells * PAPER_SWEEP_STEPS
    # the full sweep's contexts under the same memory budget: its running time
    # at the sample's running rate, plus the sample's set-up time per run, plus
    # tuning of the first context.  The tuner's trials run a fixed number of
    # steps on contexts this large, so its time grows with the context's cells.
    import torch
    free, _ = torch.cuda.mem_get_info()
    full_runs = SW.plan(labels, LG.materials.dicot_nk, [l * 1e-9 for l in PAPER_SWEEP_LAMS_NM], g["dx_nm"] * 1e-9,
                        g["n_pml"], j_src, j_ref, j_trn, PAPER_SWEEP_STEPS, n_slices=5)
    full_batches = SW.pack(full_runs, int(0.6 * free))
    full_contexts = len(full_batches)
    sample_cells = sum(r.cells for r in runs)
    first_cells = sum(full_runs[i].cells for i in full_batches[0])
    overhead = len(full_runs) * res.setup_seconds / len(runs) + res.tune_seconds * first_cells / sample_cells
    full_seconds = full / run_rate + overhead
    lam, R, T, A = res.spectrum()
    lam_te, R_te, T_te, _ = res.spectrum([1])
    lam_tm, R_tm, T_tm, _ = res.spectrum([0])
    log("sweep spectrum (slice and polarisation mean): " + ", ".join(
        "%d nm R %.4f T %.4f A %.4f" % (round(l * 1e9), r, t, a) for l, r, t, a in zip(lam, R, T, A)))
    log("sweep: %d runs in %d context(s): %.2f s (set-up %.2f, tuning %.2f, run %.2f) -> %.1f Gcell/s whole, "
        "%.1f running; full paper sweep (%d runs in %d contexts) ~%.0f s" % (
            len(runs), len(res.batches), res.seconds, res.setup_seconds, res.tune_seconds, res.run_seconds,
            rate / 1e9, run_rate / 1e9, len(full_runs), full_contexts, full_seconds))
    return {"workload": "paper-scale dicot, 8511 x 6689 cells at 23.41 nm cut into 5 periodic slices, "
                        "%s nm x 2 polarisations, %d of the paper's %d steps" % (list(lams_nm), steps,
                                                                                PAPER_SWEEP_STEPS),
            "runs": len(runs), "contexts": len(res.batches), "cell_updates": res.cell_updates,
            "value": rate / 1e9, "unit": "Gcell-updates/s", "seconds": res.seconds,
            "setup_seconds": res.setup_seconds, "tune_seconds": res.tune_seconds, "run_seconds": res.run_seconds,
            "running_rate": run_rate / 1e9,
            "full_sweep_cell_updates": full, "full_sweep_runs": len(full_runs), "full_sweep_contexts": full_contexts,
            "full_sweep_overhead_seconds": overhead, "full_sweep_seconds_extrapolated": full_seconds,
            "spectrum": {"lambda_nm": [round(l * 1e9) for l in lam], "R": R.tolist(), "T": T.tolist(),
                         "A": A.tolist(), "R_TMz": R_tm.tolist(), "T_TMz": T_tm.tolist(), "R_TEz": R_te.tolist(),
                         "T_TEz": T_te.tolist()},
            "per_run": {"slice": [r.slice for r in runs], "lambda_nm": [round(r.lambda0 * 1e9) for r in runs],
                        "polarization": [r.polarization for r in runs], "R": res.R.tolist(), "T": res.T.tolist()}}


CONV_LAMS_NM = [400, 430, 460, 500, 550, 600, 660, 700, 750, 800, 900, 1000]
CONV_TOL = 0.01


def leg_broadband(batched_seconds=None, steps: int = 20000, cw_sample=(0, 12, 26, 40, 60), conv_steps: int = 80000):
    """Broadband runs of the batched leg's two geometries (healthy and diseased
    24.09 x 48.19 um dicot, each at the grid of its shortest wavelength, with
    the Lorentz-Drude stand-in materials), one pulsed run each with monitors at
    the 61 wavelengths 400-1000 nm, in one context.  Compared with (a) the
    batched leg's 122 monochromatic runs (same wavelengths and geometries,
    tabulated materials, coarser grids at longer wavelengths) and (b)
    monochromatic runs of the healthy broadband grid and materials at a
    sample of wavelengths, batched in one context, for the agreement: at
    20000 steps neither kind of run has converged in the weakly absorbing
    near infrared (they differ by up to about 0.03), so the agreement is also
    measured at conv_steps = 80000 steps on 12 wavelengths, where it is
    stated against a tolerance of 0.01."""
    import torch
    import leafgen as LG
    from paper_2512_17132_amd import fdtd
    bbs = [LG.configs.broadband_leaf(steps=steps, geometry=g) for g in ("healthy", "diseased")]
    nf = len(bbs[0].lambdas)
    cells = sum(b.cells for b in bbs)
    sim = fdtd.Simulation(bbs, fdtd.Options(n_steps=steps, use_graph=0))
    sim.autotune()
    cfg = sim.config()
    sim.step(cfg["t_block"])
    sim.reset()
    torch.cuda.synchronize()
    sim.set_profiling(True, every=PROFILE_EVERY)
    t0 = time.perf_counter()
    sim.run()
    spec = [sim.broadband_spectra(k) for k in range(len(bbs))]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = sim.kernel_time()
    sim.close()
    rate = cells * steps / wall
    # fields, label and driven pole states, read and written once per launch
    bytes_per_cell = broadband_launch_bytes(bbs, cfg["lean_cells"]) / cfg["lean_cells"]
    achieved = bytes_per_cell * cfg["lean_cells"] / (kms * 1e-3 / max(1, launches)) / 1e9
    bb = bbs[0]
    cws = [LG.configs.Instance(bb.labels, LG.materials.model_nk(bb.model, bb.lambdas[f]), bb.dx, bb.lambdas[f],
                               bb.n_pml, steps, name="cw%d" % f) for f in cw_sample]
    s = fdtd.Simulation(cws, fdtd.Options(n_steps=steps, use_graph=0))
    s.autotune()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run()
    Rc, Tc, _ = s.spectra()
    torch.cuda.synchronize()
    wall_cw = time.perf_counter() - t0
    s.close()
    R, T, _ = spec[0]
    dR = max(abs(R[f] - Rc[k]) for k, f in enumerate(cw_sample))
    dT = max(abs(T[f] - Tc[k]) for k, f in enumerate(cw_sample))
    # agreement at a run length where both have converged: the healthy leaf
    # broadband and monochromatic at 12 wavelengths, conv_steps steps each
    # (both kinds of run cost the same per step at any length, so the
    # speed-up measured above holds there too)
    bbc = LG.configs.broadband_leaf(steps=conv_steps, geometry="healthy")
    lam_nm = list(np.round(bbc.lambdas * 1e9).astype(int))
    conv_idx = [lam_nm.index(l) for l in CONV_LAMS_NM]
    s = fdtd.Simulation([bbc], fdtd.Options(n_steps=conv_steps))
    t0 = time.perf_counter()
    s.run()
    Rbc, Tbc, _ = s.broadband_spectra(0)
    torch.cuda.synchronize()
    conv_bb_s = time.perf_counter() - t0
    s.close()
    cws = [LG.configs.Instance(bbc.labels, LG.materials.model_nk(bbc.model, bbc.lambdas[f]), bbc.dx, bbc.lambdas[f],
                               bbc.n_pml, conv_steps, name="cw%d" % f) for f in conv_idx]
    s = fdtd.Simulation(cws, fdtd.Options(n_steps=conv_steps))
    s.run()
    Rcc, Tcc, _ = s.spectra()
    s.close()
    conv_dR = [abs(float(Rbc[f]) - float(Rcc[k])) for k, f in enumerate(conv_idx)]
    conv_dT = [abs(float(Tbc[f]) - float(Tcc[k])) for k, f in enumerate(conv_idx)]
    log("broadband vs monochromatic at %d steps, %d wavelengths: max |dR| %.4f |dT| %.4f (healthy broadband run %.2f s)"
        % (conv_steps, len(conv_idx), max(conv_dR), max(conv_dT), conv_bb_s))
    te_out = leg_broadband_te(steps, spec[0])
    log("broadband: 2 instances (%.3g cells), %d steps, %d wavelengths each in %.2f s -> %.1f Gcell/s (K=%d, band %d, "
        "bulk kernel %.0f GB/s); batched monochromatic leg %s s; healthy-grid monochromatic sample of %d: %.2f s, "
        "max |dR| %.3g |dT| %.3g" % (cells, steps, nf, wall, rate / 1e9, cfg["t_block"], cfg["band_rows"], achieved,
                                     "%.2f" % batched_seconds if batched_seconds else "n/a", len(cw_sample), wall_cw,
                                     dR, dT))
    return {"workload": "healthy and diseased dicot 24.09 x 48.19 um as two broadband instances (%d x %d at %.2f nm, "
                        "%d x %d at %.2f nm), Lorentz-Drude stand-in materials (2 poles), Gaussian pulse, monitors at "
                        "%d wavelengths 400-1000 nm, %d steps"
                        % (bbs[0].nx, bbs[0].ny, bbs[0].dx * 1e9, bbs[1].nx, bbs[1].ny, bbs[1].dx * 1e9, nf, steps),
            "value": rate / 1e9, "unit": "Gcell-updates/s", "seconds": wall, "cells": cells,
            "t_block": cfg["t_block"], "band_rows": cfg["band_rows"],
            "bulk_kernel_avg_launch_ms": kms / max(1, launches), "bulk_kernel_bytes_per_cell_launch": bytes_per_cell,
            "bulk_kernel_hbm_gbs": achieved, "bulk_kernel_hbm_frac": achieved / HBM_PEAK_GBS,
            "bulk_kernel_traffic_bytes": traffic_record("broadband_leaves", cfg["t_block"], cfg["band_rows"]),
            "batched_monochromatic_seconds": batched_seconds,
            "speedup_vs_batched_monochromatic": (batched_seconds / wall) if batched_seconds else None,
            "monochromatic_sample_nm": [round(float(bb.lambdas[f]) * 1e9) for f in cw_sample],
            "monochromatic_sample_seconds": wall_cw,
            "max_abs_dR_vs_monochromatic_at_run_length": float(dR),
            "max_abs_dT_vs_monochromatic_at_run_length": float(dT),
            "agreement_converged": {
                "steps": conv_steps, "lambda_nm": CONV_LAMS_NM, "tolerance": CONV_TOL,
                "abs_dR": conv_dR, "abs_dT": conv_dT, "max_abs_dR": max(conv_dR), "max_abs_dT": max(conv_dT),
                "within_tolerance": bool(max(conv_dR) <= CONV_TOL and max(conv_dT) <= CONV_TOL),
                "note": "healthy leaf, broadband run against monochromatic runs of the same grid and materials at "
                        "the same run length; the speed-up is per step and does not depend on the run length"},
            "R_healthy": [float(x) for x in R], "T_healthy": [float(x) for x in T],
            "te": {k: v for k, v in te_out.items() if k != "unpolarized_healthy"},
            "unpolarized_healthy": te_out.get("unpolarized_healthy")}


def leg_broadband_te(steps: int = 20000, tm_spectrum=None):
    """The healthy broadband leaf in TEz: its whole run on the broadband TEz
    streaming kernel (tuned shape, kernel timing on), beside the same run on
    the plain sweeps (their spectra must agree exactly); with the TMz spectrum
    of the same leaf, the unpolarised broadband spectrum."""
    import torch
    import leafgen as LG
    from paper_2512_17132_amd import fdtd
    te = LG.configs.broadband_leaf(steps=steps, geometry="healthy")
    te.polarization = 1
    s = fdtd.Simulation([te], fdtd.Options(n_steps=steps, use_graph=0))
    s.autotune()
    tcfg = s.config()
    s.step(tcfg["t_block"])
    s.reset()
    torch.cuda.synchronize()
    s.set_profiling(True, every=PROFILE_EVERY)
    t0 = time.perf_counter()
    s.run()
    te_spec = s.broadband_spectra(0)
    torch.cuda.synchronize()
    te_wall = time.perf_counter() - t0
    tkms, tlaunches = s.kernel_time()
    s.close()
    te_rate = te.cells * steps / te_wall
    # fields, label and the driven pole states of both edges' sides, read and
    # written once per launch, over the special and lean items of the launch
    te_bytes = broadband_te_launch_bytes(te) / te.cells
    te_achieved = broadband_te_launch_bytes(te) / (tkms * 1e-3 / max(1, tlaunches)) / 1e9
    s = fdtd.Simulation([te], fdtd.Options(n_steps=steps, kernel=1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run()
    te_plain_spec = s.broadband_spectra(0)
    torch.cuda.synchronize()
    te_plain_wall = time.perf_counter() - t0
    s.close()
    te_plain_rate = te.cells * steps / te_plain_wall
    te_dR = float(np.abs(np.asarray(te_spec[0]) - np.asarray(te_plain_spec[0])).max())
    te_dT = float(np.abs(np.asarray(te_spec[1]) - np.asarray(te_plain_spec[1])).max())
    traffic = traffic_record("broadband_healthy_te", tcfg["t_block"], tcfg["band_rows"])
    msg = ("broadband TEz, healthy leaf: streaming kernel (K=%d, band %d, special %d) %.2f s -> %.1f Gcell/s, bulk "
           "kernel %.0f GB/s; plain sweeps %.2f s -> %.1f Gcell/s (%.1fx); spectra max |dR| %.2g |dT| %.2g"
           % (tcfg["t_block"], tcfg["band_rows"], tcfg["special_rows"], te_wall, te_rate / 1e9, te_achieved,
              te_plain_wall, te_plain_rate / 1e9, te_plain_wall / te_wall, te_dR, te_dT))
    out = {"workload": "the healthy leaf in broadband TEz (%d x %d at %.2f nm, 2 poles, 61 wavelengths), %d steps"
                       % (te.nx, te.ny, te.dx * 1e9, steps),
           "value": te_rate / 1e9, "unit": "Gcell-updates/s", "seconds": te_wall,
           "t_block": tcfg["t_block"], "band_rows": tcfg["band_rows"], "special_rows": tcfg["special_rows"],
           "bulk_kernel_avg_launch_ms": tkms / max(1, tlaunches), "bulk_kernel_bytes_per_cell_launch": te_bytes,
           "bulk_kernel_hbm_gbs": te_achieved, "bulk_kernel_hbm_frac": te_achieved / HBM_PEAK_GBS,
           "bulk_kernel_traffic_bytes": traffic,
           "plain_sweeps": {"value": te_plain_rate / 1e9, "seconds": te_plain_wall},
           "speedup_vs_plain_sweeps": te_plain_wall / te_wall,
           "max_abs_dR_vs_plain": te_dR, "max_abs_dT_vs_plain": te_dT,
           "R": [float(x) for x in te_spec[0]], "T": [float(x) for x in te_spec[1]]}
    if tm_spectrum is not None:
        Ru, Tu, Au = fdtd.unpolarized(tm_spectrum, te_spec)
        msg += "; unpolarised R(550 nm) %.4f T %.4f" % (Ru[15], Tu[15])
        out["unpolarized_healthy"] = {"R": [float(x) for x in Ru], "T": [float(x) for x in Tu],
                                      "A": [float(x) for x in Au]}
    log(msg)
    return out


def leg_adjoint(fd_h: float = 1e-4):
    """The differentiation form: the 1024 x 2048 monocot, 8000 steps, loss = R.
    Times the plain forward (replayed from its captured graph), the recorded
    forward and the backward; then central differences of R on the GPU, at
    h = 1e-4 in every differentiable label's n and k (one-sided at k = 0; all
    perturbed runs in one batched context), beside the adjoint's gradient.  In FP32 the differences
    are limited by rounding in the monitor sums (R changes by about 1e-4 |dR/dn|
    against FP32 noise of about 1e-6), so they are reported, not compared."""
    import dataclasses
    import numpy as np
    import torch
    import leafgen as LG
    from paper_2512_17132_amd import fdtd
    inst = LG.configs.monocot_config()[0]
    steps = inst.n_steps
    sim = fdtd.Simulation([inst], fdtd.Options(n_steps=steps, checkpoint_every=-1, use_graph=1))
    sim.autotune()
    # warm-up of every path (the first plain run captures the graph)
    sim.run()
    sim.spectra()
    sim.reset()
    sim.run(record=True)
    sim.spectra()
    sim.backward([1.0])
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run()
    R, T, A = sim.spectra()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(record=True)
    sim.spectra()
    torch.cuda.synchronize()
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    gnk, geps = sim.backward([1.0])
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    cfg = sim.config()
    sim.close()
    log("adjoint: forward %.3f s (graph replay), recorded forward %.3f s, backward %.3f s; device memory %.1f GB"
        % (t_fwd, t_rec, t_bwd, cfg["device_bytes"] / 1e9))
    # the same with checkpoints every 80 steps (segments replayed in the
    # backward), the form the library takes when the whole run's Ez history
    # does not fit in half the free device memory
    seg_every = 80
    sim = fdtd.Simulation([inst], fdtd.Options(n_steps=steps, checkpoint_every=seg_every, use_graph=1,
                                               t_block=cfg["t_block"], band_rows=cfg["band_rows"],
                                               special_rows=cfg["special_rows"]))
    sim.autotune()
    sim.run(record=True)
    sim.spectra()
    sim.backward([1.0])
    sim.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(record=True)
    sim.spectra()
    torch.cuda.synchronize()
    t_rec_seg = time.perf_counter() - t0
    t0 = time.perf_counter()
    gnk_seg, _ = sim.backward([1.0])
    torch.cuda.synchronize()
    t_bwd_seg = time.perf_counter() - t0
    seg_bytes = sim.config()["device_bytes"]
    sim.close()
    same_seg = bool(np.array_equal(gnk_seg[0], gnk[0]))
    log("adjoint with checkpoints every %d steps: recorded forward %.3f s, backward %.3f s (%.2f x forward); device "
        "memory %.1f GB; gradients identical: %s" % (seg_every, t_rec_seg, t_bwd_seg, t_bwd_seg / t_fwd, seg_bytes / 1e9,
                                                    same_seg))
    # differences in every differentiable label's n and k (air fixed): central,
    # (R(x+h) - R(x-h))/2h, or where x - h < 0 (k = 0; a negative k is not a
    # material) the one-sided form of the same order, (-3R(x) + 4R(x+h) - R(x+2h))/2h
    labels = range(1, inst.nk.shape[0])
    pert, stencils = [], []
    for L in labels:
        for c in range(2):
            x = inst.nk[L, c]
            st = [(1.0, 0.5), (-1.0, -0.5)] if x - fd_h >= 0 else [(0.0, -1.5), (1.0, 2.0), (2.0, -0.5)]
            terms = []
            for off, w in st:
                nk = inst.nk.copy()
                nk[L, c] += off * fd_h
                terms.append((len(pert), w))
                pert.append(dataclasses.replace(inst, nk=nk))
            stencils.append(("central" if len(st) == 2 else "one-sided", terms))
    s = fdtd.Simulation(pert, fdtd.Options(n_steps=steps, t_block=cfg["t_block"], band_rows=cfg["band_rows"],
                                           special_rows=cfg["special_rows"]))
    t0 = time.perf_counter()
    s.run()
    Rp, _, _ = s.spectra()
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    s.close()
    fd = np.array([sum(w * Rp[i] for i, w in terms) / fd_h for _, terms in stencils])
    adj = np.array([gnk[0][L, c] for L in labels for c in range(2)])
    rel = np.abs(fd - adj) / np.maximum(np.abs(adj), 1e-30)
    log("adjoint vs GPU central differences (h = %g, %d runs in %.2f s): worst relative difference %.2e"
        % (fd_h, len(pert), t_fd, rel.max()))
    names = LG.materials.MONOCOT_LABELS
    return {"workload": "monocot 1024 x 2048, dx = 20 nm, lambda = 550 nm, %d steps, loss = R; checkpoint_every = -1 "
                        "(the whole run's Ez history when it fits in half the free device memory, as here)" % steps,
            "forward_s": t_fwd, "forward_graph_replay": True, "recorded_forward_s": t_rec, "backward_s": t_bwd,
            "adjoint_over_forward": t_bwd / t_fwd, "adjoint_over_recorded_forward": t_bwd / t_rec,
            "recorded_forward_plus_backward_over_forward": (t_rec + t_bwd) / t_fwd,
            "device_bytes": cfg["device_bytes"],
            "checkpointed": {"checkpoint_every": seg_every, "recorded_forward_s": t_rec_seg, "backward_s": t_bwd_seg,
                             "adjoint_over_forward": t_bwd_seg / t_fwd, "device_bytes": seg_bytes,
                             "gradients_identical": same_seg},
            "forward_gcell_s": inst.cells * steps / t_fwd / 1e9,
            "R": float(R[0]), "dR_dn": [float(x) for x in gnk[0][:, 0]], "dR_dk": [float(x) for x in gnk[0][:, 1]],
            "central_differences": {
                "h": fd_h, "runs": len(pert), "seconds": t_fd, "labels": [names[L] for L in labels],
                "stencil_n": [stencils[2 * k][0] for k in range(len(labels))],
                "stencil_k": [stencils[2 * k + 1][0] for k in range(len(labels))],
                "dR_dn_fd": [float(x) for x in fd[0::2]], "dR_dk_fd": [float(x) for x in fd[1::2]],
                "dR_dn_adjoint": [float(x) for x in adj[0::2]], "dR_dk_adjoint": [float(x) for x in adj[1::2]],
                "relative_difference_worst": float(rel.max()), "relative_difference_median": float(np.median(rel)),
                "gated": False},
            "t_block": cfg["t_block"], "band_rows": cfg["band_rows"]}


def profile_pass(args):
    """Short headline run + a device copy of known size (COPY_BYTES read and
    COPY_BYTES written), for rocprofv3 counter collection."""
    import torch
    import leafgen as LG
    from paper_2512_17132_amd import fdtd
    torch.cuda.set_device(0)
    K, B = args.t_block or 10, args.band_rows or 192
    n_steps = args.time_steps
    W = args.bulk_columns
    kernel_cells = None   # cells whose updates the measured kernel makes (default: the lean items')
    if args.profile_workload == "large":
        insts = LG.configs.large_config_parallel()
        name, bytes_per_cell, n_steps = LARGE_NAME, BYTES_PER_CELL_LAUNCH, insts[0].n_steps
        K, B = args.t_block or 12, args.band_rows or 512
        W = W or 256
    elif args.profile_workload == "broadband":
        insts = [LG.configs.broadband_leaf(steps=args.time_steps, geometry=g) for g in ("healthy", "diseased")]
        name, bytes_per_cell = "broadband_leaves", None
        if args.profile_pol:
            # the healthy leaf in broadband TEz
            import copy
            inst = copy.copy(insts[0])
            inst.polarization = 1
            insts, name = [inst], "broadband_healthy"
            K, B = args.t_block or 5, args.band_rows or 64
            bytes_per_cell, kernel_cells = broadband_te_launch_bytes(inst) / inst.cells, inst.cells
    else:
        inst = LG.configs.dicot_config(steps=args.time_steps)[0]
        if args.profile_pol:
            import copy
            inst = copy.copy(inst)
            inst.polarization = 1
        insts, name, bytes_per_cell = [inst], inst.name, BYTES_PER_CELL_LAUNCH
    sim = fdtd.Simulation(insts, fdtd.Options(n_steps=n_steps, t_block=K, band_rows=B, use_graph=0,
                                              bulk_columns=W))
    sim.step(K * args.profile_launches)
    torch.cuda.synchronize()
    cfg = sim.config()
    if bytes_per_cell is None:
        bytes_per_cell = broadband_launch_bytes(insts, cfg["lean_cells"]) / cfg["lean_cells"]
    kernel_cells = kernel_cells or cfg["lean_cells"]
    x = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"profile_pass": True, "workload": name, "polarization": args.profile_pol,
                      "bytes_per_cell": bytes_per_cell,
                      "t_block": cfg["t_block"],
                      "band_rows": cfg["band_rows"], "bulk_columns": cfg["bulk_columns"], "lean_cells": cfg["lean_cells"],
                      "kernel_cells": kernel_cells, "launches": args.profile_launches, "copy_bytes": COPY_BYTES}))
    sim.close()


def derive_traffic(fetch_dir: str, write_dir: str):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the bulk kernel, each scaled
    by what the same counter reads for the reference copy (COPY_BYTES read and
    COPY_BYTES written), into profiles/traffic.json."""
    import csv
    import glob

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        return list(csv.DictReader(open(f)))

    def pass_info(d):
        for f in glob.glob(os.path.join(d, "*.log")) + glob.glob(os.path.join(d, "..", os.path.basename(d) + ".log")):
            for line in open(f):
                if line.startswith('{"profile_pass"'):
                    return json.loads(line)
        return {}

    info = pass_info(fetch_dir)
    te = bool(info.get("polarization"))
    if info.get("workload") == "broadband_leaves":
        bulk_re = r"k_tblock_bb<\d+, false>"
    elif info.get("workload") == "broadband_healthy":
        bulk_re = r"k_tblock_bt<\d+>"
    else:
        bulk_re = (r"k_tblock_te<\d+, false>" if te else
                   r"k_tblock_wg<\d+, false>" if info.get("bulk_columns") == 256 else r"k_tblock<\d+, false, false>")
    meas = {}
    for key, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rs = [r for r in rows(d) if r["Counter_Name"] == key]
        bulk = [float(r["Counter_Value"]) for r in rs if re.search(bulk_re, r["Kernel_Name"])]
        copies = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), float(r["Counter_Value"]))
                  for r in rs if "copyBuffer" in r["Kernel_Name"]]
        if not bulk or not copies:
            raise RuntimeError("counter %s: %d bulk and %d copy dispatches" % (key, len(bulk), len(copies)))
        copy_kib = max(copies)[1]          # the longest copy dispatch is the reference copy
        scale = (COPY_BYTES / 1024.0) / copy_kib
        meas[key] = {"bulk_kib_per_dispatch": sum(bulk) / len(bulk), "dispatches": len(bulk),
                     "reference_copy_kib": copy_kib, "scale": scale,
                     "bytes_per_launch": sum(bulk) / len(bulk) * scale * 1024.0}
    total = meas["FETCH_SIZE"]["bytes_per_launch"] + meas["WRITE_SIZE"]["bytes_per_launch"]
    workload = info.get("workload", "dicot4096x8192") + ("_te" if te else "")
    rec = {"kernel_hash": kernel_source_hash(workload), "t_block": info.get("t_block"), "band_rows": info.get("band_rows"),
           "bytes_per_launch": total, "counters": meas,
           "algorithmic_bytes_per_launch": info.get("bytes_per_cell", BYTES_PER_CELL_LAUNCH) *
           info.get("kernel_cells", info.get("lean_cells", 0))}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    allrec = json.load(open(path)) if os.path.exists(path) else {}
    shapes = allrec.get(workload, {})
    if "kernel_hash" in shapes:          # a record of one shape only
        shapes = {}
    shapes = {k: v for k, v in shapes.items() if v.get("kernel_hash") == rec["kernel_hash"]}
    rec["bulk_columns"] = info.get("bulk_columns", 64)
    shapes[shape_key(rec["t_block"], rec["band_rows"], rec["bulk_columns"])] = rec
    allrec[workload] = shapes
    os.makedirs(os.path.dirname(path), exist_ok=True)
    json.dump(allrec, open(path, "w"), indent=1)
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed whole runs of the headline batch")
    ap.add_argument("--warmup", type=int, default=1, help="untimed whole runs before them")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--deadline-s", type=float, default=780.0,
                    help="an extra leg starts only if it is expected to end before this much wall time")
    ap.add_argument("--cpu-steps", type=int, default=480,
                    help="oracle steps of the host sample, centred on the start of the monitor window")
    ap.add_argument("--cpu-steps-single", type=int, default=24, help="oracle steps of the one-thread sample")
    ap.add_argument("--time-steps", type=int, default=20000, help="FDTD steps of the dicot workload's runs")
    ap.add_argument("--t-block", type=int, default=0)
    ap.add_argument("--band-rows", type=int, default=0)
    ap.add_argument("--bulk-columns", type=int, default=0, choices=(0, 64, 256),
                    help="profile pass: columns per bulk TMz work item (0: 64, or 256 on the headline batch)")
    ap.add_argument("--profile-pass", action="store_true")
    ap.add_argument("--profile-launches", type=int, default=12)
    ap.add_argument("--profile-pol", type=int, default=0, choices=(0, 1), help="profile pass in TMz (0) or TEz (1)")
    ap.add_argument("--profile-workload", default="dicot", choices=("large", "dicot", "broadband"),
                    help="profile pass on the headline batch, the dicot workload or the two broadband leaves")
    ap.add_argument("--derive-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--leg", choices=("te", "adjoint", "broadband", "broadband_te", "dicot"),
                    help="run this extra leg alone and print its JSON (for profiling)")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="with --leg te: replay the timed run from its captured graph (1) or launch directly (0)")
    args = ap.parse_args()
    t_start = time.time()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (independent instances would shard across GPUs with no "
              "exchange); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.derive_traffic:
        derive_traffic(*args.derive_traffic)
        return
    if args.profile_pass:
        profile_pass(args)
        return
    if args.leg:
        import torch
        import leafgen as LG
        torch.cuda.set_device(0)
        if args.leg == "te":
            r = leg_te(LG.configs.dicot_config(steps=args.time_steps)[0], None, use_graph=args.graph)
        elif args.leg == "dicot":
            r = leg_dicot(LG.configs.dicot_config(steps=args.time_steps)[0])
        elif args.leg == "adjoint":
            r = leg_adjoint()
        elif args.leg == "broadband_te":
            r = leg_broadband_te()
        else:
            r = leg_broadband(None)
        print(json.dumps({"leg": args.leg, **r}), flush=True)
        return

    import torch
    import leafgen as LG
    from paper_2512_17132_amd import fdtd

    # inputs are rasterised in fresh interpreters (spawned process pools),
    # the large ones before this process touches the GPU
    t0 = time.time()
    insts = LG.configs.large_config_parallel()
    log("headline batch: %d instances, %.3g cells, %d steps, generated in %.1fs"
        % (len(insts), sum(i.cells for i in insts), insts[0].n_steps, time.time() - t0))
    insts_b = None
    paper_lab = None
    paper_pool = None
    if not args.no_extras:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        paper_pool = ProcessPoolExecutor(max_workers=1, mp_context=mp.get_context("spawn"))
        paper_lab = paper_pool.submit(LG.configs.paper_dicot)
        t0 = time.time()
        insts_b = batched_instances(args.time_steps)
        log("batched: %d instances, %.3g cells (%d x %d .. %d x %d), generated in %.1fs"
            % (len(insts_b), sum(i.cells for i in insts_b), min(i.nx for i in insts_b), min(i.ny for i in insts_b),
               max(i.nx for i in insts_b), max(i.ny for i in insts_b), time.time() - t0))
    torch.cuda.set_device(0)

    # ---- headline: the 8-instance batch, whole runs ----
    n_steps = insts[0].n_steps
    cells = sum(i.cells for i in insts)
    sim = fdtd.Simulation(insts, fdtd.Options(n_steps=n_steps, t_block=args.t_block, band_rows=args.band_rows,
                                              use_graph=0))
    rate_tune = sim.autotune()
    cfg = sim.config()
    log("config", cfg, "autotune best %.1f Gcell/s" % (rate_tune / 1e9))
    for w in range(args.warmup):
        sim.reset()
        t0 = time.time()
        sim.run()
        R, T, A = sim.spectra()
        log("warmup run %d (%.1f s): R %s T %s" % (w, time.time() - t0, np.round(R, 5).tolist(),
                                                  np.round(T, 5).tolist()))
    sim.reset()
    wall, kms, launches, (R, T, A) = timed_runs(sim, args.steps)
    cfg = sim.config()
    sim.close()
    copy_gbs = copy_bandwidth_gbs()
    log("device copy bandwidth: %.0f GB/s" % copy_gbs)
    value = cells * n_steps * args.steps / wall
    K, B, W = cfg["t_block"], cfg["band_rows"], cfg["bulk_columns"]
    avg_launch_s = kms * 1e-3 / max(1, launches)
    bytes_per_launch = BYTES_PER_CELL_LAUNCH * cfg["lean_cells"]
    achieved = bytes_per_launch / avg_launch_s / 1e9
    log("timed: %.3f s for %d runs -> %.1f Gcell/s; bulk kernel %.3f ms avg over %d timed launches (every %d-th; "
        "K=%d, band %d, bulk items of %d columns)" % (wall, args.steps, value / 1e9, kms / max(1, launches), launches,
                                                      PROFILE_EVERY, K, B, W))
    traffic = traffic_record(LARGE_NAME, K, B, W)
    out = {
        "metric": "FDTD Gcell-updates/s + % HBM roofline; batched vs plain; adjoint/forward time",
        "value": value / 1e9,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded dicot cross-section generator)",
        "config": {"workload": "large plain + batched: synthetic dicot cross-section at dx = 12.5 nm, %d x %d cells, "
                               "lambda = 450/550/680/850 nm x {healthy, diseased} = %d instances (%d cells) in one "
                               "context, %d FP32 steps, 32-cell CPML, compensated monitor sums over the last %d steps; "
                               "one step = reset + whole run + spectra"
                               % (insts[0].nx, insts[0].ny, len(insts), cells, n_steps, n_steps // 2),
                   "instances": [i.name for i in insts], "cells": cells, "time_steps": n_steps, "t_block": K,
                   "band_rows": B, "bulk_columns": W, "R": [float(x) for x in R], "T": [float(x) for x in T],
                   "A": [float(x) for x in A]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": bulk_kernel_name(K, W), "avg_launch_ms": kms / max(1, launches),
                     "launches": launches, "timed_every": PROFILE_EVERY,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "steps_per_launch": K,
                     "copy_bandwidth": copy_gbs, "frac_of_copy_bandwidth": achieved / copy_gbs,
                     "effective_frac_at_25B_per_cell_update": value * 25 / (HBM_PEAK_GBS * 1e9)},
    }

    inst_c = insts[0]
    if not args.no_cpu:
        w0 = n_steps - n_steps // 2
        n0 = w0 - args.cpu_steps // 2
        rate, dt, cores = run_oracle_sample(inst_c, n0, n0 + args.cpu_steps)
        host = host_cpu()
        out["cpu_baseline"] = {"value": rate / 1e9, "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
                               "sample": "FP64 oracle (plain separate E/H sweeps, OpenMP), steps %d-%d of one "
                                         "%d x %d instance (%s) of the headline batch, from a zero state, the "
                                         "monitor window opening at step %d so that half of the sampled steps "
                                         "carry the monitor sums (%.1f s on %d threads; the per-step cost does "
                                         "not depend on the field values)"
                                         % (n0, n0 + args.cpu_steps - 1, inst_c.nx, inst_c.ny, inst_c.name, w0, dt,
                                            cores),
                               **host}
        if args.cpu_steps_single > 0:
            rate1, dt1, _ = run_oracle_sample(inst_c, n0, n0 + args.cpu_steps_single, threads=1)
            out["cpu_baseline"]["single_core"] = {
                "value": rate1 / 1e9, "unit": "Gcell-updates/s", "cores": 1,
                "sample": "the same oracle on one thread, steps %d-%d (%.1f s)"
                          % (n0, n0 + args.cpu_steps_single - 1, dt1)}
            log("oracle: %.2f Gcell/s on %d threads, %.3f on one (%s, nproc %s)"
                % (rate / 1e9, cores, rate1 / 1e9, host["cpu_model"], host["nproc"]))
    insts = None

    def leg(name, est_s, fn):
        """Runs an extra leg if it is expected to end before the deadline."""
        used = time.time() - t_start
        if used + est_s > args.deadline_s:
            log("%s: skipped (%.0f s used, about %.0f s needed, deadline %.0f s)" % (name, used, est_s,
                                                                                     args.deadline_s))
            out[name] = {"skipped": "about %.0f s needed after %.0f s, past the %.0f s deadline"
                                    % (est_s, used, args.deadline_s)}
            return
        try:
            out[name] = fn()
        except Exception as e:  # report, do not hide the headline
            out[name] = {"error": repr(e)}

    if not args.no_extras:
        dicot = LG.configs.dicot_config(steps=args.time_steps)[0]
        leg("dicot", 8, lambda: leg_dicot(dicot))
        leg("large_one", 15, lambda: leg_large_one(inst_c))
        if "value" in out.get("large_one", {}):
            out["large_one"]["batched_over_one"] = out["value"] / out["large_one"]["value"]
        leg("adjoint", 8, leg_adjoint)
        d = out.get("dicot", {})
        leg("te", 6, lambda: leg_te(dicot, (np.array([d["R"]]), np.array([d["T"]]), np.array([d["A"]]))
                                    if "R" in d else None))
        leg("batched", 40, lambda: leg_batched(insts_b, args.time_steps))
        insts_b = None
        leg("broadband", 20, lambda: leg_broadband(out.get("batched", {}).get("seconds")))
        leg("sweep", 30, lambda: leg_sweep(paper_lab.result()))
        paper_pool.shutdown(cancel_futures=True)
    out["wall_seconds"] = time.time() - t_start
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
