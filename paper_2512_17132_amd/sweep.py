"""Spectral sweeps over wavelength x polarisation x slice, averaged (Sec. 4 and
4.2).

The paper simulates a wide leaf cross-section as a few side-by-side slices,
each closed by periodic side walls, runs every slice at every wavelength in
both polarisations as an independent monochromatic simulation, and reports R
and T averaged over the slices and the two polarisations.  This module plans
those runs, packs them into batched contexts (``fdtd.Simulation``, one set of
launches per context) under a device-memory budget, and averages the
spectra.  Runs of one context may differ in length: each leaves the batched
launches at its own step count.  Every time step runs in the library's HIP
kernels; this module arranges instances and averages the returned scalars.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import fdtd


@dataclass
class Run:
    """One monochromatic run of one slice (the instance interface of
    ``fdtd.Simulation``)."""
    labels: np.ndarray      # (ny, nx) uint8, C-contiguous (shared by the runs of a slice)
    nk: np.ndarray          # (n_labels, 2) at lambda0
    dx: float
    lambda0: float
    n_pml: int
    j_src: int
    j_ref: int
    j_trn: int
    polarization: int       # 0 TMz (S), 1 TEz (P)
    n_steps: int
    courant: float = 0.99
    slice: int = 0

    @property
    def cells(self) -> int:
        return int(self.labels.shape[0] * self.labels.shape[1])


def slice_bounds(nx: int, n_slices: int) -> list[tuple[int, int]]:
    """Column ranges [x0, x1) of n_slices side-by-side slices covering 0..nx,
    widths differing by at most one column."""
    if not 1 <= n_slices <= nx:
        raise ValueError("need 1 <= n_slices <= nx")
    edges = [(k * nx) // n_slices for k in range(n_slices + 1)]
    return list(zip(edges[:-1], edges[1:]))


def steps_per_period(lam: float, dx: float, courant: float) -> float:
    """Time steps in one period of the source: lambda / (c dt) with
    c dt = S dx / sqrt(2)."""
    return lam / (courant / math.sqrt(2.0) * dx)


def steps_for_periods(periods: float, floor: int = 0):
    """A run-length rule: enough steps for `periods` source periods (at least
    `floor`), rounded up to an even count."""
    def rule(lam: float, dx: float, courant: float) -> int:
        n = max(floor, int(math.ceil(periods * steps_per_period(lam, dx, courant))))
        return n + (n & 1)
    return rule


def plan(labels: np.ndarray, nk_of, wavelengths, dx: float, n_pml: int, j_src: int, j_ref: int, j_trn: int,
         n_steps, n_slices: int = 5, polarizations=(0, 1), courant: float = 0.99) -> list[Run]:
    """Runs of a sweep, slice-major: for each slice, each wavelength, each
    polarisation.  nk_of(lambda) gives the per-label (n, k) table; n_steps is
    a step count or a rule (lambda, dx, courant) -> steps."""
    labels = np.asarray(labels, dtype=np.uint8)
    ny, nx = labels.shape
    slices = [np.ascontiguousarray(labels[:, a:b]) for a, b in slice_bounds(nx, n_slices)]
    runs = []
    for s, lab in enumerate(slices):
        for lam in wavelengths:
            nk = np.ascontiguousarray(nk_of(lam), dtype=np.float64)
            n = int(n_steps(lam, dx, courant)) if callable(n_steps) else int(n_steps)
            for pol in polarizations:
                runs.append(Run(lab, nk, dx, float(lam), n_pml, j_src, j_ref, j_trn, int(pol), n, courant, s))
    return runs


def _align(b: int) -> int:
    return (b + 255) // 256 * 256


def device_bytes(run: Run) -> int:
    """Device memory the library allocates for one run (fields, layer states,
    labels and tables; the adjoint's buffers are not included)."""
    ny, nx = run.labels.shape
    pitch = (nx + 63) // 64 * 64
    f = _align(ny * pitch * 4)
    p = _align((2 * run.n_pml + 1) * pitch * 4)
    return (2 * (3 * f + 2 * p) + _align(ny * pitch) + _align(256 * 8) + 2 * _align(16 * ny)
            + 2 * _align(8 * run.n_steps) + _align(32 * pitch) + 256)


def pack(runs: list[Run], budget_bytes: int) -> list[list[int]]:
    """Groups run indices into contexts of at most budget_bytes each, longest
    runs first so that the runs of one context have similar lengths."""
    order = sorted(range(len(runs)), key=lambda i: (-runs[i].n_steps, runs[i].slice, runs[i].lambda0,
                                                    runs[i].polarization))
    batches, cur, used = [], [], 0
    for i in order:
        b = device_bytes(runs[i])
        if b > budget_bytes:
            raise ValueError("run %d alone needs %d bytes, above the budget of %d" % (i, b, budget_bytes))
        if cur and used + b > budget_bytes:
            batches.append(cur)
            cur, used = [], 0
        cur.append(i)
        used += b
    if cur:
        batches.append(cur)
    return batches


@dataclass
class SweepResult:
    runs: list[Run]
    R: np.ndarray
    T: np.ndarray
    A: np.ndarray
    batches: list[list[int]]
    seconds: float = 0.0            # wall time of the whole sweep
    run_seconds: float = 0.0        # of it, running the steps and fitting the spectra
    setup_seconds: float = 0.0      # of it, creating contexts (host tables, uploads)
    tune_seconds: float = 0.0       # of it, autotuning launch shapes
    cell_updates: int = 0
    batch_seconds: list[float] = field(default_factory=list)
    # (t_block, band_rows, special_rows, bulk_columns) per context
    shapes: list[tuple[int, int, int, int]] = field(default_factory=list)

    def spectrum(self, polarizations=None):
        """(wavelengths, R, T, A): the library's mean over slices and the given
        polarisations (default: all of the sweep's) at each wavelength
        (fdtd_combine_spectra)."""
        lams = sorted({r.lambda0 for r in self.runs})
        pols = set(polarizations) if polarizations is not None else {r.polarization for r in self.runs}
        index = {lam: k for k, lam in enumerate(lams)}
        sel = [i for i, r in enumerate(self.runs) if r.polarization in pols]
        group = [index[self.runs[i].lambda0] for i in sel]
        missing = sorted(set(range(len(lams))) - set(group))
        if missing:
            raise ValueError("no runs at %g m for polarisations %s" % (lams[missing[0]], sorted(pols)))
        R, T, A = fdtd.combine_spectra(self.R[sel], self.T[sel], group, len(lams))
        return np.array(lams), R, T, A


def run_sweep(runs: list[Run], budget_bytes: int | None = None, progress=None, retune: bool = False,
              **opts) -> SweepResult:
    """Runs every planned run in batched contexts on the current device and
    returns per-run R, T, A.  budget_bytes defaults to 60 % of the free device
    memory; opts are further fdtd.Options fields (t_block, band_rows, ...).
    The first context is autotuned and the later ones reuse its launch shape
    (the contexts of a sweep hold the same slice grids); retune=True tunes
    every context, and a t_block or band_rows in opts fixes that part."""
    if budget_bytes is None:
        import torch
        free, _ = torch.cuda.mem_get_info()
        budget_bytes = int(0.6 * free)
    batches = pack(runs, budget_bytes)
    R, T, A = (np.zeros(len(runs)) for _ in range(3))
    res = SweepResult(runs, R, T, A, batches)
    t0 = time.perf_counter()
    for b, idx in enumerate(batches):
        t1 = time.perf_counter()
        group = [runs[i] for i in idx]
        steps = [r.n_steps for r in group]
        with fdtd.Simulation(group, fdtd.Options(n_steps=max(steps), **opts), run_steps=steps) as s:
            t2 = time.perf_counter()
            res.setup_seconds += t2 - t1
            if not (opts.get("t_block", 0) > 0 and opts.get("band_rows", 0) > 0):
                s.autotune()
            t3 = time.perf_counter()
            res.tune_seconds += t3 - t2
            s.run()
            r, t, a = s.spectra()
            cfg = s.config()        # the launch shape is settled once the run has started
            res.shapes.append((cfg["t_block"], cfg["band_rows"], cfg["special_rows"], cfg["bulk_columns"]))
            if not retune:
                opts.setdefault("t_block", cfg["t_block"])
                opts.setdefault("band_rows", cfg["band_rows"])
                opts.setdefault("special_rows", cfg["special_rows"])
                opts.setdefault("bulk_columns", cfg["bulk_columns"])
            res.run_seconds += time.perf_counter() - t3
        R[idx], T[idx], A[idx] = r, t, a
        res.cell_updates += sum(g.cells * g.n_steps for g in group)
        res.batch_seconds.append(time.perf_counter() - t1)
        if progress:
            progress(b, len(batches), len(idx), res.batch_seconds[-1])
    res.seconds = time.perf_counter() - t0
    return res
