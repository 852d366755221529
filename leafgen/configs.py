"""The five workloads the solver is measured and checked on, as seeded
synthetic inputs.

Each workload is a list of instances.  An instance is one monochromatic TMz
run: a uint8 label map, a per-label (n, k) table at its wavelength, and the
grid description.  Row placement inside the domain (bottom to top): CPML,
transmission monitor j_trn = n_pml + 4, the structure, TF/SF row
j_src = ny - n_pml - 8, reflection monitor j_ref = ny - n_pml - 4, CPML.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import geometry as G
from . import materials as M

SEED_BASE = 17132


@dataclass
class Instance:
    labels: np.ndarray          # (ny, nx) uint8
    nk: np.ndarray              # (n_labels, 2) float64
    dx: float                   # metres
    lambda0: float              # metres
    n_pml: int
    n_steps: int
    courant: float = 0.99
    ramp_periods: float = 5.0
    name: str = ""
    polarization: int = 0       # 0: TMz (S), 1: TEz (P)

    @property
    def ny(self) -> int:
        return self.labels.shape[0]

    @property
    def nx(self) -> int:
        return self.labels.shape[1]

    @property
    def j_src(self) -> int:
        return self.ny - self.n_pml - 8

    @property
    def j_ref(self) -> int:
        return self.ny - self.n_pml - 4

    @property
    def j_trn(self) -> int:
        return self.n_pml + 4

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def slab_config(nx: int = 256, ny: int = 256, steps: int = 3000) -> list[Instance]:
    """Plain method, tiny: 256 x 256, dx = 20 nm, 16-cell CPML, vacuum with a
    1.0 um slab (n = 1.45, k = 0.01) at mid-height (50 rows), lambda = 600 nm,
    3000 steps."""
    lo = ny // 2 - 25
    lab = G.slab(nx, ny, lo, lo + 50)
    return [Instance(lab, M.slab_nk(1.45, 0.01), 20e-9, 600e-9, 16, steps, name="slab256")]


def dicot_config(nx: int = 4096, ny: int = 8192, dx_nm: float = 25.0, steps: int = 20000,
                 lam_nm: float = 550.0, seed: int = SEED_BASE + 2) -> list[Instance]:
    """Synthetic dicot cross-section, plain method: 4096 x 8192 cells at 25 nm
    (about 102 x 205 um), lambda = 550 nm, 20000 steps, 32-cell CPML."""
    lab = G.dicot(nx, ny, dx_nm, seed)
    return [Instance(lab, M.dicot_nk(lam_nm * 1e-9), dx_nm * 1e-9, lam_nm * 1e-9, 32, steps,
                     name="dicot%dx%d" % (nx, ny))]


BATCH_LX_UM = 24.09
BATCH_LY_UM = 48.19
BATCH_LAYERS = G.DicotLayers(cuticle=1.5, upper_epidermis=6.0, palisade=12.0, spongy=11.0,
                             lower_epidermis=4.0, epi_width=(6.0, 10.0), low_epi_width=(5.0, 8.0),
                             palisade_cell=(5.0, 11.0), spongy_axes=(2.0, 4.0), chl_mu=1.0,
                             chl_sigma=0.25)


def batched_config(lams_nm=None, steps: int = 20000, seed: int = SEED_BASE + 3,
                   geometries=("healthy", "diseased"), scale: float = 1.0) -> list[Instance]:
    """Batched form: wavelengths 400-1000 nm in 10 nm steps x {healthy, diseased}
    geometries of one 24.09 x 48.19 um domain, each rasterised at
    dx = lambda/(n_max * 20) (n_max = 1.52 healthy, 1.7 diseased), so grid sizes
    differ between instances (732 x 1465 up to 2048 x 4096)."""
    if lams_nm is None:
        lams_nm = list(range(400, 1001, 10))
    out = []
    for geo in geometries:
        nmax = 1.7 if geo == "diseased" else 1.52
        for lam in lams_nm:
            dx = lam / (nmax * 20.0) / scale
            nx = int(round(BATCH_LX_UM * 1e3 / dx))
            ny = int(round(BATCH_LY_UM * 1e3 / dx))
            lab = G.dicot(nx, ny, dx, seed, diseased=(geo == "diseased"), layers=BATCH_LAYERS,
                          hypha_seed=seed + 77)
            out.append(Instance(lab, M.dicot_nk(lam * 1e-9), dx * 1e-9, lam * 1e-9, 32, steps,
                                name="%s_%dnm" % (geo, lam)))
    return out


@dataclass
class BroadbandInstance:
    """One broadband TMz run: a pulse centred on lambda0 covering the monitor
    wavelengths, and a Lorentz-Drude table per label (materials.dicot_model)."""
    labels: np.ndarray
    model: np.ndarray
    lambdas: np.ndarray
    pulse_tau: float
    pulse_t0: float
    dx: float
    lambda0: float
    n_pml: int
    n_steps: int
    n_poles: int = M.MODEL_POLES
    courant: float = 0.99
    name: str = ""

    ny = Instance.ny
    nx = Instance.nx
    j_src = Instance.j_src
    j_ref = Instance.j_ref
    j_trn = Instance.j_trn
    cells = Instance.cells


def gaussian_pulse(lam_min: float, lam_max: float, edge: float = 3.0, delay: float = 4.0):
    """(lambda0, tau, t0) of exp(-((t - t0)/tau)^2) sin(w0 (t - t0)) with w0 the
    middle of the band in frequency, the spectrum down to exp(-edge) at its
    edges, and the peak delay * tau after the start."""
    c0 = 299792458.0
    wlo, whi = 2 * math.pi * c0 / lam_max, 2 * math.pi * c0 / lam_min
    tau = 4.0 * math.sqrt(edge) / (whi - wlo)
    return 2 * math.pi * c0 / (0.5 * (wlo + whi)), tau, delay * tau


def broadband_leaf(lams_nm=None, geometry: str = "healthy", steps: int = 20000, seed: int = SEED_BASE + 3,
                   scale: float = 1.0) -> BroadbandInstance:
    """The batched workload's 24.09 x 48.19 um dicot as one broadband run: the
    grid of its shortest wavelength (dx = lambda_min/(20 n_max)), the
    Lorentz-Drude stand-in materials, monitors at 400-1000 nm every 10 nm."""
    if lams_nm is None:
        lams_nm = list(range(400, 1001, 10))
    nmax = 1.7 if geometry == "diseased" else 1.52
    dx = min(lams_nm) / (nmax * 20.0) / scale
    nx = int(round(BATCH_LX_UM * 1e3 / dx))
    ny = int(round(BATCH_LY_UM * 1e3 / dx))
    lab = G.dicot(nx, ny, dx, seed, diseased=(geometry == "diseased"), layers=BATCH_LAYERS, hypha_seed=seed + 77)
    lams = np.array(lams_nm, dtype=np.float64) * 1e-9
    lam0, tau, t0 = gaussian_pulse(lams.min(), lams.max())
    return BroadbandInstance(lab, M.dicot_model(), lams, tau, t0, dx * 1e-9, lam0, 32, steps,
                             name="%s_broadband" % geometry)


def _batched_one(args) -> Instance:
    lam, geo, steps, seed, scale = args
    return batched_config([lam], steps, seed, geometries=(geo,), scale=scale)[0]


def batched_config_parallel(steps: int = 20000, workers: int = 16, seed: int = SEED_BASE + 3,
                            scale: float = 1.0) -> list[Instance]:
    """batched_config with the instances rasterised in worker processes.  The
    workers are fresh interpreters ("spawn"), never forks of the caller, so this
    is safe to call from a process that already uses the GPU."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    jobs = [(lam, geo, steps, seed, scale) for geo in ("healthy", "diseased") for lam in range(400, 1001, 10)]
    with ProcessPoolExecutor(max_workers=max(1, workers), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_batched_one, jobs, chunksize=2))


def _large_geometry(args) -> np.ndarray:
    nx, ny, seed, geo = args
    return G.dicot(nx, ny, 12.5 * 8192 / nx, seed, diseased=(geo == "diseased"))


def large_config_parallel(nx: int = 8192, ny: int = 16384, steps: int = 40000, seed: int = SEED_BASE + 2,
                          lams_nm=(450, 550, 680, 850)) -> list[Instance]:
    """large_config with the two geometries rasterised in two worker processes
    (fresh interpreters, safe from a process that already uses the GPU)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    geos = ("healthy", "diseased")
    with ProcessPoolExecutor(max_workers=2, mp_context=mp.get_context("spawn")) as ex:
        labs = list(ex.map(_large_geometry, [(nx, ny, seed, g) for g in geos]))
    out = []
    for geo, lab in zip(geos, labs):
        for lam in lams_nm:
            out.append(Instance(lab, M.dicot_nk(lam * 1e-9), 12.5e-9 * 8192 / nx, lam * 1e-9, 32, steps,
                                name="%s_%dnm" % (geo, lam)))
    return out


# the paper's healthy dicot (Sec. 4): 140 um thick, about 200 um wide
PAPER_DICOT_LAYERS = G.DicotLayers(upper_epidermis=16.0, palisade=58.0, spongy=48.0, lower_epidermis=14.0)
PAPER_DICOT_GRID = dict(nx=8511, ny=6689, dx_nm=23.41, n_pml=32)


def paper_dicot(nx: int = 8511, ny: int = 6689, dx_nm: float = 23.41, seed: int = SEED_BASE + 5,
                diseased: bool = False) -> np.ndarray:
    """Label map at the paper's dicot grid (8511 x 6689 cells at 23.41 nm,
    CPML included): a 140 um thick synthetic leaf, centred, with air above
    and below.  Wavelength tables come from materials.dicot_nk."""
    return G.dicot(nx, ny, dx_nm, seed, diseased=diseased, layers=PAPER_DICOT_LAYERS)


def rows(ny: int, n_pml: int) -> tuple[int, int, int]:
    """(j_src, j_ref, j_trn) of the row layout every workload here uses."""
    return ny - n_pml - 8, ny - n_pml - 4, n_pml + 4


def monocot_config(nx: int = 1024, ny: int = 2048, steps: int = 8000, seed: int = SEED_BASE + 4,
                   n_pml: int = 32) -> list[Instance]:
    """Differentiation form: 1024 x 2048 synthetic monocot at 20 nm
    (20.48 x 40.96 um), lambda = 550 nm, 8000 steps, 32-cell CPML.  Smaller
    grids keep the physical domain and coarsen dx."""
    dx_nm = 20.0 * 1024 / nx
    lab = G.monocot(nx, ny, dx_nm, seed)
    return [Instance(lab, M.monocot_nk(550e-9), dx_nm * 1e-9, 550e-9, n_pml, steps,
                     name="monocot%dx%d" % (nx, ny))]


def large_config(nx: int = 8192, ny: int = 16384, steps: int = 40000, seed: int = SEED_BASE + 2,
                 lams_nm=(450, 550, 680, 850)) -> list[Instance]:
    """Large plain + batched: the dicot geometry at 12.5 nm (8192 x 16384),
    4 wavelengths x {healthy, diseased}, 40000 steps."""
    out = []
    for geo in ("healthy", "diseased"):
        lab = G.dicot(nx, ny, 12.5 * 8192 / nx, seed, diseased=(geo == "diseased"))
        for lam in lams_nm:
            out.append(Instance(lab, M.dicot_nk(lam * 1e-9), 12.5e-9 * 8192 / nx, lam * 1e-9, 32, steps,
                                name="%s_%dnm" % (geo, lam)))
    return out


def random_instance(nx: int, ny: int, seed: int, n_labels: int = 5, steps: int = 600,
                    n_pml: int = 12, dx: float = 20e-9, lam: float = 500e-9, lossy: bool = True,
                    block=(3, 5)) -> Instance:
    """Seeded random piecewise-constant map for parity tests: labels 1..n_labels-1
    get n in [1.3, 1.8] and (if lossy) k in [0, 0.08]; label 0 is air."""
    rng = np.random.default_rng(seed + 9000)
    lo = n_pml + 8
    hi = ny - n_pml - 10
    lab = G.random_blocks(nx, ny, seed, n_labels, lo, hi, block)
    nk = np.zeros((n_labels, 2))
    nk[0] = (1.0, 0.0)
    nk[1:, 0] = rng.uniform(1.3, 1.8, n_labels - 1)
    nk[1:, 1] = rng.uniform(0.0, 0.08, n_labels - 1) if lossy else 0.0
    return Instance(lab, nk, dx, lam, n_pml, steps, name="random%d" % seed)


def cylinder_config(l_over_lambda, steps: int = 20000, n_pml: int = 32, nx: int = 100, ny: int = 896,
                    h: float = 0.01, radius: float = 0.3, n_cyl: float = 2.0) -> list[Instance]:
    """The paper's validation workload (Sec. 3, its parameter table): a periodic
    array of dielectric cylinders of index 2 with period L = nx h = 1 m,
    S-polarised normal incidence, h = 0.01 m, 101 x 897 grid points, i.e.
    100 x 896 cells with the periodic axis taken as x.  One instance per
    normalised frequency L/lambda.  The size 0.3 m is taken as the radius: with
    it the spectrum shows the transmission drop to nearly zero near
    L/lambda = 0.82 and the near-total transmission below 0.8 that the paper
    describes; read as a diameter, the minimum sits near 0.855 and about a
    quarter of the power is reflected below 0.8."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    xc, yc = 0.5 * nx, 0.5 * ny
    r = radius / h
    lab = (((xx + 0.5 - xc) ** 2 + (yy + 0.5 - yc) ** 2) <= r * r).astype(np.uint8)
    nk = np.array([[1.0, 0.0], [n_cyl, 0.0]])
    L = nx * h
    return [Instance(lab, nk, h, L / f, n_pml, steps, name="cylinders_L/lambda=%.4f" % f) for f in l_over_lambda]
