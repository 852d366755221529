"""FP64 CPU oracle for the 2D TMz and TEz FDTD method (arXiv 2512.17132, Sec. 2.2-2.6).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  Nothing here is shared with the GPU
library: this package loads its own C file (``fdtd_oracle.c``) built with gcc,
and works in SI units following the paper's notation (TMz: E at half-integer
times, eqs. 18-20; TEz: H at half-integer times, eqs. 14-16).

Functions with no closed-form pin say so in their docstring; every other one is
checked by ``tests/test_oracle_*.py`` against values fixed by the paper or by
the mathematics (discrete and continuous transfer matrices, energy balance,
symmetries, finite differences).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdtd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

C0 = 299792458.0
MU0 = 1.25663706212e-6
EPS0 = 1.0 / (MU0 * C0 * C0)
ETA0 = MU0 * C0


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        pp = ctypes.POINTER(_Problem)
        L.orc_time_step.restype = ctypes.c_double
        L.orc_time_step.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_omega.restype = ctypes.c_double
        L.orc_omega.argtypes = [pp]
        L.orc_material.argtypes = [ctypes.c_double] * 4 + [dp]
        L.orc_material_eps.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_pixel_coefficients.argtypes = [pp, u8p, ctypes.c_int32, dp, dp, dp]
        L.orc_cpml_profiles.argtypes = [pp, dp, dp]
        L.orc_incident.argtypes = [pp, dp, dp]
        L.orc_run.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                              ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.orc_gram.argtypes = [pp, dp]
        L.orc_spectra.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        L.orc_incident_sums.argtypes = [pp, dp, dp]
        L.orc_spectra_grad.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, dp]
        L.orc_step_adjoint.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_adjoint.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.orc_grad_chain.argtypes = [pp, u8p, ctypes.c_int32, dp, dp, dp, dp, dp]
        L.orc_edge_coefficients.argtypes = [pp, u8p, ctypes.c_int32, dp, dp, dp, dp, dp]
        L.orc_incident_te.argtypes = [pp, dp, dp]
        L.orc_run_te.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                 ctypes.c_int32, ctypes.c_int32, dp]
        L.orc_ade_coefficients.argtypes = [pp, ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.orc_incident_pulse.argtypes = [pp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_run_ade.argtypes = [pp, u8p, ctypes.c_int32, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.orc_spectra_pulse.argtypes = [pp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_incident_pulse_te.argtypes = [pp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_edge_model_coefficients.argtypes = [pp, u8p, ctypes.c_int32, dp, dp, dp, dp, dp]
        L.orc_run_te_ade.argtypes = [pp, u8p, ctypes.c_int32, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                     dp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n_pml", ctypes.c_int32),
                ("j_src", ctypes.c_int32), ("j_ref", ctypes.c_int32), ("j_trn", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("dft_start", ctypes.c_int32),
                ("aux_pad", ctypes.c_int32), ("aux_pml", ctypes.c_int32),
                ("aux_src_off", ctypes.c_int32), ("literal_orders", ctypes.c_int32),
                ("polarization", ctypes.c_int32),
                ("h", ctypes.c_double), ("courant", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("ramp_periods", ctypes.c_double), ("cpml_order", ctypes.c_double),
                ("cpml_sigma_fac", ctypes.c_double), ("cpml_alpha_fac", ctypes.c_double),
                ("cpml_kappa_max", ctypes.c_double)]


@dataclass
class Problem:
    """One monochromatic TMz run (Sec. 2.1-2.6).  Lengths in metres."""
    nx: int
    ny: int
    h: float
    lambda0: float
    n_steps: int
    n_pml: int = 16
    j_src: int = -1            # default: ny - n_pml - 8
    j_ref: int = -1            # default: ny - n_pml - 4
    j_trn: int = -1            # default: n_pml + 4
    courant: float = 0.99
    dft_start: int = -1        # default: n_steps - n_steps // 2
    ramp_periods: float = 5.0
    cpml_order: float = 3.0
    cpml_sigma_fac: float = 0.8
    cpml_alpha_fac: float = 0.05
    cpml_kappa_max: float = 1.0
    aux_pad: int = 64
    aux_pml: int = 128
    aux_src_off: int = 16
    literal_orders: int = 0
    polarization: int = 0      # 0: TMz (S, Ez monitored); 1: TEz (P, Ex monitored)

    def __post_init__(self):
        if self.j_src < 0:
            self.j_src = self.ny - self.n_pml - 8
        if self.j_ref < 0:
            self.j_ref = self.ny - self.n_pml - 4
        if self.j_trn < 0:
            self.j_trn = self.n_pml + 4
        if self.dft_start < 0:
            self.dft_start = self.n_steps - self.n_steps // 2

    def c(self) -> _Problem:
        d = asdict(self)
        return _Problem(**{k: d[k] for k, _ in _Problem._fields_})

    @property
    def dt(self) -> float:
        return time_step(self.h, self.courant)

    @property
    def omega(self) -> float:
        return 2.0 * np.pi * C0 / self.lambda0


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_f64(a, shape):
    """The C side writes doubles in place: refuse anything else."""
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags.c_contiguous and a.shape == shape):
        raise TypeError("expected a C-contiguous float64 array of shape %s" % (shape,))


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def time_step(h: float, courant: float) -> float:
    """CFL time step of Sec. 2.3 scaled by the Courant number S."""
    return lib().orc_time_step(h, courant)


def material(n: float, k: float, omega: float, dt: float):
    """Eqs. 1-2 and 17: returns (eps_r, sigma, Ce, Cb)."""
    out = np.zeros(4)
    lib().orc_material(n, k, omega, dt, _p(out))
    return tuple(out)


def material_eps(eps_r: float, sigma: float, dt: float):
    out = np.zeros(2)
    lib().orc_material_eps(eps_r, sigma, dt, _p(out))
    return tuple(out)


def pixel_coefficients(prob: Problem, labels: np.ndarray, nk: np.ndarray):
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    nk = np.ascontiguousarray(nk, dtype=np.float64).reshape(-1, 2)
    assert labels.shape == (prob.ny, prob.nx)
    assert int(labels.max()) < nk.shape[0]
    ce = np.empty(labels.shape)
    cb = np.empty(labels.shape)
    pc = prob.c()
    lib().orc_pixel_coefficients(ctypes.byref(pc), _u8(labels), nk.shape[0], _p(nk), _p(ce), _p(cb))
    return ce, cb


def cpml_profiles(prob: Problem):
    pe = np.zeros((prob.ny, 3))
    ph = np.zeros((prob.ny, 3))
    pc = prob.c()
    lib().orc_cpml_profiles(ctypes.byref(pc), _p(pe), _p(ph))
    return pe, ph


def incident(prob: Problem):
    """1D auxiliary-grid incident fields: (e_inc[n] at t=(n+1/2)dt, h_inc[n] at t=n dt)."""
    e = np.zeros(prob.n_steps)
    h = np.zeros(prob.n_steps)
    pc = prob.c()
    rc = lib().orc_incident(ctypes.byref(pc), _p(e), _p(h))
    if rc != 0:
        raise ValueError("orc_incident failed: %d" % rc)
    return e, h


@dataclass
class State:
    ez: np.ndarray
    hx: np.ndarray
    hy: np.ndarray
    pez: np.ndarray
    phx: np.ndarray

    @classmethod
    def zeros(cls, prob: Problem):
        z = lambda: np.zeros((prob.ny, prob.nx))
        return cls(z(), z(), z(), z(), z())

    def copy(self):
        return State(*(a.copy() for a in (self.ez, self.hx, self.hy, self.pez, self.phx)))


def run(prob: Problem, ce, cb, e_inc=None, h_inc=None, state: State | None = None,
        n_begin: int = 0, n_end: int | None = None, mon=None, history: bool = False):
    """Advance ``state`` through steps [n_begin, n_end) (eqs. 18-20 + CPML + TF/SF).

    Returns (state, mon, hist); mon is the [4][nx] monitor-sum array (eqs. 29-30),
    hist (if requested) holds Ez after each step."""
    if n_end is None:
        n_end = prob.n_steps
    if state is None:
        state = State.zeros(prob)
    if mon is None:
        mon = np.zeros((4, prob.nx))
    for a in (state.ez, state.hx, state.hy, state.pez, state.phx):
        _check_f64(a, (prob.ny, prob.nx))
    _check_f64(mon, (4, prob.nx))
    for a in (e_inc, h_inc):
        if a is not None:
            _check_f64(a, (prob.n_steps,))
    ce = np.ascontiguousarray(ce, dtype=np.float64)
    cb = np.ascontiguousarray(cb, dtype=np.float64)
    hist = np.zeros((n_end - n_begin, prob.ny, prob.nx)) if history else None
    null = ctypes.POINTER(ctypes.c_double)()
    pc = prob.c()
    rc = lib().orc_run(ctypes.byref(pc), _p(ce), _p(cb),
                       _p(e_inc) if e_inc is not None else null,
                       _p(h_inc) if h_inc is not None else null,
                       _p(state.ez), _p(state.hx), _p(state.hy), _p(state.pez), _p(state.phx),
                       n_begin, n_end, _p(mon), _p(hist) if history else null)
    if rc != 0:
        raise RuntimeError("orc_run failed: %d" % rc)
    return state, mon, hist


def gram(prob: Problem):
    g = np.zeros(3)
    pc = prob.c()
    lib().orc_gram(ctypes.byref(pc), _p(g))
    return g


def incident_sums(prob: Problem, e_inc):
    out = np.zeros(2)
    pc = prob.c()
    lib().orc_incident_sums(ctypes.byref(pc), _p(np.ascontiguousarray(e_inc)), _p(out))
    return out


def spectra(prob: Problem, mon, inc_sums):
    """Eqs. 31-34 with the tone fit and discrete-flux weights: (R, T, A, orders)."""
    nx = prob.nx
    out = np.zeros(3)
    w = np.zeros(nx)
    rp = np.zeros(nx)
    tp = np.zeros(nx)
    pc = prob.c()
    rc = lib().orc_spectra(ctypes.byref(pc), _p(np.ascontiguousarray(mon)), float(inc_sums[0]),
                           float(inc_sums[1]), _p(out), _p(w), _p(rp), _p(tp))
    if rc != 0:
        raise ValueError("orc_spectra failed: %d" % rc)
    m = np.arange(-((nx - 1) // 2), nx // 2 + 1)
    return out[0], out[1], out[2], dict(m=m, w=w, ref=rp, trn=tp)


def spectra_grad(prob: Problem, mon, inc_sums, dL_dR: float, dL_dT: float):
    d = np.zeros((4, prob.nx))
    pc = prob.c()
    rc = lib().orc_spectra_grad(ctypes.byref(pc), _p(np.ascontiguousarray(mon)), float(inc_sums[0]),
                                float(inc_sums[1]), dL_dR, dL_dT, _p(d))
    if rc != 0:
        raise ValueError("orc_spectra_grad failed")
    return d


def step_adjoint(prob: Problem, ce, cb, adj: State, ez_old=None, ez_new=None, gce=None, gcb=None):
    """Transpose of one source-free step, in place on ``adj``."""
    for a in (adj.ez, adj.hx, adj.hy, adj.pez, adj.phx, ce, cb):
        _check_f64(a, (prob.ny, prob.nx))
    null = ctypes.POINTER(ctypes.c_double)()
    pc = prob.c()
    lib().orc_step_adjoint(ctypes.byref(pc), _p(ce), _p(cb), _p(adj.ez), _p(adj.hx), _p(adj.hy),
                           _p(adj.pez), _p(adj.phx),
                           _p(ez_old) if ez_old is not None else null,
                           _p(ez_new) if ez_new is not None else null,
                           _p(gce) if gce is not None else null,
                           _p(gcb) if gcb is not None else null)
    return adj


def adjoint(prob: Problem, ce, cb, hist, dmon):
    """Reverse sweep of a whole run: per-pixel (dL/dCe, dL/dCb)."""
    gce = np.zeros((prob.ny, prob.nx))
    gcb = np.zeros((prob.ny, prob.nx))
    pc = prob.c()
    rc = lib().orc_adjoint(ctypes.byref(pc), _p(ce), _p(cb), _p(np.ascontiguousarray(hist)),
                           _p(np.ascontiguousarray(dmon)), _p(gce), _p(gcb))
    if rc != 0:
        raise RuntimeError("orc_adjoint failed")
    return gce, gcb


def grad_chain(prob: Problem, labels, nk, gce, gcb):
    """Per-label (dL/dn, dL/dk) and per-pixel dL/deps_r (sigma fixed)."""
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    nk = np.ascontiguousarray(nk, dtype=np.float64).reshape(-1, 2)
    gnk = np.zeros_like(nk)
    geps = np.zeros((prob.ny, prob.nx))
    pc = prob.c()
    lib().orc_grad_chain(ctypes.byref(pc), _u8(labels), nk.shape[0], _p(nk), _p(gce), _p(gcb),
                         _p(gnk), _p(geps))
    return gnk, geps


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (for timing on a
    given number of host cores)."""
    lib().orc_set_num_threads(int(n))


def simulate(prob: Problem, labels=None, nk=None, ce=None, cb=None, history=False, keep_state=True):
    """Full run from zero fields: returns dict with R, T, A, orders, monitors, fields."""
    if ce is None:
        ce, cb = pixel_coefficients(prob, labels, nk)
    e_inc, h_inc = incident(prob)
    state, mon, hist = run(prob, ce, cb, e_inc, h_inc, history=history)
    inc = incident_sums(prob, e_inc)
    R, T, A, orders = spectra(prob, mon, inc)
    out = dict(R=R, T=T, A=A, orders=orders, mon=mon, inc=inc, ce=ce, cb=cb,
               e_inc=e_inc, h_inc=h_inc)
    if keep_state:
        out["state"] = state
    if history:
        out["hist"] = hist
    return out


def gradient(prob: Problem, labels, nk, dL_dR: float = 1.0, dL_dT: float = 0.0):
    """Forward + discrete adjoint: (result, grad_nk[n_labels,2], grad_eps[ny,nx])."""
    res = simulate(prob, labels, nk, history=True)
    dmon = spectra_grad(prob, res["mon"], res["inc"], dL_dR, dL_dT)
    gce, gcb = adjoint(prob, res["ce"], res["cb"], res["hist"], dmon)
    gnk, geps = grad_chain(prob, labels, nk, gce, gcb)
    res.pop("hist")
    return res, gnk, geps, (gce, gcb)


# ---------------------------------------------------------------------------
# TEz (P polarisation): Hz at cell centres, Ex on bottom edges, Ey on left edges
# ---------------------------------------------------------------------------

def edge_coefficients(prob: Problem, labels: np.ndarray, nk: np.ndarray):
    """Per-edge (Ce, Cb) of Ex and Ey: averaged eps_r and sigma of the two cells
    an edge separates (reading: the paper does not state the edge rule)."""
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    nk = np.ascontiguousarray(nk, dtype=np.float64).reshape(-1, 2)
    assert labels.shape == (prob.ny, prob.nx)
    out = [np.empty(labels.shape) for _ in range(4)]
    pc = prob.c()
    lib().orc_edge_coefficients(ctypes.byref(pc), _u8(labels), nk.shape[0], _p(nk), *[_p(a) for a in out])
    return tuple(out)


def incident_te(prob: Problem):
    """TEz incident fields: (ex_inc[n] on edge j_src+1 at (n+1) dt, hz_inc[n] on row j_src at (n+1/2) dt)."""
    e = np.zeros(prob.n_steps)
    h = np.zeros(prob.n_steps)
    pc = prob.c()
    rc = lib().orc_incident_te(ctypes.byref(pc), _p(e), _p(h))
    if rc != 0:
        raise ValueError("orc_incident_te failed: %d" % rc)
    return e, h


@dataclass
class StateTE:
    hz: np.ndarray
    ex: np.ndarray
    ey: np.ndarray
    phz: np.ndarray
    pex: np.ndarray

    @classmethod
    def zeros(cls, prob: Problem):
        z = lambda: np.zeros((prob.ny, prob.nx))
        return cls(z(), z(), z(), z(), z())


def run_te(prob: Problem, coefs, e_inc=None, h_inc=None, state: StateTE | None = None,
           n_begin: int = 0, n_end: int | None = None, mon=None):
    """Advance a TEz state through steps [n_begin, n_end) (eqs. 14-16 + CPML + TF/SF)."""
    if n_end is None:
        n_end = prob.n_steps
    if state is None:
        state = StateTE.zeros(prob)
    if mon is None:
        mon = np.zeros((4, prob.nx))
    for a in (state.hz, state.ex, state.ey, state.phz, state.pex):
        _check_f64(a, (prob.ny, prob.nx))
    _check_f64(mon, (4, prob.nx))
    for a in (e_inc, h_inc):
        if a is not None:
            _check_f64(a, (prob.n_steps,))
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in coefs]
    for c in cs:
        _check_f64(c, (prob.ny, prob.nx))
    null = ctypes.POINTER(ctypes.c_double)()
    pc = prob.c()
    rc = lib().orc_run_te(ctypes.byref(pc), *[_p(c) for c in cs],
                          _p(e_inc) if e_inc is not None else null,
                          _p(h_inc) if h_inc is not None else null,
                          _p(state.hz), _p(state.ex), _p(state.ey), _p(state.phz), _p(state.pex),
                          n_begin, n_end, _p(mon))
    if rc != 0:
        raise RuntimeError("orc_run_te failed: %d" % rc)
    return state, mon


def simulate_te(prob: Problem, labels, nk):
    """Full TEz run from zero fields: dict with R, T, A, orders, monitors, state."""
    assert prob.polarization == 1
    coefs = edge_coefficients(prob, labels, nk)
    e_inc, h_inc = incident_te(prob)
    state, mon = run_te(prob, coefs, e_inc, h_inc)
    inc = incident_sums(prob, e_inc)
    R, T, A, orders = spectra(prob, mon, inc)
    return dict(R=R, T=T, A=A, orders=orders, mon=mon, inc=inc, coefs=coefs,
                e_inc=e_inc, h_inc=h_inc, state=state)


# ---------------------------------------------------------------------------
# Dispersive labels and broadband runs (Sec. 2.2's Lorentz-Drude alternative)
# ---------------------------------------------------------------------------

def ade_coefficients(prob: Problem, model: np.ndarray, n_poles: int):
    """Per-label (Ce, Cb, then alpha, xi, zeta per pole) of the polarisation
    ADE.  model[L] = (eps_inf, sigma, then a_p, w_p, g_p per pole)."""
    model = np.ascontiguousarray(model, dtype=np.float64).reshape(-1, 2 + 3 * n_poles)
    out = np.zeros_like(model)
    pc = prob.c()
    lib().orc_ade_coefficients(ctypes.byref(pc), model.shape[0], n_poles, _p(model), _p(out))
    return out


def incident_pulse(prob: Problem, tau: float, t0: float):
    """1D auxiliary-grid fields for the Gaussian-modulated pulse centred on
    prob.lambda0.  TMz: (e_inc[n] at (n+1/2) dt, h_inc[n] at n dt); TEz
    (prob.polarization = 1): (ex_inc[n] on edge j_src+1 at (n+1) dt,
    hz_inc[n] on row j_src at (n+1/2) dt)."""
    e = np.zeros(prob.n_steps)
    h = np.zeros(prob.n_steps)
    pc = prob.c()
    f = lib().orc_incident_pulse_te if prob.polarization else lib().orc_incident_pulse
    rc = f(ctypes.byref(pc), tau, t0, _p(e), _p(h))
    if rc != 0:
        raise ValueError("incident pulse failed: %d" % rc)
    return e, h


@dataclass
class StateADE(State):
    pol: np.ndarray = None       # [n_poles][2][ny][nx]: P^{n-1/2}, P^{n-3/2}

    @classmethod
    def zeros(cls, prob: Problem, n_poles: int = 1):
        z = lambda: np.zeros((prob.ny, prob.nx))
        return cls(z(), z(), z(), z(), z(), np.zeros((max(n_poles, 1), 2, prob.ny, prob.nx)))


def run_ade(prob: Problem, labels, coef, n_poles: int, lambdas, e_inc=None, h_inc=None,
            state: StateADE | None = None, n_begin: int = 0, n_end: int | None = None, mon=None):
    """Advance a TMz state with dispersive labels through steps [n_begin, n_end);
    mon[f][4][nx] receives the monitor sums at every wavelength of lambdas."""
    if n_end is None:
        n_end = prob.n_steps
    lambdas = np.ascontiguousarray(lambdas, dtype=np.float64)
    if state is None:
        state = StateADE.zeros(prob, n_poles)
    if mon is None:
        mon = np.zeros((len(lambdas), 4, prob.nx))
    for a in (state.ez, state.hx, state.hy, state.pez, state.phx):
        _check_f64(a, (prob.ny, prob.nx))
    _check_f64(state.pol, (max(n_poles, 1), 2, prob.ny, prob.nx))
    _check_f64(mon, (len(lambdas), 4, prob.nx))
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    assert labels.shape == (prob.ny, prob.nx) and int(labels.max()) < coef.shape[0]
    null = ctypes.POINTER(ctypes.c_double)()
    pc = prob.c()
    rc = lib().orc_run_ade(ctypes.byref(pc), _u8(labels), n_poles, _p(coef),
                           _p(e_inc) if e_inc is not None else null,
                           _p(h_inc) if h_inc is not None else null,
                           _p(state.ez), _p(state.hx), _p(state.hy), _p(state.pez), _p(state.phx),
                           _p(state.pol), n_begin, n_end, len(lambdas), _p(lambdas), _p(mon))
    if rc != 0:
        raise RuntimeError("orc_run_ade failed: %d" % rc)
    return state, mon


def pulse_transform(prob: Problem, e_inc, lam: float):
    """sum_n e_inc[n] e^{i w t_n} over the monitor window, t_n = (n+1/2) dt in
    TMz and (n+1) dt in TEz (the times of the monitored field)."""
    n = np.arange(prob.dft_start, prob.n_steps)
    t = (n + (1.0 if prob.polarization else 0.5)) * prob.dt
    w = 2.0 * np.pi * C0 / lam
    return complex(np.sum(e_inc[n] * np.cos(w * t)), np.sum(e_inc[n] * np.sin(w * t)))


def spectra_pulse(prob: Problem, lam: float, mon_f, inc: complex):
    out = np.zeros(3)
    pc = prob.c()
    rc = lib().orc_spectra_pulse(ctypes.byref(pc), lam, _p(np.ascontiguousarray(mon_f)), inc.real, inc.imag,
                                 _p(out))
    if rc != 0:
        raise ValueError("orc_spectra_pulse failed: %d" % rc)
    return out


@dataclass
class StateTEADE(StateTE):
    polx: np.ndarray = None      # Ex edges: [2 sides][n_poles][2][ny][nx] = P^n, P^{n-1}
    poly: np.ndarray = None      # Ey edges, likewise

    @classmethod
    def zeros(cls, prob: Problem, n_poles: int = 1):
        z = lambda: np.zeros((prob.ny, prob.nx))
        zp = lambda: np.zeros((2, max(n_poles, 1), 2, prob.ny, prob.nx))
        return cls(z(), z(), z(), z(), z(), zp(), zp())


def edge_model_coefficients(prob: Problem, labels, model, n_poles: int):
    """Per-edge (Ce, Cb) of Ex and Ey for dispersive labels: eq. 17 at the mean
    eps_inf and mean sigma of the two cells an edge separates (the edge's
    permittivity is the mean of theirs at every frequency)."""
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    model = np.ascontiguousarray(model, dtype=np.float64).reshape(-1, 2 + 3 * n_poles)
    assert labels.shape == (prob.ny, prob.nx) and int(labels.max()) < model.shape[0]
    out = [np.empty(labels.shape) for _ in range(4)]
    pc = prob.c()
    lib().orc_edge_model_coefficients(ctypes.byref(pc), _u8(labels), n_poles, _p(model), *[_p(a) for a in out])
    return tuple(out)


def run_te_ade(prob: Problem, labels, coef, edge_coefs, n_poles: int, lambdas, e_inc=None, h_inc=None,
               state: StateTEADE | None = None, n_begin: int = 0, n_end: int | None = None, mon=None):
    """Advance a TEz state with dispersive labels through steps [n_begin, n_end).
    Each edge's polarisation is half the sum of its two cells' pole responses
    to the edge field; mon[f][4][nx] receives the Ex monitor sums at every
    wavelength of lambdas."""
    if n_end is None:
        n_end = prob.n_steps
    lambdas = np.ascontiguousarray(lambdas, dtype=np.float64)
    if state is None:
        state = StateTEADE.zeros(prob, n_poles)
    if mon is None:
        mon = np.zeros((len(lambdas), 4, prob.nx))
    for a in (state.hz, state.ex, state.ey, state.phz, state.pex):
        _check_f64(a, (prob.ny, prob.nx))
    for a in (state.polx, state.poly):
        _check_f64(a, (2, max(n_poles, 1), 2, prob.ny, prob.nx))
    _check_f64(mon, (len(lambdas), 4, prob.nx))
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    assert labels.shape == (prob.ny, prob.nx) and int(labels.max()) < coef.shape[0]
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in edge_coefs]
    for c in cs:
        _check_f64(c, (prob.ny, prob.nx))
    null = ctypes.POINTER(ctypes.c_double)()
    pc = prob.c()
    rc = lib().orc_run_te_ade(ctypes.byref(pc), _u8(labels), n_poles, _p(coef), *[_p(c) for c in cs],
                              _p(e_inc) if e_inc is not None else null,
                              _p(h_inc) if h_inc is not None else null,
                              _p(state.hz), _p(state.ex), _p(state.ey), _p(state.phz), _p(state.pex),
                              _p(state.polx), _p(state.poly), n_begin, n_end, len(lambdas), _p(lambdas), _p(mon))
    if rc != 0:
        raise RuntimeError("orc_run_te_ade failed: %d" % rc)
    return state, mon


def simulate_pulse(prob: Problem, labels, model, n_poles: int, lambdas, tau: float, t0: float):
    """Full broadband run from zero fields (dft_start should be 0), TMz or TEz
    by prob.polarization: per-wavelength R, T, A arrays plus monitors,
    incident transforms and final state."""
    coef = ade_coefficients(prob, model, n_poles)
    e_inc, h_inc = incident_pulse(prob, tau, t0)
    edge = None
    if prob.polarization:
        edge = edge_model_coefficients(prob, labels, model, n_poles)
        state, mon = run_te_ade(prob, labels, coef, edge, n_poles, lambdas, e_inc, h_inc)
    else:
        state, mon = run_ade(prob, labels, coef, n_poles, lambdas, e_inc, h_inc)
    inc = [pulse_transform(prob, e_inc, lam) for lam in lambdas]
    rta = np.array([spectra_pulse(prob, lam, mon[f], inc[f]) for f, lam in enumerate(lambdas)])
    return dict(R=rta[:, 0], T=rta[:, 1], A=rta[:, 2], mon=mon, inc=np.array(inc), coef=coef, edge=edge,
                e_inc=e_inc, h_inc=h_inc, state=state)
