"""Python binding of libfdtd.so (the C ABI declared in include/fdtd.h).

Argument marshalling only: every step of the FDTD path runs in the library's
HIP kernels.  PyTorch supplies the HIP stream (and device tensors for the
per-pixel gradient).  The library must be built (``__graft_entry__.build()``);
nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

FDTD_OK = 0
ERRORS = {-1: "FDTD_E_INVAL", -2: "FDTD_E_MATERIAL", -3: "FDTD_E_NOMEM", -4: "FDTD_E_HIP",
          -5: "FDTD_E_STATE", -6: "FDTD_E_UNSTABLE"}


class FdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERRORS.get(code, str(code)), msg))
        self.code = code


class _Instance(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n_pml", ctypes.c_int32),
                ("j_src", ctypes.c_int32), ("j_ref", ctypes.c_int32), ("j_trn", ctypes.c_int32),
                ("n_labels", ctypes.c_int32), ("polarization", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_freqs", ctypes.c_int32),
                ("dx", ctypes.c_double), ("courant", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("labels", ctypes.POINTER(ctypes.c_uint8)), ("nk", ctypes.POINTER(ctypes.c_double)),
                ("n_poles", ctypes.c_int32), ("_reserved", ctypes.c_int32),
                ("model", ctypes.POINTER(ctypes.c_double)), ("lambdas", ctypes.POINTER(ctypes.c_double)),
                ("pulse_tau", ctypes.c_double), ("pulse_t0", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("dft_start", ctypes.c_int32),
                ("ramp_periods", ctypes.c_double), ("kernel", ctypes.c_int32),
                ("t_block", ctypes.c_int32), ("band_rows", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32), ("literal_orders", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("adj_t_block", ctypes.c_int32),
                ("special_rows", ctypes.c_int32), ("adj_band_rows", ctypes.c_int32),
                ("bulk_columns", ctypes.c_int32), ("_reserved", ctypes.c_int32 * 2)]


_lib = None


def load():
    """Loads libfdtd.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libfdtd.so is not built; run __graft_entry__.build() first (%s)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.fdtd_create.argtypes = [ctypes.POINTER(_Instance), i32, ctypes.POINTER(_Opts), vp, ctypes.POINTER(vp)]
    L.fdtd_run.argtypes = [vp, i32]
    L.fdtd_step.argtypes = [vp, i32]
    L.fdtd_step_noalloc.argtypes = [vp, i32]
    L.fdtd_reset.argtypes = [vp]
    L.fdtd_steps_done.argtypes = [vp, ip]
    L.fdtd_spectra.argtypes = [vp, dp, dp, dp]
    L.fdtd_broadband_spectra.argtypes = [vp, i32, dp, dp, dp]
    L.fdtd_orders.argtypes = [vp, i32, i32, ip, dp, dp, dp, ip]
    L.fdtd_fields.argtypes = [vp, i32, fp, fp, fp]
    L.fdtd_monitors.argtypes = [vp, i32, dp]
    L.fdtd_set_fields.argtypes = [vp, i32, fp, fp, fp, fp, fp]
    L.fdtd_backward.argtypes = [vp, dp, dp, dp, fp]
    L.fdtd_get_config.argtypes = [vp, ip, ip, ip, ip, i64p, i64p, ip, ip]
    L.fdtd_autotune.argtypes = [vp, i32, dp]
    L.fdtd_set_profiling.argtypes = [vp, i32]
    L.fdtd_kernel_time.argtypes = [vp, dp, i64p]
    L.fdtd_destroy.argtypes = [vp]
    L.fdtd_destroy.restype = None
    L.fdtd_last_error.argtypes = [vp]
    L.fdtd_last_error.restype = ctypes.c_char_p
    L.fdtd_strerror.argtypes = [ctypes.c_int]
    L.fdtd_strerror.restype = ctypes.c_char_p
    L.fdtd_combine_spectra.argtypes = [dp, dp, i32, ip, i32, dp, dp, dp]
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a is not None else ctypes.POINTER(ctypes.c_float)()


def current_stream():
    """The current torch HIP stream as a raw handle (None without a GPU)."""
    import torch
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


@dataclass
class Options:
    n_steps: int
    dft_start: int = 0
    ramp_periods: float = 5.0
    kernel: int = 0
    t_block: int = 0
    band_rows: int = 0
    checkpoint_every: int = 0
    literal_orders: int = 0
    use_graph: int = 1
    adj_t_block: int = 0
    special_rows: int = 0
    adj_band_rows: int = 0
    bulk_columns: int = 0

    def c(self) -> _Opts:
        o = _Opts()
        for k, _ in _Opts._fields_:
            if k != "_reserved":
                setattr(o, k, getattr(self, k))
        return o


class Simulation:
    """A batch of monochromatic TMz runs on the GPU (one fdtd_ctx).

    instances: objects with labels (ny, nx) uint8, nk (n_labels, 2), dx,
    lambda0, n_pml, courant, the rows j_src, j_ref, j_trn and optionally
    polarization (0 TMz, 1 TEz) (leafgen.Instance).  For TEz instances
    fields() returns (Hz, Ex, Ey) and set_fields takes them in that order.

    run_steps: optional per-instance run lengths (each in 1..opts.n_steps, the
    longest equal to it).  A shorter instance leaves the batched launches at
    its own count and its monitor window is the last half of its own run.

    A broadband instance (TMz) also has ``lambdas`` (monitor wavelengths),
    ``model`` ((n_labels, 2 + 3 n_poles): eps_inf, sigma, then a_p, w_p, g_p
    per pole), ``pulse_tau`` and ``pulse_t0``; its lambda0 is the pulse's
    centre and nk is not used (see broadband_spectra and pulse_for_band)."""

    def __init__(self, instances, opts: Options, stream="current", run_steps=None):
        self.lib = load()
        self.instances = list(instances)
        self.opts = opts
        if run_steps is not None and len(run_steps) != len(self.instances):
            raise ValueError("run_steps needs one entry per instance")
        if stream == "current":
            stream = current_stream()
        arr = (_Instance * len(self.instances))()
        self._keep = []
        for k, inst in enumerate(self.instances):
            lab = np.ascontiguousarray(inst.labels, dtype=np.uint8)
            a = arr[k]
            lambdas = getattr(inst, "lambdas", None)
            if lambdas is not None:
                n_poles = int(getattr(inst, "n_poles", 0))
                model = np.ascontiguousarray(inst.model, dtype=np.float64).reshape(-1, 2 + 3 * n_poles)
                lams = np.ascontiguousarray(lambdas, dtype=np.float64).ravel()
                self._keep += [model, lams]
                a.n_freqs, a.n_poles = len(lams), n_poles
                a.model, a.lambdas = _dp(model), _dp(lams)
                a.pulse_tau, a.pulse_t0 = float(inst.pulse_tau), float(inst.pulse_t0)
                n_labels = model.shape[0]
            else:
                nk = np.ascontiguousarray(inst.nk, dtype=np.float64).reshape(-1, 2)
                self._keep.append(nk)
                a.nk = _dp(nk)
                n_labels = nk.shape[0]
            self._keep.append(lab)
            a.ny, a.nx = lab.shape
            a.n_pml = inst.n_pml
            a.j_src, a.j_ref, a.j_trn = inst.j_src, inst.j_ref, inst.j_trn
            a.n_labels = n_labels
            a.polarization = int(getattr(inst, "polarization", 0))
            a.n_steps = int(run_steps[k]) if run_steps is not None else 0
            a.dx, a.courant, a.lambda0 = inst.dx, inst.courant, inst.lambda0
            a.labels = lab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self._ctx = ctypes.c_void_p()
        o = opts.c()
        rc = self.lib.fdtd_create(arr, len(self.instances), ctypes.byref(o),
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(self._ctx))
        self._keep = []
        if rc != FDTD_OK:
            raise FdtdError(rc, self.lib.fdtd_last_error(None).decode())

    # -- helpers --
    def _check(self, rc):
        if rc != FDTD_OK:
            raise FdtdError(rc, self.lib.fdtd_last_error(self._ctx).decode())

    def close(self):
        if self._ctx:
            self.lib.fdtd_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- C ABI --
    def run(self, record: bool = False):
        self._check(self.lib.fdtd_run(self._ctx, 1 if record else 0))

    def step(self, n: int):
        self._check(self.lib.fdtd_step(self._ctx, n))

    def step_noalloc(self, n: int):
        """fdtd_step with the work-item lists staged in the library's fixed
        device array (allocates no device memory)."""
        self._check(self.lib.fdtd_step_noalloc(self._ctx, n))

    def reset(self):
        self._check(self.lib.fdtd_reset(self._ctx))

    def steps_done(self) -> int:
        n = ctypes.c_int32()
        self._check(self.lib.fdtd_steps_done(self._ctx, ctypes.byref(n)))
        return n.value

    def spectra(self):
        k = len(self.instances)
        R, T, A = np.zeros(k), np.zeros(k), np.zeros(k)
        self._check(self.lib.fdtd_spectra(self._ctx, _dp(R), _dp(T), _dp(A)))
        return R, T, A

    def broadband_spectra(self, inst: int = 0):
        """(R, T, A) of a broadband instance at each of its monitor wavelengths."""
        nf = len(self.instances[inst].lambdas)
        R, T, A = np.zeros(nf), np.zeros(nf), np.zeros(nf)
        self._check(self.lib.fdtd_broadband_spectra(self._ctx, inst, _dp(R), _dp(T), _dp(A)))
        return R, T, A

    def orders(self, inst: int = 0):
        nx = self.instances[inst].labels.shape[1]
        m = np.zeros(nx, np.int32)
        w, rp, tp = np.zeros(nx), np.zeros(nx), np.zeros(nx)
        n = ctypes.c_int32()
        self._check(self.lib.fdtd_orders(self._ctx, inst, nx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                         _dp(w), _dp(rp), _dp(tp), ctypes.byref(n)))
        k = n.value
        return dict(m=m[:k], w=w[:k], ref=rp[:k], trn=tp[:k])

    def fields(self, inst: int = 0):
        ny, nx = self.instances[inst].labels.shape
        ez, hx, hy = (np.zeros((ny, nx), np.float32) for _ in range(3))
        self._check(self.lib.fdtd_fields(self._ctx, inst, _fp(ez), _fp(hx), _fp(hy)))
        return ez, hx, hy

    def monitors(self, inst: int = 0):
        """Monitor sums [4][nx]; a broadband instance gives [n_freqs][4][nx]."""
        it = self.instances[inst]
        nx = it.labels.shape[1]
        lambdas = getattr(it, "lambdas", None)
        nf = len(lambdas) if lambdas is not None else 0
        mon = np.zeros((max(1, nf), 4, nx))
        self._check(self.lib.fdtd_monitors(self._ctx, inst, _dp(mon)))
        return mon if nf else mon[0]

    def set_fields(self, inst: int, ez=None, hx=None, hy=None, psi_ez=None, psi_hx=None):
        cv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        arrs = [cv(a) for a in (ez, hx, hy, psi_ez, psi_hx)]
        self._check(self.lib.fdtd_set_fields(self._ctx, inst, *[_fp(a) for a in arrs]))

    def backward(self, dL_dR, dL_dT=None, want_eps: bool = True):
        """Returns (grad_nk list of (n_labels, 2) arrays, grad_eps list of torch
        tensors (ny, nx) on the device, or None)."""
        import torch
        k = len(self.instances)
        dR = np.ascontiguousarray(np.broadcast_to(np.asarray(dL_dR, np.float64), (k,)))
        dT = None if dL_dT is None else np.ascontiguousarray(np.broadcast_to(np.asarray(dL_dT, np.float64), (k,)))
        nl = [np.asarray(i.nk).reshape(-1, 2).shape[0] for i in self.instances]
        gnk = np.zeros(2 * sum(nl))
        geps = None
        ptr = ctypes.POINTER(ctypes.c_float)()
        if want_eps:
            total = sum(int(np.prod(i.labels.shape)) for i in self.instances)
            geps = torch.empty(total, dtype=torch.float32, device="cuda")
            ptr = ctypes.cast(ctypes.c_void_p(geps.data_ptr()), ctypes.POINTER(ctypes.c_float))
        self._check(self.lib.fdtd_backward(self._ctx, _dp(dR), _dp(dT) if dT is not None else None, _dp(gnk), ptr))
        out_nk, off = [], 0
        for n in nl:
            out_nk.append(gnk[off:off + 2 * n].reshape(n, 2))
            off += 2 * n
        out_eps = None
        if want_eps:
            out_eps, off = [], 0
            for i in self.instances:
                ny, nx = i.labels.shape
                out_eps.append(geps[off:off + ny * nx].view(ny, nx))
                off += ny * nx
        return out_nk, out_eps

    def config(self):
        k, t, b, it, sb, bc = (ctypes.c_int32() for _ in range(6))
        nb, lc = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.fdtd_get_config(self._ctx, ctypes.byref(k), ctypes.byref(t), ctypes.byref(b),
                                             ctypes.byref(it), ctypes.byref(nb), ctypes.byref(lc), ctypes.byref(sb),
                                             ctypes.byref(bc)))
        return dict(kernel=k.value, t_block=t.value, band_rows=b.value, items=it.value, device_bytes=nb.value,
                    lean_cells=lc.value, special_rows=sb.value, bulk_columns=bc.value)

    def autotune(self, trial_steps: int = 0) -> float:
        r = ctypes.c_double()
        self._check(self.lib.fdtd_autotune(self._ctx, trial_steps, ctypes.byref(r)))
        return r.value

    def set_profiling(self, on, every: int = 1):
        """Time the bulk kernel: on=False turns timing off; otherwise every
        `every`-th launch is bracketed by HIP events (kernel_time averages
        over the timed launches)."""
        self._check(self.lib.fdtd_set_profiling(self._ctx, max(1, int(every)) if on else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.fdtd_kernel_time(self._ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def combine_spectra(R, T, group, n_groups: int):
    """fdtd_combine_spectra: per group, the mean R and T of its runs and
    A = 1 - R - T of the means (Sec. 2.1 and 4.2).  R, T and group are
    sequences of one entry per run; returns three arrays of n_groups."""
    L = load()
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    T = np.ascontiguousarray(T, dtype=np.float64).ravel()
    g = np.ascontiguousarray(group, dtype=np.int32).ravel()
    if not (len(R) == len(T) == len(g)):
        raise ValueError("R, T and group need one entry per run")
    out = [np.zeros(int(n_groups)) for _ in range(3)]
    rc = L.fdtd_combine_spectra(_dp(R), _dp(T), len(R), g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                int(n_groups), *[_dp(a) for a in out])
    if rc != FDTD_OK:
        raise FdtdError(rc, L.fdtd_last_error(None).decode())
    return tuple(out)


def unpolarized(tm, te):
    """Unpolarised spectra: the library's mean of the TMz and TEz results of
    the same wavelength (the reading of "results are later combined",
    Sec. 2.1).  tm, te are (R, T, A) tuples of equal-length arrays; returns
    (R, T, A)."""
    n = len(np.atleast_1d(tm[0]))
    groups = np.concatenate([np.arange(n), np.arange(n)])
    return combine_spectra(np.concatenate([np.atleast_1d(tm[0]), np.atleast_1d(te[0])]),
                           np.concatenate([np.atleast_1d(tm[1]), np.atleast_1d(te[1])]), groups, n)


C0 = 299792458.0


def pulse_for_band(lam_min: float, lam_max: float, edge: float = 3.0, delay: float = 4.0):
    """A Gaussian-modulated pulse for a broadband run covering [lam_min, lam_max]:
    returns (lambda0, tau, t0) with the centre frequency midway between the band
    edges, the spectrum down to exp(-edge) of its peak at the edges, and the
    peak delay*tau after the start."""
    wlo, whi = 2 * np.pi * C0 / lam_max, 2 * np.pi * C0 / lam_min
    tau = 4.0 * np.sqrt(edge) / (whi - wlo)
    return 2 * np.pi * C0 / (0.5 * (wlo + whi)), tau, delay * tau

