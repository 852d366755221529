"""The C ABI without a GPU: libfdtd.so loads, exports every entry point that
include/fdtd.h declares, and rejects bad inputs on the host (fdtd_create
validates everything before its first HIP call, so these run anywhere)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_17132_amd import fdtd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdtd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const\s+char\s*\*)\s*(fdtd_\w+)\s*\(", text, flags=re.M)
    assert len(names) == 21, names
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fdtd.LIB_PATH):
        pytest.skip("libfdtd.so not built")
    return fdtd.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", fdtd.LIB_PATH], capture_output=True, text=True)
    if out.returncode == 0:
        exported = {line.split()[-1] for line in out.stdout.splitlines() if line.strip()}
        missing = [n for n in names if n not in exported]
        assert not missing, missing
        # nothing else with the library prefix leaks out of the ABI
        extra = sorted(e for e in exported if e.startswith("fdtd_") and e not in names)
        assert not extra, extra


def test_strerror_names_every_status(lib):
    texts = [lib.fdtd_strerror(c).decode() for c in [0] + sorted(fdtd.ERRORS)]
    assert all(texts) and len(set(texts)) == len(texts)
    assert lib.fdtd_strerror(-99).decode() == "unknown status"


def test_null_context_calls_are_rejected(lib):
    n = ctypes.c_int32()
    assert lib.fdtd_run(None, 0) == -1
    assert lib.fdtd_step(None, 1) == -1
    assert lib.fdtd_steps_done(None, ctypes.byref(n)) == -1
    lib.fdtd_destroy(None)  # documented no-op


class Inst:
    """A valid small instance; tests break one field at a time."""

    def __init__(self, **kw):
        self.labels = np.zeros((64, 32), np.uint8)
        self.labels[24:40] = 1
        self.nk = np.array([[1.0, 0.0], [1.5, 0.01]])
        self.dx, self.lambda0, self.courant, self.n_pml = 20e-9, 600e-9, 0.99, 8
        self.j_trn, self.j_src, self.j_ref = 12, 48, 52
        for k, v in kw.items():
            setattr(self, k, v)


def create(insts, run_steps=None, **opts):
    o = dict(n_steps=100)
    o.update(opts)
    try:
        sim = fdtd.Simulation(insts, fdtd.Options(**o), stream=None, run_steps=run_steps)
    except fdtd.FdtdError as e:
        return e.code, str(e)
    sim.close()
    return 0, ""


def bad(**kw):
    return [Inst(**kw)]


CASES = [
    ("courant above one", bad(courant=1.05), {}, -1),
    ("courant zero", bad(courant=0.0), {}, -1),
    ("negative dx", bad(dx=-1e-9), {}, -1),
    ("wavelength below cutoff", bad(lambda0=30e-9), {}, -1),
    ("rows out of order", bad(j_ref=40), {}, -1),
    ("transmission row in the layer", bad(j_trn=8), {}, -1),
    ("reflection row in the layer", bad(j_ref=55), {}, -1),
    ("no absorbing layer", bad(n_pml=0, j_trn=4), {}, -1),
    ("absorbing layer too deep", bad(n_pml=65), {}, -1),
    ("grid too short", bad(labels=np.zeros((20, 32), np.uint8), j_trn=9, j_src=10, j_ref=11), {}, -1),
    ("no steps", bad(), dict(n_steps=0), -1),
    ("monitor window of one step", bad(), dict(dft_start=99), -1),
    ("t_block 9", bad(), dict(t_block=9), -1),
    ("t_block above 12", bad(), dict(t_block=14), -1),
    ("adj_t_block odd above 8", bad(), dict(adj_t_block=9), -1),
    ("adj_t_block above 12", bad(), dict(adj_t_block=14), -1),
    ("unknown kernel", bad(), dict(kernel=2), -1),
    ("special band of 17 rows", bad(), dict(special_rows=17), -1),
    ("negative special band", bad(), dict(special_rows=-1), -1),
    ("bulk items of 128 columns", bad(), dict(bulk_columns=128), -1),
    ("negative bulk columns", bad(), dict(bulk_columns=-1), -1),
    ("eps_r below one", bad(nk=np.array([[1.0, 0.0], [1.0, 0.5]])), {}, -2),
    ("negative k", bad(nk=np.array([[1.0, 0.0], [1.5, -0.01]])), {}, -2),
    ("non-finite n", bad(nk=np.array([[1.0, 0.0], [np.nan, 0.0]])), {}, -2),
    ("label beyond table", bad(nk=np.array([[1.0, 0.0]])), {}, -2),
    ("matter on the source row", bad(j_src=30, j_ref=50), {}, -2),
    ("matter on the transmission row", bad(j_trn=24), {}, -2),
    ("lossy air around the structure", bad(nk=np.array([[1.0, 1e-6], [1.5, 0.01]])), {}, -2),
]


@pytest.mark.parametrize("name,insts,opts,code", CASES, ids=[c[0] for c in CASES])
def test_create_rejects_bad_input_before_touching_the_gpu(lib, name, insts, opts, code):
    rc, msg = create(insts, **opts)
    assert rc == code, (rc, msg)
    assert msg  # fdtd_last_error(NULL) carries the reason


@pytest.mark.parametrize("run_steps,opts,what", [
    ([100, 120], {}, "n_steps must be in"),
    ([100, -1], {}, "n_steps must be in"),
    ([60, 80], {}, "longest instance"),
    ([100, 3], {}, "monitor window"),
    ([100, 50], dict(dft_start=60), "monitor window"),
])
def test_per_instance_run_lengths_are_validated(lib, run_steps, opts, what):
    rc, msg = create([Inst(), Inst()], run_steps=run_steps, **opts)
    assert rc == -1 and what in msg, msg


def broadband(**kw):
    """A valid broadband instance (one Lorentz pole); tests break one field."""
    wp = 2 * np.pi * 299792458.0 / 400e-9
    d = dict(lambdas=np.array([500e-9, 600e-9]), n_poles=1, pulse_tau=3e-15, pulse_t0=1.2e-14,
             model=np.array([[1.0, 0.0, 0.0, 0.0, 0.0], [2.0, 0.0, 0.3 * wp * wp, wp, 0.1 * wp]]))
    d.update(kw)
    return [Inst(**d)]


BB_CASES = [
    ("TEz with 17 labels", broadband(polarization=1, model=np.vstack([[1.0, 0, 0, 0, 0]] + [[2.0, 0, 0, 0, 0]] * 16)),
     "16 labels"),
    ("three poles", broadband(n_poles=3, model=np.zeros((2, 11))), "n_poles"),
    ("eps_inf below one", broadband(model=np.array([[1.0, 0, 0, 0, 0], [0.9, 0, 0, 0, 0]])), "eps_inf"),
    ("negative sigma", broadband(model=np.array([[1.0, 0, 0, 0, 0], [2.0, -1.0, 0, 0, 0]])), "sigma"),
    ("negative damping", broadband(model=np.array([[1.0, 0, 0, 0, 0], [2.0, 0, 1e30, 1e15, -1.0]])), "pole"),
    ("pole above 1/dt", broadband(model=np.array([[1.0, 0, 0, 0, 0], [2.0, 0, 1e30, 1e18, 0.0]])), "1/dt"),
    ("non-finite model", broadband(model=np.array([[1.0, 0, 0, 0, 0], [np.nan, 0, 0, 0, 0]])), "non-finite"),
    ("dispersive monitor row", broadband(model=np.array([[1.0, 0, 1.0, 0, 0], [2.0, 0, 0, 0, 0]])), "vacuum"),
    ("monitor wavelength below cutoff", broadband(lambdas=np.array([500e-9, 30e-9])), "cutoff"),
    ("zero tau", broadband(pulse_tau=0.0), "pulse_tau"),
]


@pytest.mark.parametrize("name,insts,what", BB_CASES, ids=[c[0] for c in BB_CASES])
def test_broadband_inputs_are_validated(lib, name, insts, what):
    rc, msg = create(insts)
    assert rc in (-1, -2) and what in msg, (rc, msg)


def test_second_instance_is_named_in_the_error(lib):
    rc, msg = create([Inst(), Inst(courant=2.0)])
    assert rc == -1 and "instance 1" in msg


def test_empty_batch_is_rejected(lib):
    out = ctypes.c_void_p()
    o = fdtd.Options(n_steps=10).c()
    rc = lib.fdtd_create(None, 0, ctypes.byref(o), None, ctypes.byref(out))
    assert rc == -1 and not out.value


def _combine(lib, R, T, group, n_groups):
    R = np.ascontiguousarray(R, np.float64)
    T = np.ascontiguousarray(T, np.float64)
    g = np.ascontiguousarray(group, np.int32)
    out = [np.full(n_groups, -7.0) for _ in range(3)]
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = lib.fdtd_combine_spectra(dp(R), dp(T), len(R), g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  n_groups, *[dp(a) for a in out])
    return rc, out


def test_combine_spectra_averages_groups_on_the_host(lib):
    """Slices x polarisations of two wavelengths in one call (no context, no
    device): each group's mean R and T, A = 1 - R - T of the means."""
    R = [0.10, 0.30, 0.20, 0.05, 0.15, 0.40]
    T = [0.50, 0.40, 0.60, 0.70, 0.65, 0.45]
    group = [0, 1, 0, 1, 0, 1]
    rc, (Ro, To, Ao) = _combine(lib, R, T, group, 2)
    assert rc == 0
    assert Ro[0] == pytest.approx(0.15, abs=1e-15) and To[0] == pytest.approx(0.5833333333333334, abs=1e-15)
    assert Ro[1] == pytest.approx(0.25, abs=1e-15) and To[1] == pytest.approx(0.5166666666666667, abs=1e-15)
    assert np.allclose(Ao, 1.0 - Ro - To, rtol=0, atol=1e-15)
    # the Python binding routes through the same call
    r2, t2, a2 = fdtd.combine_spectra(R, T, group, 2)
    assert np.array_equal(r2, Ro) and np.array_equal(t2, To) and np.array_equal(a2, Ao)
    ru, tu, au = fdtd.unpolarized((np.array([0.1, 0.2]), np.array([0.5, 0.6]), None),
                                  (np.array([0.3, 0.0]), np.array([0.4, 0.7]), None))
    assert np.allclose(ru, [0.2, 0.1]) and np.allclose(tu, [0.45, 0.65]) and np.allclose(au, [0.35, 0.25])


@pytest.mark.parametrize("R,T,group,n_groups,what", [
    ([0.1, 0.2], [0.5, 0.5], [0, 2], 2, "group out of range"),
    ([0.1, 0.2], [0.5, 0.5], [0, -1], 2, "group out of range"),
    ([0.1, 0.2], [0.5, 0.5], [0, 0], 2, "no runs"),
    ([0.1, np.nan], [0.5, 0.5], [0, 1], 2, "non-finite"),
    ([0.1, 0.2], [0.5, np.inf], [0, 1], 2, "non-finite"),
])
def test_combine_spectra_rejects_bad_groups(lib, R, T, group, n_groups, what):
    rc, out = _combine(lib, R, T, group, n_groups)
    assert rc == -1 and what in lib.fdtd_last_error(None).decode()
    assert all(np.all(a == -7.0) for a in out)       # nothing written


def test_field_set_size_limit_follows_the_layout(lib):
    """An instance's field set (Ez, Hx, Hy and both layer arrays, 256-byte
    aligned) must not exceed 2 GiB, the range of the kernels' 32-bit buffer
    offsets.  At nx = 8192 (pitch 8192) and 64 layer cells a set takes
    3 * 32768 ny + 2 * 129 * 32768 bytes: ny = 21759 fits (2147450880 bytes),
    ny = 21760 does not (2147549184)."""
    n_pml = 64
    for ny, too_big in [(21759, False), (21760, True)]:
        labels = np.zeros((ny, 8192), np.uint8)
        inst = Inst(labels=labels, nk=np.array([[1.0, 0.0]]), n_pml=n_pml, j_trn=n_pml + 4, j_src=ny - n_pml - 8,
                    j_ref=ny - n_pml - 4)
        rc, msg = create([inst], n_steps=10)
        if too_big:
            assert rc == -1 and "2 GiB" in msg, (ny, rc, msg)
        else:
            assert "2 GiB" not in msg and rc != -1 and rc != -2, (ny, rc, msg)
        del labels, inst
