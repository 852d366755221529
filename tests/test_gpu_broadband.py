"""Broadband runs on the GPU (Sec. 2.2's Lorentz-Drude alternative): dispersive
labels stepped through their polarisation ADEs, a pulsed source and monitors
at many wavelengths, against the FP64 oracle's broadband path on the same
seeded inputs (fields within 1e-3 relative L2, per-wavelength monitors within
1e-3, R and T within 1e-4), and batched with monochromatic instances; in TMz
and in TEz (edge permittivity the mean of its two cells')."""
from types import SimpleNamespace

import numpy as np
import pytest

import leafgen as LG
import oracle as O
from parity_util import oracle_fields_normalised, rel_l2

pytestmark = pytest.mark.gpu

C0 = 299792458.0


def lorentz(eps_inf, d_eps, lam_p, gamma_rel, sigma=0.0):
    wp = 2 * np.pi * C0 / lam_p
    return [eps_inf, sigma, d_eps * wp * wp, wp, gamma_rel * wp]


def bb_instance(fdtd, labels, model, n_poles, lams, steps, dx=20e-9, n_pml=16):
    ny = labels.shape[0]
    lam0, tau, t0 = fdtd.pulse_for_band(min(lams), max(lams))
    return SimpleNamespace(labels=labels, model=np.asarray(model, float), n_poles=n_poles,
                           lambdas=np.asarray(lams, float), pulse_tau=tau, pulse_t0=t0, lambda0=lam0, dx=dx,
                           courant=0.99, n_pml=n_pml, j_src=ny - n_pml - 8, j_ref=ny - n_pml - 4, j_trn=n_pml + 4,
                           n_steps=steps)


def oracle_bb(inst, n_mid):
    """The oracle's broadband run, with the fields after n_mid steps (the pulse
    has left the domain by the end of the run)."""
    ny, nx = inst.labels.shape
    prob = O.Problem(nx=nx, ny=ny, h=inst.dx, lambda0=inst.lambda0, n_steps=inst.n_steps, n_pml=inst.n_pml,
                     j_src=inst.j_src, j_ref=inst.j_ref, j_trn=inst.j_trn, courant=inst.courant, dft_start=0)
    coef = O.ade_coefficients(prob, inst.model, inst.n_poles)
    e_inc, h_inc = O.incident_pulse(prob, inst.pulse_tau, inst.pulse_t0)
    st, mon = O.run_ade(prob, inst.labels, coef, inst.n_poles, inst.lambdas, e_inc, h_inc, n_end=n_mid)
    mid = (st.ez.copy(), st.hx * O.ETA0, st.hy * O.ETA0)
    st, mon = O.run_ade(prob, inst.labels, coef, inst.n_poles, inst.lambdas, e_inc, h_inc, state=st, mon=mon,
                        n_begin=n_mid)
    rta = np.array([O.spectra_pulse(prob, lam, mon[f], O.pulse_transform(prob, e_inc, lam))
                    for f, lam in enumerate(inst.lambdas)])
    return mid, dict(R=rta[:, 0], T=rta[:, 1], mon=mon)


def gpu_bb(fdtd, insts, steps, n_mid=None, **kw):
    with fdtd.Simulation(insts, fdtd.Options(n_steps=steps, **kw)) as s:
        mid = None
        if n_mid:
            s.step(n_mid)
            mid = [s.fields(k) for k in range(len(insts))]
        s.run()
        out = []
        for k, inst in enumerate(insts):
            spec = s.broadband_spectra(k) if hasattr(inst, "lambdas") else None
            out.append((spec, s.fields(k), s.monitors(k)))
        return out, s.spectra(), mid


def check(inst, got, mid, ref, tag):
    (R, T, A), _, mon = got
    omid, ores = ref
    errs = [rel_l2(mid[0], omid[0]), rel_l2(mid[1], omid[1])]
    if np.abs(omid[2]).max() > 0:
        errs.append(rel_l2(mid[2], omid[2]))
    merr = max(rel_l2(mon[k], ores["mon"][k]) for k in range(len(inst.lambdas)))
    print(tag, "fields", errs, "monitors", merr, "R", R, ores["R"], "T", T, ores["T"], flush=True)
    assert max(errs) < 1e-3 and merr < 1e-3
    assert np.abs(R - ores["R"]).max() < 1e-4 and np.abs(T - ores["T"]).max() < 1e-4


@pytest.mark.parametrize("kw", [dict(), dict(kernel=1)])
def test_lorentz_slab_against_the_oracle(gpu_lib, kw):
    ny = 400
    lab = np.zeros((ny, 8), np.uint8)
    lab[150:250] = 1
    model = [[1.0, 0.0, 0.0, 0.0, 0.0], lorentz(2.0, 0.5, 500e-9, 0.1, sigma=1e4)]
    inst = bb_instance(gpu_lib, lab, model, 1, [450e-9, 500e-9, 550e-9, 650e-9, 800e-9, 900e-9], 5000)
    n_mid = int(round(inst.pulse_t0 / (inst.courant / np.sqrt(2) * inst.dx / C0))) + 300   # pulse in the slab
    ref = oracle_bb(inst, n_mid)
    out, (Rm, _, _), mid = gpu_bb(gpu_lib, [inst], inst.n_steps, n_mid=n_mid, **kw)
    check(inst, out[0], mid[0], ref, "lorentz-slab")
    assert np.isnan(Rm[0])        # fdtd_spectra has no single value for a broadband run


def test_random_map_with_two_poles_against_the_oracle(gpu_lib):
    base = LG.configs.random_instance(70, 150, 61, n_labels=5, steps=0, n_pml=12)
    rng = np.random.default_rng(61)
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 5):
        p1 = lorentz(rng.uniform(1.5, 2.5), rng.uniform(0.1, 0.6), rng.uniform(350e-9, 700e-9),
                     rng.uniform(0.02, 0.2), sigma=rng.uniform(0, 3e4))
        p2 = lorentz(0.0, rng.uniform(0.05, 0.3), rng.uniform(300e-9, 900e-9), rng.uniform(0.05, 0.3))
        model.append(p1 + p2[2:])
    lams = np.linspace(420e-9, 880e-9, 12)
    inst = bb_instance(gpu_lib, base.labels, model, 2, lams, 1800, n_pml=12)
    n_mid = int(round(inst.pulse_t0 / (inst.courant / np.sqrt(2) * inst.dx / C0))) + 100
    ref = oracle_bb(inst, n_mid)
    out, _, mid = gpu_bb(gpu_lib, [inst], inst.n_steps, n_mid=n_mid, t_block=8, band_rows=32)
    check(inst, out[0], mid[0], ref, "two-pole map")


@pytest.mark.parametrize("kw", [dict(t_block=8, band_rows=32, use_graph=1), dict(t_block=12, band_rows=16, use_graph=0),
                                dict(kernel=1)])
def test_mixed_batch_equals_separate_contexts(gpu_lib, kw):
    """A monochromatic instance and two broadband ones in one context: each
    bit-identical to its own context."""
    cw = LG.configs.random_instance(90, 120, 71, n_labels=4, steps=700, n_pml=10)
    ny = 140
    lab = np.zeros((ny, 40), np.uint8)
    lab[50:90, ::4] = 1
    model = [[1.0, 0.0, 0.0, 0.0, 0.0], lorentz(1.8, 0.4, 450e-9, 0.1)]
    b1 = bb_instance(gpu_lib, lab, model, 1, [500e-9, 600e-9, 700e-9], 700, n_pml=10)
    b2 = bb_instance(gpu_lib, LG.configs.random_instance(33, 130, 72, n_labels=2, steps=0, n_pml=10).labels,
                     model, 1, [480e-9, 640e-9], 700, n_pml=10)
    insts = [b1, cw, b2]
    out, (R, T, _), _ = gpu_bb(gpu_lib, insts, 700, **kw)
    for k, inst in enumerate(insts):
        o1, (R1, T1, _), _ = gpu_bb(gpu_lib, [inst], 700, **kw)
        if hasattr(inst, "lambdas"):
            assert np.array_equal(out[k][0][0], o1[0][0][0]) and np.array_equal(out[k][0][1], o1[0][0][1])
        else:
            assert R[k] == R1[0] and T[k] == T1[0]
        for a, b in zip(out[k][1], o1[0][1]):
            assert np.array_equal(a, b), (k, kw)
        assert np.array_equal(out[k][2], o1[0][2])


def test_pole_free_broadband_equals_monochromatic_runs(gpu_lib):
    """eps_inf and a fixed sigma with no poles: each monitor wavelength of one
    broadband run gives what a monochromatic GPU run gives with the same
    (eps_r, sigma)."""
    eps_r, sigma = 1.45 ** 2, 3e4
    ny = 300
    lab = np.zeros((ny, 4), np.uint8)
    lab[110:170] = 1
    lams = [500e-9, 650e-9, 800e-9]
    inst = bb_instance(gpu_lib, lab, [[1.0, 0.0], [eps_r, sigma]], 0, lams, 4000, n_pml=32)
    out, _, _ = gpu_bb(gpu_lib, [inst], inst.n_steps)
    R, T, _ = out[0][0]
    for f, lam in enumerate(lams):
        w = 2 * np.pi * C0 / lam
        # (n, k) with n^2 - k^2 = eps_r and 2 n k = sigma/(w eps0)
        e2 = sigma / (w * O.EPS0)
        n = np.sqrt(0.5 * (eps_r + np.hypot(eps_r, e2)))
        cw = SimpleNamespace(labels=lab, nk=np.array([[1.0, 0.0], [n, e2 / (2 * n)]]), dx=20e-9, lambda0=lam,
                             courant=0.99, n_pml=32, j_src=ny - 40, j_ref=ny - 36, j_trn=36, n_steps=12000)
        with gpu_lib.Simulation([cw], gpu_lib.Options(n_steps=12000)) as s:
            s.run()
            Rc, Tc, _ = s.spectra()
        print(lam, R[f], Rc[0], T[f], Tc[0])
        assert abs(R[f] - Rc[0]) < 1e-4 and abs(T[f] - Tc[0]) < 1e-4


def test_broadband_launch_configurations_bit_identical(gpu_lib):
    """Plain sweeps and the streaming kernel at several (K, band) shapes give
    bit-identical fields, polarisation-driven monitors and spectra (ragged nx
    and ny, two poles)."""
    base = LG.configs.random_instance(150, 131, 81, n_labels=4, steps=0, n_pml=10)
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 4):
        model.append(lorentz(1.5 + 0.3 * L, 0.2 * L, 400e-9 + 80e-9 * L, 0.1, sigma=1e4 * L) +
                     lorentz(0.0, 0.1, 700e-9, 0.05)[2:])
    inst = bb_instance(gpu_lib, base.labels, model, 2, [450e-9, 550e-9, 700e-9], 303, n_pml=10)
    outs = []
    for kw in [dict(kernel=1), dict(t_block=1, band_rows=7), dict(t_block=3, band_rows=16),
               dict(t_block=8, band_rows=33), dict(t_block=5, band_rows=200), dict(t_block=10, band_rows=13),
               dict(t_block=12, band_rows=40)]:
        out, _, _ = gpu_bb(gpu_lib, [inst], 303, **kw)
        outs.append((out[0], kw))
    (s0, f0, m0), _ = outs[0]
    for (s, f, m), kw in outs[1:]:
        for a, b in zip(f, f0):
            assert np.array_equal(a, b), kw
        assert np.array_equal(m, m0), kw
        assert np.array_equal(s[0], s0[0]) and np.array_equal(s[1], s0[1]), kw


@pytest.mark.parametrize("pol", [0, 1])
def test_plain_broadband_stepped_in_uneven_chunks_bit_identical(gpu_lib, pol):
    """The plain sweeps keep the monitored field of up to 12 steps in capture
    slots and add them in one monitor launch, and add what is pending at the
    end of every step() call: a run stepped in uneven chunks gives the fields,
    monitors and spectra of one whole run, bit for bit (TMz and TEz)."""
    base = LG.configs.random_instance(70, 97, 61, n_labels=3, steps=0, n_pml=10)
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 3):
        model.append(lorentz(1.4 + 0.3 * L, 0.3, 420e-9 + 90e-9 * L, 0.1, sigma=2e4 * L) +
                     lorentz(0.0, 0.2, 650e-9, 0.08)[2:])
    steps = 203
    inst = bb_instance(gpu_lib, base.labels, model, 2, [450e-9, 550e-9, 700e-9], steps, n_pml=10)
    inst.polarization = pol
    ref, _, _ = gpu_bb(gpu_lib, [inst], steps, kernel=1)
    s0, f0, m0 = ref[0]
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=steps, kernel=1)) as s:
        for n in (5, 13, 1, 24, 12, 30):
            s.step(n)
        s.run()
        spec, f, m = s.broadband_spectra(0), s.fields(0), s.monitors(0)
    assert np.abs(m0).max() > 0
    for a, b in zip(f, f0):
        assert np.array_equal(a, b)
    assert np.array_equal(m, m0)
    assert np.array_equal(spec[0], s0[0]) and np.array_equal(spec[1], s0[1])


# --- broadband TEz (edge permittivity the mean of its cells') ---

def te_bb_instance(fdtd, labels, model, n_poles, lams, steps, **kw):
    inst = bb_instance(fdtd, labels, model, n_poles, lams, steps, **kw)
    inst.polarization = 1
    return inst


def oracle_bb_te(inst, n_mid):
    ny, nx = inst.labels.shape
    prob = O.Problem(nx=nx, ny=ny, h=inst.dx, lambda0=inst.lambda0, n_steps=inst.n_steps, n_pml=inst.n_pml,
                     j_src=inst.j_src, j_ref=inst.j_ref, j_trn=inst.j_trn, courant=inst.courant, dft_start=0,
                     polarization=1)
    coef = O.ade_coefficients(prob, inst.model, inst.n_poles)
    edge = O.edge_model_coefficients(prob, inst.labels, inst.model, inst.n_poles)
    e_inc, h_inc = O.incident_pulse(prob, inst.pulse_tau, inst.pulse_t0)
    st, mon = O.run_te_ade(prob, inst.labels, coef, edge, inst.n_poles, inst.lambdas, e_inc, h_inc, n_end=n_mid)
    mid = (st.hz.copy() * O.ETA0, st.ex.copy(), st.ey.copy())
    st, mon = O.run_te_ade(prob, inst.labels, coef, edge, inst.n_poles, inst.lambdas, e_inc, h_inc, state=st,
                           mon=mon, n_begin=n_mid)
    rta = np.array([O.spectra_pulse(prob, lam, mon[f], O.pulse_transform(prob, e_inc, lam))
                    for f, lam in enumerate(inst.lambdas)])
    return mid, dict(R=rta[:, 0], T=rta[:, 1], mon=mon)


def test_te_lorentz_slab_against_the_oracle(gpu_lib):
    ny = 400
    lab = np.zeros((ny, 8), np.uint8)
    lab[150:250] = 1
    model = [[1.0, 0.0, 0.0, 0.0, 0.0], lorentz(2.0, 0.5, 500e-9, 0.1, sigma=1e4)]
    inst = te_bb_instance(gpu_lib, lab, model, 1, [450e-9, 500e-9, 550e-9, 650e-9, 800e-9, 900e-9], 5000)
    n_mid = int(round(inst.pulse_t0 / (inst.courant / np.sqrt(2) * inst.dx / C0))) + 300
    ref = oracle_bb_te(inst, n_mid)
    out, _, mid = gpu_bb(gpu_lib, [inst], inst.n_steps, n_mid=n_mid)
    check(inst, out[0], mid[0], ref, "te-lorentz-slab")


def test_te_random_map_with_two_poles_against_the_oracle(gpu_lib):
    base = LG.configs.random_instance(70, 150, 62, n_labels=5, steps=0, n_pml=12)
    rng = np.random.default_rng(62)
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 5):
        p1 = lorentz(rng.uniform(1.5, 2.5), rng.uniform(0.1, 0.6), rng.uniform(350e-9, 700e-9),
                     rng.uniform(0.02, 0.2), sigma=rng.uniform(0, 3e4))
        p2 = lorentz(0.0, rng.uniform(0.05, 0.3), rng.uniform(300e-9, 900e-9), rng.uniform(0.05, 0.3))
        model.append(p1 + p2[2:])
    lams = np.linspace(420e-9, 880e-9, 12)
    inst = te_bb_instance(gpu_lib, base.labels, model, 2, lams, 1800, n_pml=12)
    n_mid = int(round(inst.pulse_t0 / (inst.courant / np.sqrt(2) * inst.dx / C0))) + 100
    ref = oracle_bb_te(inst, n_mid)
    out, _, mid = gpu_bb(gpu_lib, [inst], inst.n_steps, n_mid=n_mid)
    check(inst, out[0], mid[0], ref, "te two-pole map")


@pytest.mark.parametrize("kw", [dict(), dict(t_block=8, band_rows=24, use_graph=1),
                                dict(t_block=5, band_rows=16, use_graph=0),
                                dict(t_block=3, band_rows=16, special_rows=4, use_graph=1)])
def test_te_and_tm_broadband_batch_equals_separate_contexts(gpu_lib, kw):
    """A broadband TEz, a broadband TMz and a monochromatic instance in one
    context, each on its own streaming kernel: each is bit-identical to its
    own context on the plain path and on the streaming kernel."""
    ny = 140
    lab = np.zeros((ny, 40), np.uint8)
    lab[50:90, ::4] = 1
    model = [[1.0, 0.0, 0.0, 0.0, 0.0], lorentz(1.8, 0.4, 450e-9, 0.1, sigma=5e3)]
    te = te_bb_instance(gpu_lib, lab, model, 1, [500e-9, 600e-9, 700e-9], 700, n_pml=10)
    tm = bb_instance(gpu_lib, lab, model, 1, [500e-9, 600e-9, 700e-9], 700, n_pml=10)
    cw = LG.configs.random_instance(90, 120, 73, n_labels=4, steps=700, n_pml=10)
    insts = [te, tm, cw]
    with gpu_lib.Simulation(insts, gpu_lib.Options(n_steps=700, **kw)) as s:
        assert s.config()["kernel"] == 0
    with gpu_lib.Simulation([te], gpu_lib.Options(n_steps=700)) as s:
        assert s.config()["kernel"] == 0
    out, (R, T, _), _ = gpu_bb(gpu_lib, insts, 700, **kw)
    for k, inst in enumerate(insts):
        for kw1 in [dict(kernel=1), dict()]:
            o1, (R1, T1, _), _ = gpu_bb(gpu_lib, [inst], 700, **kw1)
            if hasattr(inst, "lambdas"):
                assert np.array_equal(out[k][0][0], o1[0][0][0]) and np.array_equal(out[k][0][1], o1[0][0][1])
            else:
                assert R[k] == R1[0] and T[k] == T1[0]
            for a, b in zip(out[k][1], o1[0][1]):
                assert np.array_equal(a, b), (k, kw1)
            assert np.array_equal(out[k][2], o1[0][2])
    # unpolarised broadband spectra: the mean of the two polarisations (this
    # short run stops before the pulse has left, so the values are not physical)
    Ru, Tu, Au = gpu_lib.unpolarized(out[1][0], out[0][0])
    assert np.allclose(Ru, 0.5 * (out[0][0][0] + out[1][0][0])) and np.allclose(Tu, 0.5 * (out[0][0][1] + out[1][0][1]))


def test_te_broadband_launch_configurations_bit_identical(gpu_lib):
    """Broadband TEz: the plain sweeps and the streaming kernel at every steps-
    per-launch count and several band heights give bit-identical fields,
    polarisation-driven monitors and spectra (ragged nx and ny, two poles,
    label interfaces along both axes, so that both sides of many edges carry
    poles)."""
    base = LG.configs.random_instance(150, 131, 81, n_labels=4, steps=0, n_pml=10)
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 4):
        model.append(lorentz(1.5 + 0.3 * L, 0.2 * L, 400e-9 + 80e-9 * L, 0.1, sigma=1e4 * L) +
                     lorentz(0.0, 0.1, 700e-9, 0.05)[2:])
    inst = te_bb_instance(gpu_lib, base.labels, model, 2, [450e-9, 550e-9, 700e-9], 303, n_pml=10)
    outs = []
    for kw in [dict(kernel=1), dict(t_block=1, band_rows=7), dict(t_block=2, band_rows=16, special_rows=4),
               dict(t_block=3, band_rows=16), dict(t_block=4, band_rows=33, special_rows=8),
               dict(t_block=5, band_rows=200), dict(t_block=6, band_rows=13, special_rows=12),
               dict(t_block=7, band_rows=64), dict(t_block=8, band_rows=33), dict(t_block=10, band_rows=13),
               dict(t_block=12, band_rows=40)]:
        out, _, _ = gpu_bb(gpu_lib, [inst], 303, **kw)
        outs.append((out[0], kw))
    (s0, f0, m0), _ = outs[0]
    assert np.abs(m0).max() > 0
    for (s, f, m), kw in outs[1:]:
        for a, b in zip(f, f0):
            assert np.array_equal(a, b), kw
        assert np.array_equal(m, m0), kw
        assert np.array_equal(s[0], s0[0]) and np.array_equal(s[1], s0[1]), kw


def test_te_broadband_layered_map_bit_identical(gpu_lib):
    """Broadband TEz on a layered map whose wave rows fall in three classes:
    - air rows, where no cell drives a pole;
    - layer interiors and layer faces against air, where cells drive poles but no
      edge's second cell does;
    - faces between two dispersive layers and the vertical sides of an inset
      block, where second cells drive poles too.
    One label drives only its first pole. The streaming kernel evaluates each
    class on its own wave-uniform path. At every steps-per-launch count the
    fields, monitors and spectra must match the plain sweeps bit for bit."""
    ny, nx = 150, 150
    lab = np.zeros((ny, nx), np.uint8)
    lab[28:58, :] = 1
    lab[58:74, :] = 2
    lab[74:104, :] = 3
    lab[38:50, 21:93] = 2
    model = [[1.0, 0.0] + [0.0] * 6,
             lorentz(1.8, 0.3, 480e-9, 0.1, sigma=1e4) + lorentz(0.0, 0.1, 700e-9, 0.05)[2:],
             lorentz(2.1, 0.5, 560e-9, 0.08) + lorentz(0.0, 0.2, 650e-9, 0.1)[2:],
             lorentz(1.6, 0.4, 520e-9, 0.12, sigma=2e4) + lorentz(0.0, 0.0, 700e-9, 0.05)[2:]]
    inst = te_bb_instance(gpu_lib, lab, model, 2, [450e-9, 550e-9, 700e-9], 400, n_pml=10)
    outs = []
    for kw in [dict(kernel=1), dict(t_block=1, band_rows=9), dict(t_block=2, band_rows=16, special_rows=4),
               dict(t_block=3, band_rows=21), dict(t_block=4, band_rows=64, special_rows=8),
               dict(t_block=5, band_rows=64, special_rows=4), dict(t_block=6, band_rows=17),
               dict(t_block=8, band_rows=40), dict(t_block=12, band_rows=24)]:
        out, _, _ = gpu_bb(gpu_lib, [inst], 400, **kw)
        outs.append((out[0], kw))
    (s0, f0, m0), _ = outs[0]
    assert np.abs(m0).max() > 0 and np.abs(f0[1][20:110]).max() > 0
    for (s, f, m), kw in outs[1:]:
        for a, b in zip(f, f0):
            assert np.array_equal(a, b), kw
        assert np.array_equal(m, m0), kw
        assert np.array_equal(s[0], s0[0]) and np.array_equal(s[1], s0[1]), kw


def test_pole_free_te_broadband_equals_monochromatic_te_runs(gpu_lib):
    eps_r, sigma = 1.45 ** 2, 3e4
    ny = 300
    lab = np.zeros((ny, 4), np.uint8)
    lab[110:170] = 1
    lams = [500e-9, 650e-9, 800e-9]
    inst = te_bb_instance(gpu_lib, lab, [[1.0, 0.0], [eps_r, sigma]], 0, lams, 4000, n_pml=32)
    out, _, _ = gpu_bb(gpu_lib, [inst], inst.n_steps)
    R, T, _ = out[0][0]
    for f, lam in enumerate(lams):
        w = 2 * np.pi * C0 / lam
        e2 = sigma / (w * O.EPS0)
        n = np.sqrt(0.5 * (eps_r + np.hypot(eps_r, e2)))
        cw = SimpleNamespace(labels=lab, nk=np.array([[1.0, 0.0], [n, e2 / (2 * n)]]), dx=20e-9, lambda0=lam,
                             courant=0.99, n_pml=32, j_src=ny - 40, j_ref=ny - 36, j_trn=36, n_steps=12000,
                             polarization=1)
        with gpu_lib.Simulation([cw], gpu_lib.Options(n_steps=12000)) as s:
            s.run()
            Rc, Tc, _ = s.spectra()
        print(lam, R[f], Rc[0], T[f], Tc[0])
        assert abs(R[f] - Rc[0]) < 1e-4 and abs(T[f] - Tc[0]) < 1e-4


@pytest.mark.parametrize("nx", [1, 7, 65])
def test_te_broadband_narrow_widths_16_labels_and_drude_against_the_oracle(gpu_lib, nx):
    """Broadband TEz on one-column and ragged grids, with the full 16-label
    pair table and a Drude term (w_p = 0) among the poles."""
    ny = 160
    rng = np.random.default_rng(90 + nx)
    lab = np.zeros((ny, nx), np.uint8)
    lab[50:110] = rng.integers(1, 16, size=(60, nx))
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 16):
        p1 = lorentz(rng.uniform(1.3, 2.2), rng.uniform(0.05, 0.4), rng.uniform(350e-9, 700e-9),
                     rng.uniform(0.05, 0.3), sigma=rng.uniform(0, 2e4))
        drude = [0.0, 0.0, (2 * np.pi * C0 / rng.uniform(2e-6, 6e-6)) ** 2, 0.0, 2 * np.pi * C0 / 5e-6]
        model.append(p1 + (drude[2:] if L % 3 == 0 else lorentz(0.0, 0.1, 800e-9, 0.1)[2:]))
    inst = te_bb_instance(gpu_lib, lab, model, 2, np.linspace(450e-9, 850e-9, 5), 1200, n_pml=12)
    n_mid = int(round(inst.pulse_t0 / (inst.courant / np.sqrt(2) * inst.dx / C0))) + 150
    ref = oracle_bb_te(inst, n_mid)
    out, _, mid = gpu_bb(gpu_lib, [inst], inst.n_steps, n_mid=n_mid)
    check(inst, out[0], mid[0], ref, "te-edges nx=%d" % nx)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_te_broadband_graph_replay_equals_direct_launches(gpu_lib, K):
    """Broadband TEz with thin special bands (many special items beside the
    lean ones): replays of the captured run equal direct launches and the
    plain sweeps bit for bit, three times over."""
    base = LG.configs.random_instance(150, 131, 81, n_labels=4, steps=0, n_pml=10)
    model = [[1.0, 0.0] + [0.0] * 6]
    for L in range(1, 4):
        model.append(lorentz(1.5 + 0.3 * L, 0.2 * L, 400e-9 + 80e-9 * L, 0.1, sigma=1e4 * L) +
                     lorentz(0.0, 0.1, 700e-9, 0.05)[2:])
    inst = te_bb_instance(gpu_lib, base.labels, model, 2, [450e-9, 550e-9, 700e-9], 303, n_pml=10)
    ref, _, _ = gpu_bb(gpu_lib, [inst], 303, kernel=1)
    kw = dict(t_block=K, band_rows=16, special_rows=4)
    for rep in range(3):
        for g in (1, 0):
            out, _, _ = gpu_bb(gpu_lib, [inst], 303, use_graph=g, **kw)
            for a, b in zip(out[0][1], ref[0][1]):
                assert np.array_equal(a, b), (rep, g)
            assert np.array_equal(out[0][2], ref[0][2]), (rep, g)
