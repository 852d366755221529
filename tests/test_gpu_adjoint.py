"""GPU discrete adjoint against the FP64 oracle's adjoint (per-label (n, k)
and per-pixel eps_r) and through the torch.autograd wrapper."""
import numpy as np
import pytest
import torch

import leafgen as LG
import oracle as O
from parity_util import problem_for, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    inst = LG.configs.random_instance(48, 110, 21, n_labels=4, steps=1400, n_pml=12)
    prob = problem_for(inst)
    res, gnk, geps, _ = O.gradient(prob, inst.labels, inst.nk, 1.0, 0.4)
    return inst, res, gnk, geps


@pytest.mark.parametrize("every", [-1, 97, 1400])
def test_adjoint_matches_oracle(gpu_lib, case, every):
    inst, res, gnk_o, geps_o = case
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps, checkpoint_every=every)) as s:
        s.run(record=True)
        R, T, _ = s.spectra()
        gnk, geps = s.backward([1.0], [0.4])
        R2, T2, _ = s.spectra()           # the forward state is restored
    assert R2[0] == R[0] and T2[0] == T[0]
    g = gnk[0]
    for L in range(1, inst.nk.shape[0]):
        for c in range(2):
            ref = gnk_o[L, c]
            assert abs(g[L, c] - ref) <= 1e-2 * abs(ref) + 1e-6, (L, c, g[L, c], ref)
    ge = geps[0].cpu().numpy()
    assert rel_l2(ge, geps_o) < 1e-2


def test_autograd_wrapper(gpu_lib, case):
    from paper_2512_17132_amd import autograd as AG
    inst, res, gnk_o, geps_o = case
    nk = torch.tensor(inst.nk[None], dtype=torch.float64, requires_grad=True)
    R, T = AG.spectra(nk, [inst], gpu_lib.Options(n_steps=inst.n_steps))
    loss = R.sum() + 0.4 * T.sum()
    loss.backward()
    g = nk.grad[0].numpy()
    assert abs(R.item() - res["R"]) < 1e-4
    for L in range(1, inst.nk.shape[0]):
        for c in range(2):
            assert abs(g[L, c] - gnk_o[L, c]) <= 1e-2 * abs(gnk_o[L, c]) + 1e-6


def test_backward_requires_recorded_run(gpu_lib, case):
    inst = case[0]
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps, checkpoint_every=-1)) as s:
        s.run()
        with pytest.raises(gpu_lib.FdtdError) as e:
            s.backward([1.0])
        assert e.value.code == -5


def _grads(fdtd, insts, n_steps, **kw):
    with fdtd.Simulation(insts, fdtd.Options(n_steps=n_steps, **kw)) as s:
        s.run(record=True)
        gnk, geps = s.backward([1.0] * len(insts), [0.3] * len(insts))
        return [g.copy() for g in gnk], [e.cpu().numpy() for e in geps]


def test_adjoint_launch_shapes_agree(gpu_lib):
    """The streaming transposed kernel at several (adjoint K, forward K, band,
    checkpoint spacing) shapes against the plain transposed sweeps: per-pixel
    gradients, and the per-label sums reduced from them in a fixed order,
    bit-identical (ragged nx and ny, every row class present)."""
    inst = LG.configs.random_instance(150, 131, 5, n_labels=6, steps=303, n_pml=10)
    ref_nk, ref_eps = _grads(gpu_lib, [inst], 303, kernel=1, checkpoint_every=-1)
    assert np.abs(ref_eps[0]).max() > 0
    for kw in [dict(t_block=8, band_rows=33, adj_t_block=1, checkpoint_every=-1),
               dict(t_block=4, band_rows=16, adj_t_block=4, checkpoint_every=50),
               dict(t_block=6, band_rows=200, adj_t_block=8, checkpoint_every=303),
               dict(t_block=3, band_rows=8, adj_t_block=3, checkpoint_every=7),
               dict(t_block=12, band_rows=40, adj_t_block=8, checkpoint_every=100),
               dict(t_block=10, band_rows=9, adj_t_block=5, checkpoint_every=-1),
               dict(t_block=8, band_rows=48, adj_t_block=10, checkpoint_every=-1),
               dict(t_block=12, band_rows=64, adj_t_block=12, checkpoint_every=61),
               # the forward's bulk bands as workgroup items (recording replays too)
               dict(t_block=12, band_rows=40, adj_t_block=8, checkpoint_every=100, bulk_columns=256),
               dict(t_block=8, band_rows=33, adj_t_block=1, checkpoint_every=-1, bulk_columns=256)]:
        gnk, geps = _grads(gpu_lib, [inst], 303, **kw)
        assert np.array_equal(geps[0], ref_eps[0]), kw
        assert np.array_equal(gnk[0], ref_nk[0]), kw


def test_batched_adjoint_equals_individual(gpu_lib):
    insts = [LG.configs.random_instance(nx, ny, sd, steps=260, n_pml=10)
             for nx, ny, sd in [(40, 100, 1), (130, 90, 2)]]
    b_nk, b_eps = _grads(gpu_lib, insts, 260, t_block=6, band_rows=20, checkpoint_every=-1)
    for k, inst in enumerate(insts):
        nk, eps = _grads(gpu_lib, [inst], 260, t_block=6, band_rows=20, checkpoint_every=-1)
        assert np.array_equal(eps[0], b_eps[k])
        assert np.array_equal(nk[0], b_nk[k])


@pytest.fixture(scope="module")
def monocot_case():
    """The differentiation form's monocot geometry on a grid the oracle's
    full-history adjoint can hold: 256 x 512 cells of the same 20.48 x 40.96 um
    domain (dx = 80 nm), 2000 steps, loss = R."""
    inst = LG.configs.monocot_config(256, 512, 2000)[0]
    prob = problem_for(inst)
    res, gnk, geps, _ = O.gradient(prob, inst.labels, inst.nk, 1.0, 0.0)
    return inst, res, gnk, geps


def test_adjoint_on_the_monocot_matches_oracle(gpu_lib, monocot_case):
    """All six differentiable labels (cuticle, wall, epidermal and mesophyll
    cytoplasm, chloroplast, vascular) within 1e-2 relative in both n and k, and
    the per-pixel eps_r map within 1e-2 relative L2."""
    inst, res, gnk_o, geps_o = monocot_case
    assert inst.nk.shape[0] == 7
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=inst.n_steps, checkpoint_every=-1)) as s:
        s.autotune()
        s.run(record=True)
        R, T, _ = s.spectra()
        gnk, geps = s.backward([1.0])
        cfg = s.config()
    g = gnk[0]
    ge = geps[0].cpu().numpy()
    worst = max(abs(g[L, c] - gnk_o[L, c]) / abs(gnk_o[L, c]) for L in range(1, 7) for c in range(2))
    print("monocot 256x512 adjoint (K=%d, band %d): R %.6f (oracle %.6f); worst per-label relative error %.2e; "
          "per-pixel rel-L2 %.2e" % (cfg["t_block"], cfg["band_rows"], R[0], res["R"], worst, rel_l2(ge, geps_o)))
    print("dR/dn, dR/dk per label (GPU | oracle):\n", np.hstack([g, gnk_o]))
    assert abs(R[0] - res["R"]) < 1e-4
    for L in range(1, 7):
        for c in range(2):
            ref = gnk_o[L, c]
            assert abs(g[L, c] - ref) <= 1e-2 * abs(ref), (L, c, g[L, c], ref)
    assert rel_l2(ge, geps_o) < 1e-2


def test_autograd_per_pixel_permittivity(gpu_lib, monocot_case):
    """spectra() with a per-pixel eps_r offset: its gradient is the oracle's
    per-pixel dR/d eps_r, nk's gradient the per-label one; a second backward
    through the retained graph adds the same gradients again."""
    from paper_2512_17132_amd import autograd as AG
    inst, res, gnk_o, geps_o = monocot_case
    nk = torch.tensor(inst.nk[None], dtype=torch.float64, requires_grad=True)
    eps = AG.pixel_offsets([inst])
    R, T = AG.spectra(nk, [inst], gpu_lib.Options(n_steps=inst.n_steps), eps_offset=eps)
    R.sum().backward(retain_graph=True)
    g1 = eps.grad.detach().cpu().numpy().reshape(inst.labels.shape).copy()
    n1 = nk.grad.detach().clone().numpy()[0]
    assert abs(R.item() - res["R"]) < 1e-4
    assert rel_l2(g1, geps_o) < 1e-2
    for L in range(1, 7):
        for c in range(2):
            assert abs(n1[L, c] - gnk_o[L, c]) <= 1e-2 * abs(gnk_o[L, c])
    R.sum().backward()
    assert np.allclose(eps.grad.detach().cpu().numpy().reshape(inst.labels.shape), 2 * g1, rtol=1e-6, atol=0)
    assert np.allclose(nk.grad.numpy()[0], 2 * n1, rtol=1e-9, atol=0)
    with pytest.raises(ValueError):
        bad = torch.ones_like(eps)
        AG.spectra(nk, [inst], gpu_lib.Options(n_steps=inst.n_steps), eps_offset=bad)


@pytest.mark.parametrize("kw", [dict(t_block=6, band_rows=24), dict(kernel=1),
                                dict(t_block=6, band_rows=24, checkpoint_every=303)])
def test_fields_after_backward_equal_the_forward_end_state(gpu_lib, kw):
    """303 steps at 6 per launch is 51 launches (50 of 6 and one of 3), so the
    forward run ends in the second field set; after the adjoint's segment
    replays (or, as one segment, with the history the recorded run wrote),
    fields() and a further backward still see the run's final state."""
    inst = LG.configs.random_instance(70, 96, 13, steps=303, n_pml=10)
    kw = dict(dict(checkpoint_every=40), **kw)
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=303, **kw)) as s:
        s.run(record=True)
        before = s.fields(0)
        spec = s.spectra()
        g1, e1 = s.backward([1.0])
        after = s.fields(0)
        g2, e2 = s.backward([1.0])
        spec2 = s.spectra()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert np.array_equal(spec[0], spec2[0]) and np.array_equal(spec[1], spec2[1])
    assert np.array_equal(e1[0].cpu().numpy(), e2[0].cpu().numpy())
    assert np.array_equal(g1[0], g2[0])


@pytest.mark.parametrize("every", [-1, 303])
def test_single_segment_recorded_run(gpu_lib, every):
    """As one segment (checkpoint_every >= n_steps, or -1 where the history
    fits), the recorded run writes the Ez history with the recording kernels:
    its fields and spectra equal a plain run's, and its gradients equal those
    of checkpointed segments replayed in the backward, bit for bit."""
    inst = LG.configs.random_instance(150, 131, 5, n_labels=6, steps=303, n_pml=10)
    kw = dict(t_block=6, band_rows=24, special_rows=4)
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=303, **kw)) as s:
        s.run()
        f0, sp0 = s.fields(0), s.spectra()
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=303, checkpoint_every=every, **kw)) as s:
        s.run(record=True)
        f1, sp1 = s.fields(0), s.spectra()
        g1, e1 = s.backward([1.0], [0.3])
        g1, e1 = g1[0].copy(), e1[0].cpu().numpy()
        f2 = s.fields(0)
        # more device memory than the segmented form: the whole history
        full_bytes = s.config()["device_bytes"]
    for a, b, c in zip(f0, f1, f2):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.array_equal(sp0[0], sp1[0]) and np.array_equal(sp0[1], sp1[1])
    g2, e2 = _grads(gpu_lib, [inst], 303, checkpoint_every=37, **kw)
    assert np.array_equal(g1, g2[0]) and np.array_equal(e1, e2[0])
    with gpu_lib.Simulation([inst], gpu_lib.Options(n_steps=303, checkpoint_every=37, **kw)) as s:
        s.run(record=True)
        seg_bytes = s.config()["device_bytes"]
    assert full_bytes > seg_bytes
