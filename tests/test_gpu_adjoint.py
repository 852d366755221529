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
    gradients bit-identical (ragged nx and ny, every row class present)."""
    inst = LG.configs.random_instance(150, 131, 5, n_labels=6, steps=303, n_pml=10)
    ref_nk, ref_eps = _grads(gpu_lib, [inst], 303, kernel=1, checkpoint_every=-1)
    assert np.abs(ref_eps[0]).max() > 0
    for kw in [dict(t_block=8, band_rows=33, adj_t_block=1, checkpoint_every=-1),
               dict(t_block=4, band_rows=16, adj_t_block=4, checkpoint_every=50),
               dict(t_block=6, band_rows=200, adj_t_block=8, checkpoint_every=303),
               dict(t_block=3, band_rows=8, adj_t_block=3, checkpoint_every=7),
               dict(t_block=12, band_rows=40, adj_t_block=8, checkpoint_every=100),
               dict(t_block=10, band_rows=9, adj_t_block=5, checkpoint_every=-1)]:
        gnk, geps = _grads(gpu_lib, [inst], 303, **kw)
        assert np.array_equal(geps[0], ref_eps[0]), kw
        assert np.allclose(gnk[0], ref_nk[0], rtol=1e-12, atol=0), kw


def test_batched_adjoint_equals_individual(gpu_lib):
    insts = [LG.configs.random_instance(nx, ny, sd, steps=260, n_pml=10)
             for nx, ny, sd in [(40, 100, 1), (130, 90, 2)]]
    b_nk, b_eps = _grads(gpu_lib, insts, 260, t_block=6, band_rows=20, checkpoint_every=-1)
    for k, inst in enumerate(insts):
        nk, eps = _grads(gpu_lib, [inst], 260, t_block=6, band_rows=20, checkpoint_every=-1)
        assert np.array_equal(eps[0], b_eps[k])
        assert np.allclose(nk[0], b_nk[k], rtol=1e-12, atol=0)
