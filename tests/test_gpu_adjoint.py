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
