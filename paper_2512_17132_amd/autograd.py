"""torch.autograd wrapper of the forward run and the hand-written discrete
adjoint (fdtd_backward): reflectance and transmittance as differentiable
functions of the per-label complex indices (n, k)."""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import fdtd


class SpectraFn(torch.autograd.Function):
    """(R, T) of every instance as a function of nk (n_inst, n_labels, 2).

    Forward: one recorded run (checkpoints for the adjoint) and the spectra.
    Backward: fdtd_backward with dL/dR, dL/dT; returns dL/dnk."""

    @staticmethod
    def forward(ctx, nk, instances, opts):
        nk_np = nk.detach().to("cpu", torch.float64).numpy()
        insts = [dataclasses.replace(inst, nk=nk_np[i, : np.asarray(inst.nk).reshape(-1, 2).shape[0]].copy())
                 for i, inst in enumerate(instances)]
        o = dataclasses.replace(opts, checkpoint_every=opts.checkpoint_every or -1)
        sim = fdtd.Simulation(insts, o)
        sim.run(record=True)
        R, T, _ = sim.spectra()
        ctx.sim = sim
        ctx.shape = tuple(nk.shape)
        ctx.dtype = nk.dtype
        ctx.device = nk.device
        return torch.from_numpy(R).to(nk.dtype), torch.from_numpy(T).to(nk.dtype)

    @staticmethod
    def backward(ctx, gR, gT):
        sim = ctx.sim
        dR = (gR if gR is not None else torch.zeros(ctx.shape[0])).detach().cpu().double().numpy()
        dT = (gT if gT is not None else torch.zeros(ctx.shape[0])).detach().cpu().double().numpy()
        gnk, _ = sim.backward(dR, dT, want_eps=False)
        sim.close()
        out = torch.zeros(ctx.shape, dtype=torch.float64)
        for i, g in enumerate(gnk):
            out[i, : g.shape[0]] = torch.from_numpy(g)
        return out.to(ctx.dtype).to(ctx.device), None, None


def spectra(nk: torch.Tensor, instances, opts: fdtd.Options):
    """Differentiable (R, T) for instances whose per-label (n, k) are taken
    from nk[i, :n_labels_i]."""
    return SpectraFn.apply(nk, list(instances), opts)
