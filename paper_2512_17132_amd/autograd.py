"""torch.autograd wrapper of the forward run and the hand-written discrete
adjoint (fdtd_backward): reflectance and transmittance as differentiable
functions of the per-label complex indices (n, k) and of a per-pixel
permittivity offset (the inversion use of the gradient named in Sec. 5)."""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import fdtd


class SpectraFn(torch.autograd.Function):
    """(R, T) of every instance as a function of nk (n_inst, n_labels, 2) and
    of eps_offset, a flat tensor of sum(ny * nx) per-pixel offsets of eps_r
    (instances in order, each row-major), or None.

    The forward path takes materials from the label map only, so the forward
    runs at eps_offset = 0 (a non-zero offset is refused); the gradient with
    respect to eps_offset is dR/d eps_r per pixel at the label-derived eps_r
    with sigma held fixed.

    Forward: one recorded run (checkpoints for the adjoint) and the spectra.
    Backward: fdtd_backward with dL/dR, dL/dT; returns dL/dnk and, when asked,
    dL/d eps_offset.  The recorded context lives as long as the graph, so a
    second backward (retain_graph=True) works."""

    @staticmethod
    def forward(ctx, nk, eps_offset, instances, opts):
        nk_np = nk.detach().to("cpu", torch.float64).numpy()
        insts = [dataclasses.replace(inst, nk=nk_np[i, : np.asarray(inst.nk).reshape(-1, 2).shape[0]].copy())
                 for i, inst in enumerate(instances)]
        cells = sum(int(np.prod(inst.labels.shape)) for inst in insts)
        if eps_offset is not None:
            if eps_offset.numel() != cells:
                raise ValueError("eps_offset needs %d entries (sum of ny*nx), got %d" % (cells, eps_offset.numel()))
            if bool(torch.any(eps_offset.detach() != 0)):
                raise ValueError("the forward run takes eps_r from the label map: eps_offset must be zero")
        o = dataclasses.replace(opts, checkpoint_every=opts.checkpoint_every or -1)
        sim = fdtd.Simulation(insts, o)
        sim.run(record=True)
        R, T, _ = sim.spectra()
        ctx.sim = sim
        ctx.shape = tuple(nk.shape)
        ctx.dtype = nk.dtype
        ctx.device = nk.device
        ctx.eps_meta = None if eps_offset is None else (eps_offset.shape, eps_offset.dtype, eps_offset.device)
        return torch.from_numpy(R).to(nk.dtype), torch.from_numpy(T).to(nk.dtype)

    @staticmethod
    def backward(ctx, gR, gT):
        sim = ctx.sim
        dR = (gR if gR is not None else torch.zeros(ctx.shape[0])).detach().cpu().double().numpy()
        dT = (gT if gT is not None else torch.zeros(ctx.shape[0])).detach().cpu().double().numpy()
        want_eps = ctx.eps_meta is not None and ctx.needs_input_grad[1]
        gnk, geps = sim.backward(dR, dT, want_eps=want_eps)
        out = torch.zeros(ctx.shape, dtype=torch.float64)
        for i, g in enumerate(gnk):
            out[i, : g.shape[0]] = torch.from_numpy(g)
        g_eps = None
        if want_eps:
            shape, dtype, device = ctx.eps_meta
            g_eps = torch.cat([e.reshape(-1) for e in geps]).to(dtype).to(device).reshape(shape)
        return out.to(ctx.dtype).to(ctx.device), g_eps, None, None


def pixel_offsets(instances, device="cuda", dtype=torch.float32) -> torch.Tensor:
    """A zero per-pixel eps_r offset for ``spectra`` (flat, sum of ny*nx,
    requires_grad)."""
    cells = sum(int(np.prod(inst.labels.shape)) for inst in instances)
    return torch.zeros(cells, dtype=dtype, device=device, requires_grad=True)


def spectra(nk: torch.Tensor, instances, opts: fdtd.Options, eps_offset: torch.Tensor | None = None):
    """Differentiable (R, T) for instances whose per-label (n, k) are taken
    from nk[i, :n_labels_i]; with eps_offset (see pixel_offsets) the per-pixel
    eps_r gradient flows to it as well."""
    return SpectraFn.apply(nk, eps_offset, list(instances), opts)
