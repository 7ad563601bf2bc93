"""Differentiable cloth rollout as a torch.autograd.Function.

``ClothRollout.apply(sim, k, c, v0, dt, n_substeps, n_steps, ckpt_every, out_steps)`` runs
the HIP rollout (cloth_rollout_forward) from the handle's initial positions and returns the
positions at the requested frames, [len(out_steps), N, 3]; its backward calls the hand-written
adjoint (cloth_rollout_backward) for dL/dk, dL/dc, dL/dv0.  Tensors must be FP32, contiguous,
on the handle's device; the library runs on the handle's stream (create the handle with
torch's current stream so the two are ordered).  Memory of the backward pass is set by
ckpt_every: one checkpoint per ckpt_every frames plus one segment of states.
"""
from __future__ import annotations

import torch

from . import cloth as B


class ClothRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, k, c, v0, dt, n_substeps, n_steps, ckpt_every, out_steps):
        for name, t in (("k", k), ("c", c), ("v0", v0)):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
        out_steps = [int(s) for s in out_steps]
        x_out = torch.empty((len(out_steps), sim.n, 3), dtype=torch.float32, device=k.device)
        B.cloth_rollout_forward(sim.h, k.data_ptr(), c.data_ptr(), v0.data_ptr(), dt, n_substeps,
                                n_steps, ckpt_every, out_steps, x_out.data_ptr())
        ctx.sim = sim
        ctx.shapes = (k.shape, c.shape, v0.shape)
        return x_out

    @staticmethod
    def backward(ctx, gx_out):
        sim = ctx.sim
        gx = gx_out.contiguous().to(torch.float32)
        ks, cs, vs = ctx.shapes
        dev = gx.device
        gk = torch.empty(ks, dtype=torch.float32, device=dev)
        gc = torch.empty(cs, dtype=torch.float32, device=dev)
        gv0 = torch.empty(vs, dtype=torch.float32, device=dev)
        B.cloth_rollout_backward(sim.h, gx.data_ptr(), gk.data_ptr(), gc.data_ptr(),
                                 gv0.data_ptr())
        return None, gk, gc, gv0, None, None, None, None, None
