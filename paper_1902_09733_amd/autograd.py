"""Differentiable soft-argmin BP (the differentiation form) as a torch.autograd.Function.

Forward: single-level checkerboard min-sum BP over K half-sweeps followed by
the soft-argmin readout, in the library's HIP kernels, saving message
checkpoints.  Backward: the library's hand-written adjoint (bp_backward),
which recomputes states from the checkpoints and returns gradients with
respect to the cost volumes, lambda and tau.  Batches are stacked cost
volumes [B][L][H][W]; lambda and tau are shared scalars, so their gradients
are sums over the batch.
"""
from __future__ import annotations

import torch

from . import stereo


class BPSoftArgmin(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, lam, tau, iters: int = 8, temperature: float = 0.5, checkpoint_every: int = 2):
        if cost.dim() == 3:
            cost = cost.unsqueeze(0)
        cost = cost.contiguous().float()
        params = stereo.BPParams(levels=1, iters=int(iters), lam=float(lam), tau=float(tau), msg_dtype="f32",
                                 temperature=float(temperature), checkpoint_every=int(checkpoint_every))
        vols = list(cost.unbind(0))
        ck = torch.empty(stereo.checkpoint_bytes(vols, params), dtype=torch.uint8, device=cost.device)
        B, _, H, W = cost.shape
        soft = torch.empty((B, H, W), dtype=torch.float32, device=cost.device)
        stereo.run(vols, params, checkpoints=ck, outputs=[{"disp": None, "soft": soft[i], "msgs": None}
                                                          for i in range(B)])
        ctx.save_for_backward(cost, ck)
        ctx.params = params
        return soft

    @staticmethod
    def backward(ctx, grad_soft):
        cost, ck = ctx.saved_tensors
        vols = list(cost.unbind(0))
        grads = list(grad_soft.contiguous().float().unbind(0))
        gcost = torch.empty_like(cost)
        _, gl, gt = stereo.backward(vols, ctx.params, ck, grads, grad_out=gcost)
        return gcost, gl.reshape(()), gt.reshape(()), None, None, None


def soft_argmin_bp(cost, lam, tau, iters: int = 8, temperature: float = 0.5, checkpoint_every: int = 2):
    """Soft-argmin disparity [B][H][W] of BP on cost [B][L][H][W] (differentiable)."""
    lam = lam if isinstance(lam, torch.Tensor) else torch.tensor(float(lam), device=cost.device)
    tau = tau if isinstance(tau, torch.Tensor) else torch.tensor(float(tau), device=cost.device)
    return BPSoftArgmin.apply(cost, lam, tau, iters, temperature, checkpoint_every)
