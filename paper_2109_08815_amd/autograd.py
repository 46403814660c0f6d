"""torch.autograd wrapper of the multiple-shooting log-likelihood.

Forward: loglik_multishoot -> (log p [N], g_def [N, K, n_s-1]) in float64.
Backward: sim_batch_adjoint as a vector-Jacobian product (seed_logp and
cot_gdef the incoming gradients), whose g_theta and S_dot are d/d theta and
d/d S of  sum_i grad_logp_i log p_i + sum grad_gdef * g_def.  Both
directions run entirely in the library's kernels; this module only copies
tensors in and out.
"""
from __future__ import annotations

import torch

from . import lib as L


class MultiShootingLikelihood:
    """Holds the device buffers of one problem and exposes a differentiable call."""

    def __init__(self, pb, obs, theta0, S0, lam_def=None, device="cuda"):
        N = theta0.shape[0]
        self.job = L.Job(pb, obs, theta=theta0, S=S0, device=device, with_g_theta=True,
                         seed_logp=torch.ones(N, dtype=torch.float64).numpy(),
                         cot_gdef=torch.zeros((N, pb.K, max(pb.n_s - 1, 1)), dtype=torch.float64).numpy())
        if lam_def is not None:
            self.job.lam_def.copy_(torch.as_tensor(lam_def, dtype=torch.float32))
        self.batch = L.Batch([self.job])
        self.n_s = pb.n_s

    def __call__(self, theta, S):
        return _Fn.apply(theta, S, self)


class _Fn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, S, mod):
        j = mod.job
        j.theta.copy_(theta.detach())
        if mod.n_s > 1:
            j.S.copy_(S.detach())
        L.loglik_multishoot(mod.batch)
        ctx.mod = mod
        return j.logp.clone(), j.gdef[:, :, : mod.n_s - 1].clone()

    @staticmethod
    def backward(ctx, grad_logp, grad_gdef):
        mod = ctx.mod
        j = mod.job
        N = j.N
        j.seed_logp.copy_(grad_logp if grad_logp is not None else torch.zeros(N, dtype=torch.float64,
                                                                                device=j.device))
        if mod.n_s > 1:
            if grad_gdef is None:
                j.cot_gdef.zero_()
            else:
                j.cot_gdef[:, :, : mod.n_s - 1].copy_(grad_gdef)
        L.sim_batch_adjoint(mod.batch)
        d_theta = j.g_theta.to(torch.float32)
        d_S = j.S_dot[:, :, : mod.n_s - 1].clone() if mod.n_s > 1 else None
        return d_theta, d_S, None
