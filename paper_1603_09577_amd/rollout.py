"""Differentiable rollout: phi(T) as a function of phi0 and the K0 entries.

``rollout(sim, phi0, k0, nsteps)`` runs the fused sweep nsteps times and
returns phi(T); its backward runs the hand-written reversed sweep
(lbm_adjoint_step) with two-level checkpointing: a copy of the state every
``seg`` steps (seg = ceil(sqrt(T)) by default) in the forward pass, and in the
backward pass each segment is recomputed into a ring of seg states and then
walked backwards.  Memory: about 2 sqrt(T) states.  Where two reversed
sweeps per launch apply (lbm_adjoint_pair_ok) and a timed trial finds them
faster (Lbm.adjoint_pairs_faster), the walk takes them (lbm_adjoint_step2);
psi and pi are the same bit for bit either way.

Gradients: dL/dphi0 (same shape as phi0) and dL/dK0 for the symmetric entries
(xx, xy, yy) in 2-D, each off-diagonal entry one parameter.
"""
import math

import numpy as np
import torch

from . import lbm as _lbm


def _k0_matrix(k0):
    k = k0.detach().cpu().numpy().astype(np.float64).reshape(-1)
    m = np.zeros((3, 3))
    if k.size == 3:
        m[0, 0], m[0, 1], m[1, 1] = k
        m[1, 0] = m[0, 1]
        m[2, 2] = 1.0
    else:
        m[0, 0], m[0, 1], m[1, 1], m[0, 2], m[1, 2], m[2, 2] = k
        m[1, 0], m[2, 0], m[2, 1] = m[0, 1], m[0, 2], m[1, 2]
    return m


class LbmRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, k0, sim, nsteps, seg, pairs):
        sim.set_k0(_k0_matrix(k0))
        sim.init(phi0.detach())
        checkpoints = []
        t = 0
        while t < nsteps:
            which, _ = sim.current()
            checkpoints.append((t, sim.f[which].clone(), sim.p.clone()))
            n = min(seg, nsteps - t)
            sim.step(n)
            t += n
        phiT = sim.phi()
        ctx.sim, ctx.checkpoints, ctx.nsteps, ctx.seg = sim, checkpoints, nsteps, seg
        ctx.pairs = pairs
        ctx.k0_len = k0.numel()
        ctx.k0_device = k0.device
        ctx.save_for_backward(phi0.detach())
        return phiT

    @staticmethod
    def backward(ctx, gphi):
        (phi0,) = ctx.saved_tensors
        sim, seg = ctx.sim, ctx.seg
        gphi = gphi.to(torch.float64).contiguous()
        if ctx.pairs == "auto":
            use_pairs = sim.adjoint_pairs_faster()   # before the seed: the trial adds to the K0 sums
        else:
            use_pairs = bool(ctx.pairs) and sim.adjoint_pair_ok
        cur_psi, pi = sim.adjoint_buffers()
        psi_other, pi_other = sim.adjoint_buffers()
        sim.adjoint_seed(gphi, cur_psi, pi)
        ring = [(torch.empty_like(sim.f[0]), torch.empty_like(sim.p)) for _ in range(seg)]
        for t0, fck, pck in reversed(ctx.checkpoints):
            n = min(seg, ctx.nsteps - t0)
            ring[0][0].copy_(fck)
            ring[0][1].copy_(pck)
            for i in range(1, n):
                ring[i][1].copy_(ring[i - 1][1])
                sim.sweep(ring[i - 1][0], ring[i][0], ring[i][1])
            i = n - 1
            while i >= 0:
                if use_pairs and i >= 1:
                    sim.adjoint_step2(ring[i][0], ring[i][1], ring[i - 1][0], ring[i - 1][1],
                                      cur_psi, pi, psi_other, pi_other)
                    pi, pi_other = pi_other, pi
                    i -= 2
                else:
                    sim.adjoint_step(ring[i][0], ring[i][1], cur_psi, pi, psi_other, pi)
                    i -= 1
                cur_psi, psi_other = psi_other, cur_psi
        gphi0 = sim.adjoint_init(phi0, cur_psi, pi)
        gk = sim.adjoint_grad_k0()
        keys = ("xx", "xy", "yy") if ctx.k0_len == 3 else ("xx", "xy", "yy", "xz", "yz", "zz")
        gk_t = torch.tensor([gk[k] for k in keys], dtype=torch.float64, device=ctx.k0_device)
        return gphi0, gk_t, None, None, None, None


def rollout(sim, phi0, k0, nsteps, seg=None, pairs="auto"):
    """phi(T) of ``sim`` (an lbm.Lbm) from phi0 with K0 entries k0
    ((xx, xy, yy) in 2-D), differentiable in phi0 and k0.  ``pairs``: "auto"
    (time both launch forms once), True (two reversed sweeps per launch where
    they apply) or False (one per launch)."""
    seg = seg or max(1, int(math.ceil(math.sqrt(nsteps))))
    if pairs != "auto":
        pairs = bool(pairs)
    return LbmRollout.apply(phi0, k0, sim, int(nsteps), int(seg), pairs)


__all__ = ["rollout", "LbmRollout"]
