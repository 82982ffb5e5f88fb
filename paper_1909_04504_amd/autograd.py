"""Differentiable rollout: kinetic energy after N predictor-corrector steps as a
function of the initial velocities and the viscosity.

Forward: sph_step from (x0, u0) with the first acceleration evaluated at the
initial state, keeping a copy of the state every k steps.  Backward: for each
k-step segment in reverse, sph_step_backward recomputes the segment from its
checkpoint and runs the hand-written adjoint kernels; sph_accel_backward then
takes the adjoint through the first acceleration evaluation.  All arithmetic
runs in the library's kernels; this module moves tensors and calls the ABI.
"""
from __future__ import annotations

import torch

from . import (DeviceParticles, FP64, accel_backward, ke_seed, make_params, step,
               step_backward, workspace)


class SPHRollout(torch.autograd.Function):
    """KE(u^N) = sum m |u^N|^2 / 2 after `nsteps` steps.

    Inputs: u0 (dim, n) float64 CUDA tensor in particle-id order, nu a 0-d
    float64 tensor; params (sph_workloads.Params-like), x0, m, ptype as device
    tensors or arrays; nsteps; k (checkpoint interval); precision; nbr_cap
    and pair_tiles (as in make_params).
    """

    @staticmethod
    def forward(ctx, u0, nu, params, x0, m, ptype, nsteps, k, precision=FP64, nbr_cap=0,
                pair_tiles=0):
        p = params.replace(nu=float(nu.item()))
        prm = make_params(p, precision, nbr_cap, pair_tiles)
        n = u0.shape[1]
        dim = u0.shape[0]
        pid = torch.arange(n, dtype=torch.int32, device=u0.device)
        dp = DeviceParticles(x0, u0.detach(), m, ptype, pid.cpu().numpy(), precision,
                             device=u0.device)
        ws = workspace(prm, n, adjoint_k=k, device=u0.device)
        step(prm, dp, 0, ws, prime=True)
        ckpts = [dp.clone()]
        segs = []
        done = 0
        diag = torch.zeros((max(k, 1), 1 + dim), dtype=torch.float64, device=u0.device)
        while done < nsteps:
            kk = min(k, nsteps - done)
            step(prm, dp, kk, ws, prime=False, diag=diag)
            segs.append(kk)
            done += kk
            if done < nsteps:
                ckpts.append(dp.clone())
        ke = diag[segs[-1] - 1, 0].clone() if segs else 0.5 * torch.zeros((), dtype=torch.float64)
        ctx.state = (prm, ckpts, segs, dp, ws, dim, n)
        return ke

    @staticmethod
    def backward(ctx, g):
        prm, ckpts, segs, final, ws, dim, n = ctx.state
        dev = final.u.device
        lam = torch.empty((3 * dim, n), dtype=torch.float64, device=dev)
        # seed: dKE/du^N = g m u^N (walls carry u = 0), formed by the library
        ke_seed(prm, final, float(g), lam)
        other = torch.empty_like(lam)
        dJ = torch.zeros(1, dtype=torch.float64, device=dev)
        for ck, kk in zip(reversed(ckpts), reversed(segs)):
            step_backward(prm, ck, kk, lam, other, dJ, ws)
            lam, other = other, lam
        c0 = ckpts[0]
        accel_backward(prm, c0, lam[2 * dim:], lam[:dim], lam[dim:2 * dim], dJ, ws)
        grad_u0 = torch.zeros((dim, n), dtype=torch.float64, device=dev)
        grad_u0[:, c0.id.long()] = lam[dim:2 * dim]
        ctx.state = None
        return grad_u0, dJ[0], None, None, None, None, None, None, None, None, None


def rollout_ke(u0, nu, params, x0, m, ptype, nsteps, k, precision=FP64, nbr_cap=0,
               pair_tiles=0):
    return SPHRollout.apply(u0, nu, params, x0, m, ptype, nsteps, k, precision, nbr_cap,
                            pair_tiles)
