"""The coupled run as a differentiable function for torch.autograd.

``trajectory(w, gamma, tau, body_force, n_steps, k)`` advances a workload's atoms and
lattice n_steps coupled steps and returns the atoms' final displacement X(T) - X(0) and
velocity [N, 3].  Its backward pass is the library's hand-written discrete adjoint
(lb_backward), with the forward recomputed from checkpoints taken every k steps, so that
gradients with respect to the friction gamma, the relaxation time tau and the external
force-density field reach any loss built from those outputs.
"""
from __future__ import annotations

import copy

import torch

from . import _abi as A
from .coupled import CoupledLB, params_from_workload


class CoupledTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, tau, body_force, w, n_steps, k, storage):
        p = params_from_workload(w, storage)
        p.gamma = float(gamma)
        p.tau = float(tau)
        p.bf_kind = A.LB_BF_FIELD
        field = body_force.detach().to(torch.float32).contiguous()
        sim = CoupledLB(p, w.x0, w.v0, w.bonds, field.cpu().numpy(),
                        device=field.device if field.is_cuda else "cuda",
                        charges=getattr(w, "charges", None))
        ckpt = sim.run_checkpointed(int(n_steps), int(k))
        disp = sim.displacement()
        _, _, _, v = sim.read_fields()
        ctx.sim, ctx.ckpt = sim, ckpt
        ctx.meta = (gamma, tau, body_force)
        return disp, v

    @staticmethod
    def backward(ctx, g_disp, g_v):
        gamma, tau, body_force = ctx.meta
        sim = ctx.sim
        zeros = torch.zeros((sim.N, 3), dtype=torch.float32, device=sim.device)
        gX = g_disp if g_disp is not None else zeros
        gv = g_v if g_v is not None else None
        out = sim.backward(ctx.ckpt, gX, gv, want_body_force=ctx.needs_input_grad[2], want_initial=False)
        sim.close()
        ctx.sim = ctx.ckpt = None
        as_like = lambda val, ref: torch.as_tensor(val, dtype=ref.dtype, device=ref.device) if torch.is_tensor(ref) else val
        d_gamma = as_like(out["gamma"], gamma) if ctx.needs_input_grad[0] else None
        d_tau = as_like(out["tau"], tau) if ctx.needs_input_grad[1] else None
        d_b = None
        if ctx.needs_input_grad[2]:
            d_b = out["body_force"].to(body_force.dtype).to(body_force.device).reshape(body_force.shape)
        return d_gamma, d_tau, d_b, None, None, None, None


def trajectory(w, gamma, tau, body_force, n_steps: int, k: int = 20, storage: str = "f32"):
    """(X(T) - X(0), v(T)) of workload w, differentiable in gamma, tau and body_force
    ([3, nz, ny, nx]); the workload's own gamma, tau and body force are replaced."""
    return CoupledTrajectory.apply(gamma, tau, body_force, copy.copy(w), n_steps, k, storage)
