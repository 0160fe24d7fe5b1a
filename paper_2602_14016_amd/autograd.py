"""The adjoint solve behind torch.autograd.

AdjointCost.apply(omega0, solver, n_steps, obs, ckpt_every) returns the cost
J per member (tensor [B]).  The forward pass runs the checkpointed forward
solve and keeps only the spectral checkpoints (every ckpt_every steps);
backward recomputes each segment from its checkpoint and runs the discrete
adjoint (the exact gradient of the discrete J, Sec. II.A Eqs. (11)-(12) in
the discretise-then-transpose form of Sec. III), scaled member by member by
grad_output.  Memory: O((n_steps / ckpt_every) + 4 ckpt_every) fields per
member instead of the whole trajectory.
"""

import torch


class AdjointCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega0, solver, n_steps, obs, ckpt_every=50):
        omega0 = omega0.detach().contiguous()
        ckpt = torch.empty(solver.checkpoint_bytes(n_steps, ckpt_every), dtype=torch.uint8, device=omega0.device)
        res = solver.forward(omega0, n_steps, obs, want_J=True, ckpt_every=ckpt_every, ckpt=ckpt, want_final=False)
        ctx.solver = solver
        ctx.n_steps = n_steps
        ctx.obs = obs
        ctx.ckpt_every = ckpt_every
        ctx.save_for_backward(ckpt)
        return res["J"]

    @staticmethod
    def backward(ctx, grad_J):
        (ckpt,) = ctx.saved_tensors
        scale = grad_J.detach().to(torch.float64).contiguous()
        g = ctx.solver.adjoint_from_checkpoints(ckpt, ctx.n_steps, ctx.obs, ctx.ckpt_every, scale=scale)
        return g, None, None, None, None


def adjoint_cost(omega0, solver, n_steps, obs, ckpt_every=50):
    return AdjointCost.apply(omega0, solver, n_steps, obs, ckpt_every)
