"""Differentiable rollout: torch.autograd.Function over the HIP step and its
hand-written discrete adjoint, with checkpointed recomputation.

QGRollout.apply(omega0, c, solver, nsteps, segment) returns omega after
nsteps steps.  The forward pass stores omega every `segment` steps (the run
continues from each stored field, so segments restart bit for bit); the
backward pass walks the segments last to first, and in each the library
recomputes the segment's stage inputs from its checkpoint and runs the
adjoint steps in reverse.  Gradients: d/d omega0 (same layout as omega0) and
d/dc (float64, one per member).
"""
import torch


class QGRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega0, c, solver, nsteps, segment):
        if nsteps % segment != 0:
            raise ValueError("nsteps must be a multiple of the checkpoint segment")
        if segment > solver.adj_segment_k:
            raise ValueError("segment exceeds the adjoint storage of the solver")
        solver.set_coef(c.detach().cpu().double().tolist())
        omega = omega0.detach().clone().contiguous()
        nseg = nsteps // segment
        _, ckpt = solver.step(omega, nsteps, save_every=segment)
        ctx.solver = solver
        ctx.segment = segment
        ctx.nseg = nseg
        ctx.c_dtype = c.dtype
        ctx.c_device = c.device
        ctx.save_for_backward(omega0.detach().clone(), ckpt)
        return omega

    @staticmethod
    def backward(ctx, grad_out):
        omega0, ckpt = ctx.saved_tensors
        S = ctx.solver
        lam = grad_out.detach().clone().contiguous().to(S.dtype)
        gc = torch.zeros(S.n, dtype=torch.float64, device=S.device)
        for j in range(ctx.nseg - 1, -1, -1):
            start = omega0 if j == 0 else ckpt[(j - 1) * S.total:j * S.total]
            S.adjoint_step(start.contiguous(), lam, ctx.segment, gc)
        return lam, gc.to(device=ctx.c_device, dtype=ctx.c_dtype), None, None, None
