"""torch.autograd.Function around the hand-written real-time adjoint step.

`evolve_real(solver, psi0, V, g, gdd, nsteps, K)` returns psi(T) after `nsteps` real-time
steps, differentiable with respect to psi0, the grid potential V and the couplings g and
g_dd.  Forward keeps a checkpoint every K steps.  Backward walks the segments in reverse:
it recomputes the K states of a segment from its checkpoint, then calls
`gp_step_real_adjoint` once per step, newest first.  Every step runs in the library's
kernels; this module only moves device pointers.

PyTorch's gradient of a real loss with respect to a complex tensor is twice the
conjugate Wirtinger derivative, so the costate is lambda = grad/2 and grad(psi0) = 2 lambda_0.
"""
from __future__ import annotations

import torch

from . import binding as B


class RealTimeEvolution(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, V, g, gdd, solver, nsteps, K):
        if nsteps < 1 or K < 1:
            raise ValueError("nsteps and K must be positive")
        solver.set_potential(V.detach().to(solver.device, torch.float64))
        solver.set_couplings(float(g), float(gdd))
        solver.set_psi(psi0.detach())
        ckpts = []
        done = 0
        while done < nsteps:
            ckpts.append(solver.get_psi_device())
            k = min(K, nsteps - done)
            solver.step_real(k)
            done += k
        psiT = solver.get_psi_device()
        ctx.solver, ctx.nsteps, ctx.K, ctx.ckpts = solver, nsteps, K, ckpts
        ctx.psi0_dtype = psi0.dtype
        return psiT

    @staticmethod
    def backward(ctx, grad_psiT):
        s = ctx.solver
        dev = s.device
        lam = (0.5 * grad_psiT).to(device=dev, dtype=s.cdtype).contiguous()
        gradV = torch.zeros(s.shape, dtype=torch.float64, device=dev)
        gg = torch.zeros(1, dtype=torch.float64, device=dev)
        ggdd = torch.zeros(1, dtype=torch.float64, device=dev)
        for seg in range(len(ctx.ckpts) - 1, -1, -1):
            start = seg * ctx.K
            k = min(ctx.K, ctx.nsteps - start)
            s.set_psi(ctx.ckpts[seg])
            states = [ctx.ckpts[seg]]
            for _ in range(k - 1):
                s.step_real(1)
                states.append(s.get_psi_device())
            for i in range(k - 1, -1, -1):
                B.gp_step_real_adjoint(s.ctx, states[i].data_ptr(), lam.data_ptr(),
                                       gradV.data_ptr(), gg.data_ptr(), ggdd.data_ptr())
        s.stream.synchronize()
        grad_psi0 = (2.0 * lam).to(ctx.psi0_dtype)
        return grad_psi0, gradV, gg[0], ggdd[0], None, None, None


def evolve_real(solver, psi0, V, g, gdd, nsteps: int, K: int):
    """psi(T) after nsteps real-time steps on `solver` (a binding.Solver), differentiable
    in psi0 (complex), V (float64 grid) and the 0-dim float64 tensors g, gdd."""
    return RealTimeEvolution.apply(psi0, V, g, gdd, solver, nsteps, K)


def overlap_loss(psiT, psi_t, dV):
    """1 - |sum conj(psi_t) psi(T) dV|^2 (computed by torch on the device)."""
    c = torch.sum(torch.conj(psi_t) * psiT) * dV
    return 1.0 - (c.real ** 2 + c.imag ** 2)
