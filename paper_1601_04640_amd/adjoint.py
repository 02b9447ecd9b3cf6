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

import math

import numpy as np
import torch

from . import binding as B


class RealTimeEvolution(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, V, g, gdd, solver, nsteps, K):
        if nsteps < 1 or K < 1:
            raise ValueError("nsteps and K must be positive")
        Vd = V.detach().to(solver.device, torch.float64).contiguous()
        solver.set_potential(Vd)
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
        # the potential and couplings of this forward: the solver may be reused (another
        # forward, a quench) before backward runs, so backward sets them again
        ctx.V, ctx.g, ctx.gdd = Vd, float(g), float(gdd)
        return psiT

    @staticmethod
    def backward(ctx, grad_psiT):
        s = ctx.solver
        dev = s.device
        s.set_potential(ctx.V)
        s.set_couplings(ctx.g, ctx.gdd)
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


class EnergyLoss(torch.autograd.Function):
    """L = E(psi(T)): the library's FP64 energy (gp_energy) of a final state, with the
    potential V and couplings g, g_dd it is evaluated at.  Backward gives the terminal
    costate dE/d conj(psi) = (T_disc + V + g_c n + g_dd Phi) psi dV, with Phi from the
    library's dipolar convolution and T_disc the forward-difference kinetic operator of the
    energy (minus half the second difference over h^2 along each axis), taken as zero on
    the boundary rows (psi(T) is zero there); and the direct terms dE/dV = n dV,
    dE/dg = 1/2 sum n^2 dV (times the quasi-2D contact factor), dE/dg_dd = 1/2 sum Phi n dV."""

    @staticmethod
    def forward(ctx, psiT, V, g, gdd, solver):
        Vd = V.detach().to(solver.device, torch.float64).contiguous()
        solver.set_potential(Vd)
        solver.set_couplings(float(g), float(gdd))
        solver.set_psi(psiT.detach())
        E = solver.energy()["energy"]
        phi = solver.dipolar_potential_device().to(torch.float64)
        psi = solver.get_psi_device().to(torch.complex128)
        solver.stream.synchronize()
        ctx.save_for_backward(psi, phi, Vd)
        ctx.solver, ctx.g, ctx.gdd, ctx.psi_dtype = solver, float(g), float(gdd), psiT.dtype
        return torch.tensor(E, dtype=torch.float64, device=solver.device)

    @staticmethod
    def backward(ctx, gE):
        psi, phi, Vd = ctx.saved_tensors
        s = ctx.solver
        w = s.params
        geom = w["geom"]
        if geom == "3d":
            hs, cfac = (w["dz"], w["dy"], w["dx"]), 1.0
        else:
            hs = (w["dy"] if geom == "2dxy" else w["dz"], w["dx"])
            perp = w["lam"] if geom == "2dxy" else w["nu"]
            cfac = math.sqrt(perp) / math.sqrt(2.0 * math.pi)   # 1/(sqrt(2 pi) d)
        dV = float(np.prod(hs))
        n = psi.real ** 2 + psi.imag ** 2
        tpsi = torch.zeros_like(psi)
        for ax, h in enumerate(hs):
            d = torch.diff(psi, dim=ax)
            lo = [0, 0] * psi.ndim
            hi = [0, 0] * psi.ndim
            # F.pad counts dimensions from the last one
            lo[2 * (psi.ndim - 1 - ax) + 0] = 1
            hi[2 * (psi.ndim - 1 - ax) + 1] = 1
            tpsi = tpsi + 0.5 * (torch.nn.functional.pad(d, lo) -
                                 torch.nn.functional.pad(d, hi)) / (h * h)
        gc = ctx.g * cfac
        lam = (tpsi + (Vd + gc * n + ctx.gdd * phi) * psi) * dV
        lam = _zero_boundary(lam)
        grad_psi = (2.0 * gE * lam).to(ctx.psi_dtype)
        gV = gE * n * dV
        gg = gE * 0.5 * torch.sum(n * n) * dV * cfac
        ggdd = gE * 0.5 * torch.sum(phi * n) * dV
        return grad_psi, gV, gg, ggdd, None


def _zero_boundary(x):
    x = x.clone()
    for ax in range(x.ndim):
        x.select(ax, 0).zero_()
        x.select(ax, x.shape[ax] - 1).zero_()
    return x


def energy_loss(psiT, V, g, gdd, solver):
    """E(psi(T)) at potential V and couplings g, g_dd (0-dim float64 tensors),
    differentiable in all four; `solver` is a binding.Solver of the grid."""
    return EnergyLoss.apply(psiT, V, g, gdd, solver)
