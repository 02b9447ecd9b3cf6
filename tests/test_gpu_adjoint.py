"""Adjoint gradients on the GPU (through gp_step_real_adjoint and the autograd Function)
against the FP64 adjoint oracle, which is itself pinned by central finite differences.
Bars: FP64 relative 1e-9; FP32 bulk with FP64 gradient reductions 1e-4 (relative to the
gradient's norm for V)."""
import numpy as np
import pytest

import oracle as O
from oracle import gp_adjoint as A
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import banner, oparams

pytestmark = pytest.mark.gpu

CASES = {
    "2dxy_48x40": (dict(geom="2dxy", nx=48, ny=40, nz=1, dx=0.25, dy=0.3, dz=1.0, dt=0.002,
                        gamma=1.0, nu=1.5, lam=4.0, g=30.0, gdd=10.0, R=0.0), 30, 8),
    "2dxz_40x32": (dict(geom="2dxz", nx=40, ny=1, nz=32, dx=0.3, dy=1.0, dz=0.35, dt=0.002,
                        gamma=1.0, nu=4.0, lam=2.0, g=20.0, gdd=12.0, R=0.0), 20, 6),
    "3d_24x20x16": (dict(geom="3d", nx=24, ny=20, nz=16, dx=0.35, dy=0.4, dz=0.45, dt=0.002,
                         gamma=1.0, nu=1.3, lam=2.0, g=25.0, gdd=8.0, R=2.8), 12, 5),
}


def inputs_for(w):
    p = oparams(w)
    shape = p.shape()
    widths = (0.9, 1.1, 1.0)[: len(shape)]
    psi0 = I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                      widths=widths, phase_noise=0.02, amp_noise=0.02, seed=1603)
    ax = I.grid_axes(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"])
    center = [0.5 * (a[1] - a[0]) * 2 for a in ax]
    psi_t = I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                       widths=widths, center=center)
    V = O.harmonic_potential(p) + 0.1 * I.smooth_random_field(shape, p.spacings(), 1.0, 1605)
    return p, psi0, psi_t, V


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_gradients_match_oracle(name, prec, gpu_lib):
    import torch
    from paper_1601_04640_amd.adjoint import evolve_real, overlap_loss
    from paper_1601_04640_amd.binding import Solver
    w, nsteps, K = CASES[name]
    banner("adjoint", name, prec, nsteps, K)
    p, psi0, psi_t, V = inputs_for(w)
    ref = A.overlap_gradients(psi0, psi_t, p, nsteps, V=V)
    s = Solver(w, prec=prec)
    cd = s.cdtype
    dev = "cuda:0"
    psi0_t = torch.from_numpy(psi0).to(dev, cd).requires_grad_(True)
    V_t = torch.from_numpy(V).to(dev).requires_grad_(True)
    g_t = torch.tensor(w["g"], dtype=torch.float64, device=dev, requires_grad=True)
    gdd_t = torch.tensor(w["gdd"], dtype=torch.float64, device=dev, requires_grad=True)
    psiT = evolve_real(s, psi0_t, V_t, g_t, gdd_t, nsteps, K)
    L = overlap_loss(psiT, torch.from_numpy(psi_t).to(dev, cd), p.dV())
    L.backward()
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert abs(float(L) - ref["loss"]) <= tol * max(abs(ref["loss"]), 1e-3)
    gV = V_t.grad.cpu().numpy()
    err_v = np.linalg.norm(gV - ref["dV"]) / np.linalg.norm(ref["dV"])
    assert err_v <= tol, err_v
    assert abs(float(g_t.grad) - ref["dg"]) <= tol * abs(ref["dg"]), (float(g_t.grad), ref["dg"])
    assert abs(float(gdd_t.grad) - ref["dgdd"]) <= tol * abs(ref["dgdd"])
    lam0 = 0.5 * psi0_t.grad.cpu().numpy().astype(np.complex128)
    err_l = np.linalg.norm(lam0 - ref["lambda0"]) / np.linalg.norm(ref["lambda0"])
    assert err_l <= tol, err_l
    s.close()


def test_adjoint_step_abi_accumulates(gpu_lib):
    """Two calls accumulate into gradV / grad_g / grad_g_dd (the ABI contract)."""
    import torch
    from paper_1601_04640_amd import binding as B
    from paper_1601_04640_amd.binding import Solver
    w, _, _ = CASES["2dxy_48x40"]
    banner("adjoint accumulate")
    p, psi0, psi_t, V = inputs_for(w)
    s = Solver(w, prec="fp64")
    s.set_potential(V)
    psi = torch.from_numpy(psi0).to("cuda:0")
    outs = []
    for reps in (1, 2):
        lam = torch.from_numpy(-psi_t * p.dV()).to("cuda:0").contiguous()
        gV = torch.zeros(V.shape, dtype=torch.float64, device="cuda:0")
        gg = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        gd = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for _ in range(reps):
            l2 = lam.clone()
            B.gp_step_real_adjoint(s.ctx, psi.data_ptr(), l2.data_ptr(), gV.data_ptr(),
                                   gg.data_ptr(), gd.data_ptr())
        torch.cuda.synchronize()
        outs.append((gV.cpu().numpy(), float(gg), float(gd)))
    np.testing.assert_allclose(outs[1][0], 2 * outs[0][0], rtol=1e-12, atol=1e-300)
    assert abs(outs[1][1] - 2 * outs[0][1]) <= 1e-12 * abs(outs[0][1])
    assert abs(outs[1][2] - 2 * outs[0][2]) <= 1e-12 * abs(outs[0][2])
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_energy_loss_gradients_match_oracle(name, prec, gpu_lib):
    """L = E(psi(T)): the terminal costate and direct terms of the energy loss, chained
    through the adjoint steps, against the FP64 oracle (itself pinned by central
    differences)."""
    import torch
    from paper_1601_04640_amd.adjoint import energy_loss, evolve_real
    from paper_1601_04640_amd.binding import Solver
    w, nsteps, K = CASES[name]
    banner("adjoint energy loss", name, prec, nsteps, K)
    p, psi0, _, V = inputs_for(w)
    ref = A.energy_gradients(psi0, p, nsteps, V=V)
    s = Solver(w, prec=prec)
    dev = "cuda:0"
    psi0_t = torch.from_numpy(psi0).to(dev, s.cdtype).requires_grad_(True)
    V_t = torch.from_numpy(V).to(dev).requires_grad_(True)
    g_t = torch.tensor(w["g"], dtype=torch.float64, device=dev, requires_grad=True)
    gdd_t = torch.tensor(w["gdd"], dtype=torch.float64, device=dev, requires_grad=True)
    L = energy_loss(evolve_real(s, psi0_t, V_t, g_t, gdd_t, nsteps, K), V_t, g_t, gdd_t, s)
    L.backward()
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert abs(float(L) - ref["loss"]) <= (1e-12 if prec == "fp64" else 1e-6) * abs(ref["loss"])
    gV = V_t.grad.cpu().numpy()
    err_v = np.linalg.norm(gV - ref["dV"]) / np.linalg.norm(ref["dV"])
    assert err_v <= tol, err_v
    assert abs(float(g_t.grad) - ref["dg"]) <= tol * abs(ref["dg"]), (float(g_t.grad), ref["dg"])
    assert abs(float(gdd_t.grad) - ref["dgdd"]) <= tol * abs(ref["dgdd"]), \
        (float(gdd_t.grad), ref["dgdd"])
    lam0 = 0.5 * psi0_t.grad.cpu().numpy().astype(np.complex128)
    err_l = np.linalg.norm(lam0 - ref["lambda0"]) / np.linalg.norm(ref["lambda0"])
    assert err_l <= tol, err_l
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solver_reused_between_forward_and_backward(prec, gpu_lib):
    """Two forwards on one solver with different V and couplings, then backward through
    the first: its gradients are those of its own V, g and g_dd (the oracle adjoint)."""
    import torch
    from paper_1601_04640_amd.adjoint import evolve_real, overlap_loss
    from paper_1601_04640_amd.binding import Solver
    w, nsteps, K = CASES["2dxy_48x40"]
    banner("adjoint solver reuse", prec)
    p, psi0, psi_t, V = inputs_for(w)
    ref = A.overlap_gradients(psi0, psi_t, p, nsteps, V=V)
    s = Solver(w, prec=prec)
    dev = "cuda:0"

    def forward(Vx, g, gdd):
        p0 = torch.from_numpy(psi0).to(dev, s.cdtype).requires_grad_(True)
        Vt = torch.from_numpy(Vx).to(dev).requires_grad_(True)
        gt = torch.tensor(g, dtype=torch.float64, device=dev, requires_grad=True)
        gdt = torch.tensor(gdd, dtype=torch.float64, device=dev, requires_grad=True)
        L = overlap_loss(evolve_real(s, p0, Vt, gt, gdt, nsteps, K),
                         torch.from_numpy(psi_t).to(dev, s.cdtype), p.dV())
        return L, Vt, gt, gdt
    L1, V1, g1, gdd1 = forward(V, w["g"], w["gdd"])
    L2, _, _, _ = forward(1.3 * V, 0.5 * w["g"], 2.0 * w["gdd"])   # reuses the solver
    L1.backward()
    tol = 1e-9 if prec == "fp64" else 1e-4
    err_v = np.linalg.norm(V1.grad.cpu().numpy() - ref["dV"]) / np.linalg.norm(ref["dV"])
    assert err_v <= tol, err_v
    assert abs(float(g1.grad) - ref["dg"]) <= tol * abs(ref["dg"])
    assert abs(float(gdd1.grad) - ref["dgdd"]) <= tol * abs(ref["dgdd"])
    s.close()
