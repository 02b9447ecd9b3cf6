"""Full-size workloads, run the way bench.py runs them (graph-replayed step loops), checked
against the FP64 oracle where it finishes in seconds, against oracle-written fixtures
(tests/golden/make_fullsize.py) where it does not, and against properties that hold at
any size (norm conservation in real time, monotone imaginary-time energy, central finite
differences of the loss for the adjoint gradients)."""
import functools
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import gp_adjoint as A
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import (FP32_E_TOL, FP32_PART_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            banner, obs_close, oparams, rel_l2)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def sampled(psi, g):
    idx = np.asarray(g["sample_index"])
    return psi.ravel()[idx], np.asarray(g["psi_re"]) + 1j * np.asarray(g["psi_im"])


def bars(prec):
    if prec == "fp64":
        return FP64_PSI_TOL, dict(tol=FP64_E_TOL)
    return FP32_PSI_TOL, dict(tol=FP32_E_TOL, part_tol=FP32_PART_TOL)


# ------------------------------------------------------------- imag3d 64^3, 500 steps
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_imag3d_64_500_steps(prec, gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    g = golden("imag3d_64_500.json")
    w = I.WORKLOADS["imag3d_64"]
    banner("imag3d_64 500 steps", prec)
    s = Solver(w, prec=prec)
    s.set_psi(I.psi0_imag3d_64())
    s.step_imag(g["steps"])
    psi = s.get_psi()
    got, ref = sampled(psi, g)
    ptol, etol = bars(prec)
    assert rel_l2(got, ref) <= ptol, rel_l2(got, ref)
    bad = obs_close(s.energy(), g["final"], **etol)
    assert not bad, bad
    hist = s.history(g["steps"])
    assert len(hist) == g["steps"]
    e_ref = np.asarray(g["history_energy"])
    mu_ref = np.asarray(g["history_mu"])
    e = np.array([h["energy"] for h in hist])
    mu = np.array([h["mu"] for h in hist])
    assert np.max(np.abs(e - e_ref) / np.abs(e_ref)) <= etol["tol"]
    assert np.max(np.abs(mu - mu_ref) / np.abs(mu_ref)) <= etol["tol"]
    assert np.all(np.diff(e) <= etol["tol"] * abs(e[-1]))   # imaginary time lowers E
    s.close()


# -------------------------------------------------- real3d 128x96x80 quench workload
@functools.lru_cache(maxsize=None)
def oracle_quench_10():
    w = I.WORKLOADS["real3d_128x96x80"]
    return O.run(I.psi0_real3d_128x96x80(), oparams(w), False, 10)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_real3d_128x96x80_steps_match_oracle(prec, gpu_lib):
    """Ten real-time steps of the quench grid (g = 15) from the seeded start."""
    from paper_1601_04640_amd.binding import Solver
    w = I.WORKLOADS["real3d_128x96x80"]
    banner("real3d_128x96x80 10 steps", prec)
    s = Solver(w, prec=prec)
    s.set_psi(I.psi0_real3d_128x96x80())
    s.step_real(10)
    ref = oracle_quench_10()
    ptol, etol = bars(prec)
    err = rel_l2(s.get_psi(), ref)
    assert err <= ptol, err
    bad = obs_close(s.energy(), O.observables(ref, oparams(w)), **etol)
    assert not bad, bad
    s.close()


def test_real3d_128x96x80_quench_properties(gpu_lib):
    """FP64 relaxation at g = 20 (dt 0.002), quench to g = 15, 2000 real-time steps:
    the norm is conserved to roundoff, the weaker repulsion contracts the cloud, and the
    FP32 run from the same state stays within the FP32 bar of the FP64 run."""
    from paper_1601_04640_amd.binding import Solver
    w = dict(I.WORKLOADS["real3d_128x96x80"])
    banner("real3d_128x96x80 quench 2000 steps")
    gs = Solver(dict(w, g=w["g_ground"], dt=0.002), prec="fp64")
    gs.set_psi(I.psi0_real3d_128x96x80())
    gs.step_imag(1500)
    psi_g = gs.get_psi()
    gs.close()
    runs = {}
    for prec in ("fp64", "fp32"):
        s = Solver(w, prec=prec)
        s.set_psi(psi_g)
        s.step_real(2000)
        runs[prec] = (s.history(2000), s.get_psi(), s.energy())
        s.close()
    hist, psi64, end64 = runs["fp64"]
    norms = np.array([h["norm"] for h in hist] + [end64["norm"]])
    assert np.max(np.abs(norms - 1.0)) <= 1e-11
    rx = np.array([h["rms"][0] for h in hist])
    assert rx.min() < rx[0] - 1e-3                          # contraction after the quench
    hist32, psi32, end32 = runs["fp32"]
    n32 = np.array([h["norm"] for h in hist32])
    assert np.max(np.abs(n32 - 1.0)) <= 1e-5
    print("fp32 vs fp64 after 2000 steps: psi rel", rel_l2(psi32, psi64),
          "energy rel", abs(end32["energy"] - end64["energy"]) / abs(end64["energy"]))
    assert rel_l2(psi32, psi64) <= 1e-3
    assert abs(end32["energy"] - end64["energy"]) <= 1e-5 * abs(end64["energy"])


# ----------------------------------------------------------------- real3d 256^3
@functools.lru_cache(maxsize=None)
def oracle_256_one_step():
    w = I.WORKLOADS["real3d_256"]
    return O.step(I.psi0_real3d_256(), oparams(w), False)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_real3d_256_step_matches_oracle(prec, gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    w = I.WORKLOADS["real3d_256"]
    banner("real3d_256 one step", prec)
    s = Solver(w, prec=prec)
    s.set_psi(I.psi0_real3d_256())
    s.step_real(1)
    err = rel_l2(s.get_psi(), oracle_256_one_step())
    ptol, _ = bars(prec)
    assert err <= ptol, err
    # then the workload's 500 steps: the norm stays 1
    s.step_real(499)
    nrm = np.array([h["norm"] for h in s.history(499)])
    assert np.max(np.abs(nrm - 1.0)) <= (1e-11 if prec == "fp64" else 1e-5)
    s.close()


# ---------------------------------------------- real2dXY 256^2 adjoint, 4000 steps
def overlap_L(psi, target, dV):
    c = np.sum(np.conj(target) * psi) * dV
    return 1.0 - abs(c) ** 2


def forward_loss(w, prec, psi0, V, target, nsteps, g=None, gdd=None):
    from paper_1601_04640_amd.binding import Solver
    s = Solver(w, prec=prec)
    s.set_potential(V)
    if g is not None:
        s.set_couplings(g, gdd)
    s.set_psi(psi0)
    s.step_real(nsteps)
    L = overlap_L(s.get_psi(), target, oparams(w).dV())
    s.close()
    return L


def gpu_gradients(w, prec, psi0, V, target, nsteps, K):
    import torch
    from paper_1601_04640_amd.adjoint import evolve_real, overlap_loss
    from paper_1601_04640_amd.binding import Solver
    s = Solver(w, prec=prec)
    dev = "cuda:0"
    p0 = torch.from_numpy(psi0).to(dev, s.cdtype).requires_grad_(True)
    Vt = torch.from_numpy(V).to(dev).requires_grad_(True)
    gt = torch.tensor(w["g"], dtype=torch.float64, device=dev, requires_grad=True)
    gdt = torch.tensor(w["gdd"], dtype=torch.float64, device=dev, requires_grad=True)
    L = overlap_loss(evolve_real(s, p0, Vt, gt, gdt, nsteps, K),
                     torch.from_numpy(target).to(dev, s.cdtype), oparams(w).dV())
    L.backward()
    out = dict(loss=float(L), dV=Vt.grad.cpu().numpy(), dg=float(gt.grad), dgdd=float(gdt.grad))
    s.close()
    return out


def adjoint_2d_inputs():
    w = I.WORKLOADS["real2dxy_256"]
    p = oparams(w)
    V = O.harmonic_potential(p) + I.trap_perturbation_real2dxy_256()
    target = I.displaced_target(w, 1610, widths=(1.0 / np.sqrt(1.5), 1.0))
    return w, I.psi0_real2dxy_256(), V, target


def check_fd(w, prec, psi0, V, target, nsteps, grads, params=("g", "gdd"), npoints=3,
             tol=1e-4):
    """Central differences of the FP64 forward loss against the adjoint gradients."""
    for name in params:
        x = w[name]
        h = 1e-4 * abs(x)
        args = dict(g=w["g"], gdd=w["gdd"])
        args[name] = x + h
        Lp = forward_loss(w, "fp64", psi0, V, target, nsteps, **args)
        args[name] = x - h
        Lm = forward_loss(w, "fp64", psi0, V, target, nsteps, **args)
        fd = (Lp - Lm) / (2 * h)
        key = "dg" if name == "g" else "dgdd"
        print(f"{prec} d/d{name}: adjoint {grads[key]:.10e} fd {fd:.10e}")
        assert abs(grads[key] - fd) <= tol * abs(fd), (name, grads[key], fd)
    dV = grads["dV"]
    gmax = np.max(np.abs(dV))
    for flat in np.argsort(np.abs(dV).ravel())[-npoints:]:
        idx = np.unravel_index(flat, dV.shape)
        h = 1e-3
        Vp = V.copy()
        Vp[idx] += h
        Lp = forward_loss(w, "fp64", psi0, Vp, target, nsteps)
        Vp[idx] -= 2 * h
        Lm = forward_loss(w, "fp64", psi0, Vp, target, nsteps)
        fd = (Lp - Lm) / (2 * h)
        print(f"{prec} dL/dV{idx}: adjoint {dV[idx]:.10e} fd {fd:.10e}")
        assert abs(dV[idx] - fd) <= tol * gmax, (idx, dV[idx], fd)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_real2dxy_256_4000_steps_fd(prec, gpu_lib):
    w, psi0, V, target = adjoint_2d_inputs()
    banner("adjoint real2dxy_256 4000 steps K=50", prec)
    grads = gpu_gradients(w, prec, psi0, V, target, 4000, 50)
    L64 = forward_loss(w, "fp64", psi0, V, target, 4000)
    assert abs(grads["loss"] - L64) <= (1e-12 if prec == "fp64" else 1e-5)
    check_fd(w, prec, psi0, V, target, 4000, grads, tol=1e-6 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_real2dxy_256_matches_oracle(prec, gpu_lib):
    """200 steps at full size, checkpoints every 50, against the FP64 adjoint oracle."""
    w, psi0, V, target = adjoint_2d_inputs()
    banner("adjoint real2dxy_256 200 steps vs oracle", prec)
    ref = A.overlap_gradients(psi0, target, oparams(w), 200, V=V)
    grads = gpu_gradients(w, prec, psi0, V, target, 200, 50)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert np.linalg.norm(grads["dV"] - ref["dV"]) <= tol * np.linalg.norm(ref["dV"])
    assert abs(grads["dg"] - ref["dg"]) <= tol * abs(ref["dg"])
    assert abs(grads["dgdd"] - ref["dgdd"]) <= tol * abs(ref["dgdd"])


# ------------------------------------------------- 128^3 adjoint, 200 steps, K = 20
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint3d_128_fd(prec, gpu_lib):
    w = I.WORKLOADS["adjoint3d_128"]
    p = oparams(w)
    banner("adjoint3d_128 200 steps K=20", prec)
    psi0 = I.psi0_adjoint3d_128()
    V = O.harmonic_potential(p)
    target = I.displaced_target(w, 1611, widths=(1.0 / np.sqrt(3.0), 1.0, 1.0))
    grads = gpu_gradients(w, prec, psi0, V, target, w["steps"], w["K"])
    check_fd(w, prec, psi0, V, target, w["steps"], grads, params=("gdd",), npoints=2,
             tol=1e-6 if prec == "fp64" else 1e-4)


# ------------------------------------------- batched 2D ensemble, 1000 imaginary steps
def test_ensemble_1000_steps(gpu_lib):
    from paper_1601_04640_amd.binding import Batch
    g = golden("ensemble_imag_1000.json")
    ens = I.batched_ensemble()
    banner("ensemble 192 x 1000 imaginary steps fp32")
    b = Batch(ens, prec="fp32")
    for i, w in enumerate(ens):
        b.set_psi(i, I.psi0_instance(w, seed=[1606, i]))
    b.step_imag(g["steps"])
    energies = b.energy()
    for rec in g["instances"]:
        i = rec["index"]
        got, ref = sampled(b.get_psi(i), rec)
        assert rel_l2(got, ref) <= FP32_PSI_TOL, (i, rel_l2(got, ref))
        bad = obs_close(energies[i], rec["final"], FP32_E_TOL, part_tol=FP32_PART_TOL)
        assert not bad, (i, bad)
    for i in range(len(ens)):
        assert abs(energies[i]["norm"] - 1.0) <= 1e-6, i
        e = np.array([h["energy"] for h in b.history(i, g["steps"])])
        assert np.all(np.diff(e) <= FP32_E_TOL * abs(e[-1])), i
    b.close()
