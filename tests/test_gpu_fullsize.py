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
from tests.gpu_util import (FP32_E_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            assert_psi_close, banner, obs_close, oparams, rel_l2)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def sampled(psi, g):
    idx = np.asarray(g["sample_index"])
    return psi.ravel()[idx], np.asarray(g["psi_re"]) + 1j * np.asarray(g["psi_im"])


def bars(prec, real_time=False):
    """psi bar and observable bars.  Long FP32 real-time runs compare the observables per
    particle (divided by the state's norm), since FP32 rounding moves the norm that the
    exact evolution conserves (by about 1e-6 over 2000 steps); the norm drift is then
    checked on its own."""
    if prec == "fp64":
        return FP64_PSI_TOL, dict(tol=FP64_E_TOL)
    return FP32_PSI_TOL, dict(tol=FP32_E_TOL, per_particle=real_time)


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
    assert_psi_close(got, ref, ptol)
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
    assert_psi_close(s.get_psi(), ref, ptol)
    bad = obs_close(s.energy(), O.observables(ref, oparams(w)), **etol)
    assert not bad, bad
    s.close()


@functools.lru_cache(maxsize=None)
def gpu_ground_state_128x96x80():
    """The FP64 imaginary-time ground state at g = 20 (dt 0.002, 1500 steps) on the GPU,
    the start of both quench runs, with its observables."""
    from paper_1601_04640_amd.binding import Solver
    w = dict(I.WORKLOADS["real3d_128x96x80"])
    gs = Solver(dict(w, g=w["g_ground"], dt=0.002), prec="fp64")
    gs.set_psi(I.psi0_real3d_128x96x80())
    gs.step_imag(1500)
    psi, ob = gs.get_psi(), gs.energy()
    gs.close()
    return psi, ob


def check_records(recs, ref_recs, every, etol, what):
    """Per-step records of the GPU run against the oracle's, every `every` steps."""
    for k, r in enumerate(ref_recs):
        bad = obs_close(recs[k * every], r, **etol)
        assert not bad, (what, k * every, bad)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_real3d_128x96x80_quench_vs_oracle(prec, gpu_lib):
    """The whole quench workload against the oracle: the FP64 ground state at g = 20
    (1500 imaginary-time steps), then g = 15 and 2000 real-time steps in `prec`.  The
    ground state, the observables every 10 steps, the final observables and psi at 1024
    sampled points are held at the parity bars; the norm stays 1."""
    from paper_1601_04640_amd.binding import Solver
    g = golden("quench_128x96x80.json")
    w = I.WORKLOADS["real3d_128x96x80"]
    banner("real3d_128x96x80 quench 1500 + 2000 steps", prec)
    psi_g, ob_g = gpu_ground_state_128x96x80()
    idx = np.asarray(g["sample_index"])
    ref_g = np.asarray(g["ground_re"]) + 1j * np.asarray(g["ground_im"])
    l2, mx = assert_psi_close(psi_g.ravel()[idx], ref_g, FP64_PSI_TOL, "ground state")
    print(f"ground state vs oracle: rel-L2 {l2:.2e}, max {mx:.2e}")
    assert not obs_close(ob_g, g["ground"], FP64_E_TOL)
    s = Solver(w, prec=prec)
    s.set_psi(psi_g)
    s.step_real(g["steps"])
    ptol, etol = bars(prec, real_time=True)
    recs = s.history(g["steps"])
    assert len(recs) == g["steps"]
    check_records(recs, g["records"], g["every"], etol, "quench")
    end = s.energy()
    assert not obs_close(end, g["final"], **etol)
    got = s.get_psi().ravel()[idx]
    ref = np.asarray(g["psi_re"]) + 1j * np.asarray(g["psi_im"])
    l2, mx = assert_psi_close(got, ref, ptol, "after 2000 steps")
    print(f"{prec} after 2000 real-time steps vs oracle: rel-L2 {l2:.2e}, max {mx:.2e}, "
          f"energy rel {abs(end['energy'] - g['final']['energy']) / abs(g['final']['energy']):.2e}")
    norms = np.array([h["norm"] for h in recs] + [end["norm"]])
    assert np.max(np.abs(norms - 1.0)) <= (1e-11 if prec == "fp64" else 1e-5)
    s.close()


# ----------------------------------------------------------------- real3d 256^3
@functools.lru_cache(maxsize=None)
def oracle_256_one_step():
    w = I.WORKLOADS["real3d_256"]
    return O.step(I.psi0_real3d_256(), oparams(w), False)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_real3d_256_500_steps_vs_oracle(prec, gpu_lib):
    """The large workload: the first step against the oracle on the whole grid, then the
    500 steps against the oracle's fixture (observables every 10 steps and at the end,
    psi at 4096 sampled points)."""
    from paper_1601_04640_amd.binding import Solver
    g = golden("real3d_256_500.json")
    w = I.WORKLOADS["real3d_256"]
    banner("real3d_256 500 steps", prec)
    s = Solver(w, prec=prec)
    s.set_psi(I.psi0_real3d_256())
    s.step_real(1)
    ptol, etol = bars(prec, real_time=True)
    assert_psi_close(s.get_psi(), oracle_256_one_step(), ptol, "one step")
    s.step_real(g["steps"] - 1)
    recs = s.history(g["steps"])
    assert len(recs) == g["steps"]
    check_records(recs, g["records"], g["every"], etol, "real3d_256")
    end = s.energy()
    assert not obs_close(end, g["final"], **etol)
    got, ref = sampled(s.get_psi(), g)
    l2, mx = assert_psi_close(got, ref, ptol, "after 500 steps")
    print(f"{prec} 256^3 after 500 steps vs oracle: rel-L2 {l2:.2e}, max {mx:.2e}")
    nrm = np.array([h["norm"] for h in recs] + [end["norm"]])
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


def check_adjoint_fixture(grads, g, prec):
    """Loss and gradients against the adjoint oracle's fixture: gradients at FP64 1e-9
    relative, FP32 1e-4; dL/dV by its norm and at the sampled points.  The loss
    1 - |c|^2, c = <psi_t, psi(T)> dV, is a function of the final state: with both states
    normalised, |dc| <= ||d psi|| (Cauchy-Schwarz), so |dL| <= 2 |c| ||d psi||, and the
    loss is held at 2 |c| times the psi bar (rel-L2 1e-10 FP64, 2e-5 FP32)."""
    tol = 1e-9 if prec == "fp64" else 1e-4
    c = np.sqrt(max(1.0 - g["loss"], 0.0))
    ltol = 2.0 * c * (FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL)
    assert abs(grads["loss"] - g["loss"]) <= ltol, (grads["loss"], g["loss"], ltol)
    assert abs(grads["dg"] - g["dg"]) <= tol * abs(g["dg"]), (grads["dg"], g["dg"])
    assert abs(grads["dgdd"] - g["dgdd"]) <= tol * abs(g["dgdd"]), (grads["dgdd"], g["dgdd"])
    dV = grads["dV"]
    assert abs(np.linalg.norm(dV) - g["dV_norm"]) <= tol * g["dV_norm"]
    got = dV.ravel()[np.asarray(g["dV_index"])]
    ref = np.asarray(g["dV_sample"])
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_real2dxy_256_4000_steps_fd(prec, gpu_lib):
    """The 4000-step adjoint workload (checkpoints every 50): against the adjoint oracle's
    fixture of the same run, and against central differences of the FP64 GPU forward."""
    w, psi0, V, target = adjoint_2d_inputs()
    banner("adjoint real2dxy_256 4000 steps K=50", prec)
    grads = gpu_gradients(w, prec, psi0, V, target, 4000, 50)
    check_adjoint_fixture(grads, golden("adjoint_real2dxy_256_4000.json"), prec)
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
    check_adjoint_fixture(grads, golden("adjoint3d_128_200.json"), prec)
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
        assert_psi_close(got, ref, FP32_PSI_TOL, i)
        bad = obs_close(energies[i], rec["final"], FP32_E_TOL)
        assert not bad, (i, bad)
    # every instance: final observables and psi at 64 sampled points against the oracle
    ga = golden("ensemble_all_1000.json")
    assert len(ga["instances"]) == len(ens)
    worst = 0.0
    for rec in ga["instances"]:
        i = rec["index"]
        got, ref = sampled(b.get_psi(i), rec)
        l2, mx = assert_psi_close(got, ref, FP32_PSI_TOL, i)
        worst = max(worst, l2, mx)
        bad = obs_close(energies[i], rec["final"], FP32_E_TOL)
        assert not bad, (i, bad)
    print(f"ensemble: all {len(ens)} instances within the FP32 bars (worst psi error {worst:.2e})")
    for i in range(len(ens)):
        assert abs(energies[i]["norm"] - 1.0) <= 1e-6, i
        e = np.array([h["energy"] for h in b.history(i, g["steps"])])
        assert np.all(np.diff(e) <= FP32_E_TOL * abs(e[-1])), i
    b.close()
