"""FP64 adjoint of the real-time split-step Crank-Nicolson step (oracle, test
infrastructure only; never imported by the GPU product path).

Gradients of a scalar loss of the final state with respect to the trap potential V on
the grid and the couplings g, g_dd.  The forward step is `gp_oracle.step(..., imag=False)`:

    psi_a   = exp(-i dt theta(psi_n)) psi_n,   theta = V + g_c n + g_dd K n,  n = |psi_n|^2
    psi_n+1 = C_z C_y C_x psi_a,               C = (1 + i dt T/2)^-1 (1 - i dt T/2) per axis

Conventions: <a, b> = sum conj(a) b (no volume element); the costate is
lambda = dL/d conj(psi) (Wirtinger), so that dL = 2 Re <lambda, d psi>.

Backward through one step (derived from the forward definitions):
  * C is complex symmetric and unitary, so its adjoint C^H = conj(C) is the same sweep
    with dt -> -dt; the factors act on different axes and are applied z, y, x.
  * mu = exp(+i dt theta) lambda_a;  s = 2 dt Im(conj(mu) psi_n)  (a real field);
    dL/dV += s, dL/dg_c += sum s n, dL/dg_dd += sum s Phi;
    lambda_n = mu + (g_c s + g_dd K s) psi_n, where K s = F^-1[U F[s]] (K symmetric:
    U is real and even).
  * in 2D the contact coupling is g_c = g/(sqrt(2 pi) d), so dL/dg = dL/dg_c/(sqrt(2 pi) d).
Terminal costates:
  * overlap loss L = 1 - |c|^2, c = sum conj(psi_t) psi(T) dV:  lambda_T = -c psi_t dV;
  * energy loss L = E(psi(T)) (observables): lambda_T = (T_disc + V + g_c n + g_dd Phi) psi dV.
"""
from __future__ import annotations

import math

import numpy as np

from . import gp_oracle as G


def overlap_loss(psi, psi_t, p: G.Params):
    c = complex(np.sum(np.conj(psi_t) * psi)) * p.dV()
    return 1.0 - abs(c) ** 2, c


def overlap_costate(psi, psi_t, p: G.Params):
    _, c = overlap_loss(psi, psi_t, p)
    return -c * psi_t * p.dV()


def forward_states(psi0, p: G.Params, nsteps, V=None, kernel=None):
    """All states psi_0..psi_nsteps of a real-time run."""
    if V is None:
        V = G.harmonic_potential(p)
    if kernel is None:
        kernel = G.dipolar_kernel(p)
    out = [np.asarray(psi0, dtype=np.complex128)]
    for _ in range(nsteps):
        out.append(G.step(out[-1], p, False, V=V, kernel=kernel))
    return out


def adjoint_step(psi_n, lam, p: G.Params, V, kernel):
    """Costate at the start of a real-time step from the costate at its end.
    Returns (lambda_n, s, sum s n, sum s Phi) with s the dL/dV contribution."""
    dt = p.dt
    lam = np.asarray(lam, dtype=np.complex128)
    nd = lam.ndim
    # adjoint CN sweeps: reverse axis order (z, y, x) with dt -> -dt
    for ax_from_end, h in zip(range(nd, 0, -1), p.spacings()):
        lam = G.cn_sweep(lam, nd - ax_from_end, -1j * dt / (4.0 * h * h))
    n = np.abs(psi_n) ** 2
    phi = G.dipolar_potential(n, p, kernel)
    gc = G.contact_coupling(p)
    theta = V + gc * n + p.gdd * phi
    mu = np.exp(1j * dt * theta) * lam
    s = 2.0 * dt * np.imag(np.conj(mu) * psi_n)
    ks = G.dipolar_potential(s, p, kernel)
    lam_n = mu + (gc * s + p.gdd * ks) * psi_n
    return lam_n, s, float(np.sum(s * n)), float(np.sum(s * phi))


def contact_factor(p: G.Params):
    """d g_c / d g: 1 in 3D, 1/(sqrt(2 pi) d) in quasi-2D."""
    return 1.0 if p.geom == "3d" else 1.0 / (math.sqrt(2.0 * math.pi) * p.d_perp())


def overlap_gradients(psi0, psi_t, p: G.Params, nsteps, V=None):
    """L = 1 - |<psi_t|psi(T)>|^2 after nsteps real-time steps and its gradients with
    respect to V (grid), g and g_dd, plus the costate of the initial state."""
    if V is None:
        V = G.harmonic_potential(p)
    kernel = G.dipolar_kernel(p)
    states = forward_states(psi0, p, nsteps, V, kernel)
    L, _ = overlap_loss(states[-1], psi_t, p)
    lam = overlap_costate(states[-1], psi_t, p)
    gV = np.zeros(V.shape)
    gg = 0.0
    ggdd = 0.0
    for k in range(nsteps - 1, -1, -1):
        lam, s, sn, sphi = adjoint_step(states[k], lam, p, V, kernel)
        gV += s
        gg += sn
        ggdd += sphi
    return {"loss": L, "dV": gV, "dg": gg * contact_factor(p), "dgdd": ggdd, "lambda0": lam,
            "final": states[-1]}


def energy_costate(psi, p: G.Params, V=None, kernel=None):
    """dE/d conj(psi) of the observables' energy functional (for an energy loss)."""
    if V is None:
        V = G.harmonic_potential(p)
    n = np.abs(psi) ** 2
    phi = G.dipolar_potential(n, p, kernel)
    tpsi = np.zeros_like(psi)
    for ax, h in enumerate(p.spacings()):
        # d/d conj(psi_k) of 1/2 sum_i |D_i|^2/h^2 with D_i = psi_{i+1} - psi_i is
        # 1/2 (D_{k-1} - D_k)/h^2 (D_{-1} = D_{N-1} = 0): minus the second difference
        d = np.diff(psi, axis=ax)
        pad_lo = [(0, 0)] * psi.ndim
        pad_lo[ax] = (1, 0)
        pad_hi = [(0, 0)] * psi.ndim
        pad_hi[ax] = (0, 1)
        tpsi += 0.5 * (np.pad(d, pad_lo) - np.pad(d, pad_hi)) / (h * h)
    return (tpsi + V * psi + G.contact_coupling(p) * n * psi + p.gdd * phi * psi) * p.dV()


def energy_gradients(psi0, p: G.Params, nsteps, V=None):
    """L = E(psi(T)) (the observables' energy of the state after nsteps real-time steps)
    and its gradients with respect to V (grid), g and g_dd, plus the costate of the
    initial state.  E depends on V, g and g_dd directly as well as through psi(T): the
    direct terms are dE/dV = n dV, dE/dg_c = 1/2 sum n^2 dV, dE/dg_dd = 1/2 sum Phi n dV,
    with n and Phi of psi(T); the rest comes back through the adjoint steps from the
    terminal costate (energy_costate)."""
    if V is None:
        V = G.harmonic_potential(p)
    kernel = G.dipolar_kernel(p)
    states = forward_states(psi0, p, nsteps, V, kernel)
    psiT = states[-1]
    L = G.observables(psiT, p, V=V, kernel=kernel)["energy"]
    n = np.abs(psiT) ** 2
    phi = G.dipolar_potential(n, p, kernel)
    dV = p.dV()
    gV = n * dV
    gg = 0.5 * float(np.sum(n * n)) * dV
    ggdd = 0.5 * float(np.sum(phi * n)) * dV
    # psi(T) is zero on the boundary rows whatever the inputs (Dirichlet), so its
    # perturbations are too, and the costate's boundary rows carry nothing; the adjoint
    # steps take them as zero (the adjoint of a sweep whose boundary outputs are fixed)
    lam = G.zero_boundary(energy_costate(psiT, p, V=V, kernel=kernel))
    for k in range(nsteps - 1, -1, -1):
        lam, s, sn, sphi = adjoint_step(states[k], lam, p, V, kernel)
        gV = gV + s
        gg += sn
        ggdd += sphi
    return {"loss": L, "dV": gV, "dg": gg * contact_factor(p), "dgdd": ggdd, "lambda0": lam,
            "final": psiT}
