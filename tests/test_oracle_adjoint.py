"""Pins of the FP64 adjoint oracle: every gradient against central finite differences of
the (separately pinned) forward oracle, and the adjoint identity of the CN sweep."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import gp_adjoint as A
from paper_1601_04640_amd import inputs as I

CASES = {
    "2dxy": dict(geom="2dxy", nx=24, ny=20, dx=0.35, dy=0.4, dt=0.004, gamma=1.0, nu=1.4,
                 lam=4.0, g=30.0, gdd=10.0),
    "2dxz": dict(geom="2dxz", nx=20, nz=24, dx=0.4, dz=0.3, dt=0.004, gamma=1.0, nu=4.0,
                 lam=2.0, g=20.0, gdd=15.0),
    "3d": dict(geom="3d", nx=12, ny=10, nz=14, dx=0.6, dy=0.7, dz=0.5, dt=0.004, gamma=1.0,
               nu=1.2, lam=1.8, g=25.0, gdd=9.0, R=2.5),
}
NSTEPS = 4


def setup(name):
    w = CASES[name]
    p = O.Params(**w)
    shape = p.shape()
    ax = I.grid_axes(w["geom"], w["nx"], w.get("ny", 1), w.get("nz", 1), w["dx"],
                     w.get("dy", 0.1), w.get("dz", 0.1))
    widths = [0.9, 1.1, 1.0][:len(shape)]
    psi0 = I.gaussian(w["geom"], w["nx"], w.get("ny", 1), w.get("nz", 1), w["dx"],
                      w.get("dy", 0.1), w.get("dz", 0.1), widths=widths, phase_noise=0.02,
                      amp_noise=0.02, seed=3)
    center = [0.3 * (a[1] - a[0]) * 2 for a in ax]
    psi_t = I.gaussian(w["geom"], w["nx"], w.get("ny", 1), w.get("nz", 1), w["dx"],
                       w.get("dy", 0.1), w.get("dz", 0.1), widths=widths, center=center)
    V = O.harmonic_potential(p) + 0.1 * I.smooth_random_field(shape, p.spacings(), 1.0, 5)
    return p, psi0, psi_t, V


def loss(p, psi0, psi_t, V):
    psi = O.run(psi0, p, False, NSTEPS, V=V)
    return A.overlap_loss(psi, psi_t, p)[0]


@pytest.fixture(scope="module", params=list(CASES))
def grads(request):
    p, psi0, psi_t, V = setup(request.param)
    return request.param, p, psi0, psi_t, V, A.overlap_gradients(psi0, psi_t, p, NSTEPS, V=V)


def central(f, h):
    return (f(h) - f(-h)) / (2 * h)


def test_couplings_match_finite_differences(grads):
    name, p, psi0, psi_t, V, g = grads
    for key, attr in (("dg", "g"), ("dgdd", "gdd")):
        base = getattr(p, attr)
        h = 1e-5 * base
        fd = central(lambda e: loss(O.Params(**{**p.__dict__, attr: base + e}), psi0, psi_t, V), h)
        assert abs(g[key] - fd) <= 1e-6 * abs(fd) + 1e-12, (name, key, g[key], fd)


def test_grid_potential_matches_finite_differences(grads):
    name, p, psi0, psi_t, V, g = grads
    rng = np.random.default_rng(11)
    flat = V.ravel()
    # grid values where the condensate is: the gradient there is well above FD noise
    big = np.flatnonzero(np.abs(g["dV"].ravel()) > 1e-2 * np.abs(g["dV"]).max())
    for k in rng.choice(big, size=6, replace=False):
        k = int(k)
        h = 1e-3

        def f(e):
            W = flat.copy()
            W[k] += e
            return loss(p, psi0, psi_t, W.reshape(V.shape))
        fd = central(f, h)
        assert abs(g["dV"].ravel()[k] - fd) <= 1e-6 * abs(fd), (name, k)
    d = I.smooth_random_field(V.shape, p.spacings(), 1.0, 12)
    fd = central(lambda e: loss(p, psi0, psi_t, V + e * d), 1e-5)
    assert abs(float(np.sum(g["dV"] * d)) - fd) <= 1e-6 * abs(fd), name


def test_initial_costate_matches_finite_differences(grads):
    name, p, psi0, psi_t, V, g = grads
    rng = np.random.default_rng(13)
    d = O.zero_boundary(rng.standard_normal(psi0.shape) + 1j * rng.standard_normal(psi0.shape))
    fd = central(lambda e: loss(p, psi0 + e * d, psi_t, V), 1e-6)
    an = 2.0 * float(np.real(np.sum(np.conj(g["lambda0"]) * d)))
    assert abs(an - fd) <= 1e-6 * abs(fd), (name, an, fd)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cn_adjoint_identity(axis):
    """<w, C(A) v> = <C(conj A) w, v>: the adjoint of a CN sweep is the sweep with
    dt -> -dt (C is complex symmetric)."""
    rng = np.random.default_rng(axis)
    shape = (9, 8, 11)
    v = O.zero_boundary(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    w = O.zero_boundary(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    A_ = 0.37j
    lhs = np.vdot(w, O.cn_sweep(v, axis, A_))
    rhs = np.vdot(O.cn_sweep(w, axis, np.conj(A_)), v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_energy_costate_matches_finite_differences():
    p, psi0, _, V = setup("3d")
    lamE = A.energy_costate(psi0, p, V=V)
    rng = np.random.default_rng(17)
    d = O.zero_boundary(rng.standard_normal(psi0.shape) + 1j * rng.standard_normal(psi0.shape))
    E = lambda e: O.observables(psi0 + e * d, p, V=V)["energy"]
    fd = central(E, 1e-6)
    an = 2.0 * float(np.real(np.sum(np.conj(lamE) * d)))
    assert abs(an - fd) <= 1e-6 * abs(fd), (an, fd)


@pytest.mark.parametrize("name", ["2dxz", "3d"])
def test_energy_loss_gradients_match_finite_differences(name):
    """L = E(psi(T)) through NSTEPS real-time steps: couplings, grid values of V and the
    initial costate against central differences of the forward oracle's energy."""
    p, psi0, _, V = setup(name)

    def L(pp=p, psi=psi0, W=V):
        return O.observables(O.run(psi, pp, False, NSTEPS, V=W), pp, V=W)["energy"]
    g = A.energy_gradients(psi0, p, NSTEPS, V=V)
    assert abs(g["loss"] - L()) <= 1e-13 * abs(g["loss"])
    for key, attr in (("dg", "g"), ("dgdd", "gdd")):
        base = getattr(p, attr)
        h = 1e-5 * base
        fd = central(lambda e: L(pp=O.Params(**{**p.__dict__, attr: base + e})), h)
        assert abs(g[key] - fd) <= 1e-6 * abs(fd), (name, key, g[key], fd)
    big = np.flatnonzero(np.abs(g["dV"].ravel()) > 1e-2 * np.abs(g["dV"]).max())
    rng = np.random.default_rng(19)
    for k in rng.choice(big, size=3, replace=False):
        k = int(k)

        def f(e):
            W = V.ravel().copy()
            W[k] += e
            return L(W=W.reshape(V.shape))
        fd = central(f, 1e-4)
        assert abs(g["dV"].ravel()[k] - fd) <= 1e-6 * abs(fd), (name, k)
    d = O.zero_boundary(rng.standard_normal(psi0.shape) + 1j * rng.standard_normal(psi0.shape))
    fd = central(lambda e: L(psi=psi0 + e * d), 1e-6)
    an = 2.0 * float(np.real(np.sum(np.conj(g["lambda0"]) * d)))
    assert abs(an - fd) <= 1e-6 * abs(fd), (name, an, fd)
