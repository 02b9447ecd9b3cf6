"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds no arithmetic of the method: it only draws random numbers and
builds initial wave functions and potential perturbations (Gaussians with noise),
all in FP64 on the host with numpy's PCG64 generator.  The same arrays are handed to
both sides.  Workload parameters mirror the harmonic-trap condensates of the
paper's programs (imag/real, 2D/3D) at the grid sizes listed in the design notes.
"""
from __future__ import annotations

import math

import numpy as np


def _axis(n, h):
    return (np.arange(n, dtype=np.float64) - n // 2) * h


def grid_axes(geom, nx, ny, nz, dx, dy, dz):
    """Coordinate vectors in array-axis order (slowest first)."""
    if geom == "3d":
        return [_axis(nz, dz), _axis(ny, dy), _axis(nx, dx)]
    if geom == "2dxy":
        return [_axis(ny, dy), _axis(nx, dx)]
    return [_axis(nz, dz), _axis(nx, dx)]


def _dirichlet_normalise(psi, cell):
    psi = np.array(psi, dtype=np.complex128, copy=True)
    for ax in range(psi.ndim):
        idx = [slice(None)] * psi.ndim
        idx[ax] = 0
        psi[tuple(idx)] = 0
        idx[ax] = -1
        psi[tuple(idx)] = 0
    nrm = math.sqrt(float(np.sum(np.abs(psi) ** 2)) * cell)
    return psi / nrm


def gaussian(geom, nx, ny, nz, dx, dy, dz, widths, center=None, amp_noise=0.0,
             phase_noise=0.0, seed=None):
    """Normalised Gaussian exp(-sum (a-c_a)^2/(2 w_a^2)) times (1 + amp_noise*u) and
    exp(i 2 pi phase_noise u'), u, u' ~ U[-1, 1) i.i.d. per point (PCG64, `seed`).
    `widths` and `center` are given in array-axis order (slowest first).  Boundary
    points are zeroed and sum |psi|^2 dV = 1."""
    axes = grid_axes(geom, nx, ny, nz, dx, dy, dz)
    if center is None:
        center = [0.0] * len(axes)
    mesh = np.meshgrid(*axes, indexing="ij")
    arg = np.zeros(mesh[0].shape)
    for c, w, c0 in zip(mesh, widths, center):
        arg += (c - c0) ** 2 / (2.0 * w * w)
    psi = np.exp(-arg).astype(np.complex128)
    rng = np.random.default_rng(seed)
    if amp_noise:
        psi *= 1.0 + amp_noise * rng.uniform(-1.0, 1.0, size=psi.shape)
    if phase_noise:
        psi *= np.exp(1j * 2.0 * math.pi * phase_noise * rng.uniform(-1.0, 1.0, size=psi.shape))
    cell = float(np.prod([a[1] - a[0] for a in axes]))
    return _dirichlet_normalise(psi, cell)


def random_complex(shape, seed, cell):
    """Smooth-free random complex field (parity of individual operations)."""
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return _dirichlet_normalise(psi, cell)


def smooth_random_field(shape, spacings, corr_len, seed):
    """White N(0,1) noise filtered by a periodic Gaussian exp(-r^2/(2 l^2)) and scaled
    to unit RMS (a smooth random trap perturbation)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    ks = [2 * np.pi * np.fft.fftfreq(n, d=h) for n, h in zip(shape, spacings)]
    km = np.meshgrid(*ks, indexing="ij")
    k2 = sum(k * k for k in km)
    f = np.real(np.fft.ifftn(np.fft.fftn(w) * np.exp(-0.5 * k2 * corr_len**2)))
    return f / math.sqrt(float(np.mean(f * f)))


# --------------------------------------------------------------------- workloads
# Each workload: physical parameters (dict) + how to make psi0.  Names describe the
# workload; sizes follow the paper's harmonic-trap examples scaled to MI355X memory.
WORKLOADS = {
    "imag3d_64": dict(geom="3d", nx=64, ny=64, nz=64, dx=0.25, dy=0.25, dz=0.25,
                      dt=0.002, gamma=1.0, nu=1.0, lam=2.0, g=20.0, gdd=6.0, R=8.0,
                      imag=True, steps=500),
    "real3d_128x96x80": dict(geom="3d", nx=128, ny=96, nz=80, dx=0.2, dy=0.2, dz=0.2,
                             dt=0.001, gamma=1.0, nu=1.0, lam=2.0, g=15.0, gdd=6.0,
                             R=8.0, imag=False, steps=2000, g_ground=20.0),
    "real2dxy_256": dict(geom="2dxy", nx=256, ny=256, nz=1, dx=0.1, dy=0.1, dz=0.1,
                         dt=0.0005, gamma=1.0, nu=1.5, lam=4.0, g=30.0, gdd=10.0,
                         R=0.0, imag=False, steps=4000),
    "real3d_256": dict(geom="3d", nx=256, ny=256, nz=256, dx=0.1, dy=0.1, dz=0.1,
                       dt=0.0005, gamma=1.0, nu=1.0, lam=3.0, g=50.0, gdd=25.0,
                       R=12.8, imag=False, steps=500),
    # the large workload's adjoint companion: 128^3 at twice the spacing (same box),
    # 200 real-time steps, recompute every 20
    "adjoint3d_128": dict(geom="3d", nx=128, ny=128, nz=128, dx=0.2, dy=0.2, dz=0.2,
                          dt=0.0005, gamma=1.0, nu=1.0, lam=3.0, g=50.0, gdd=25.0,
                          R=12.8, imag=False, steps=200, K=20),
}


def psi0_imag3d_64(seed=1601):
    """Anisotropic Gaussian, widths (x, y, z) = (1, 1, 0.7), times (1 + 0.01 u)."""
    w = WORKLOADS["imag3d_64"]
    return gaussian("3d", w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                    widths=(0.7, 1.0, 1.0), amp_noise=0.01, seed=seed)


def psi0_real3d_128x96x80(seed=1602):
    """Start of the imaginary-time relaxation that precedes the quench."""
    w = WORKLOADS["real3d_128x96x80"]
    return gaussian("3d", w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                    widths=(0.7, 1.0, 1.0), amp_noise=0.01, seed=seed)


def psi0_real3d_256(seed=1607):
    """exp(-(x^2 + y^2 + 3 z^2)/2) with 0.5 % phase noise."""
    w = WORKLOADS["real3d_256"]
    return gaussian("3d", w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                    widths=(1.0 / math.sqrt(3.0), 1.0, 1.0), phase_noise=0.005, seed=seed)


def psi0_real2dxy_256():
    """Ground state of the unperturbed in-plane harmonic trap ~ exp(-(x^2 + 1.5 y^2)/2)."""
    w = WORKLOADS["real2dxy_256"]
    return gaussian("2dxy", w["nx"], w["ny"], 1, w["dx"], w["dy"], w["dz"],
                    widths=(1.0 / math.sqrt(1.5), 1.0))


def trap_perturbation_real2dxy_256(seed=1608):
    """Smooth random perturbation of the 256^2 trap: amplitude 0.1 (RMS), correlation
    length 1.0 (added to the harmonic trap by the caller)."""
    w = WORKLOADS["real2dxy_256"]
    return 0.1 * smooth_random_field((w["ny"], w["nx"]), (w["dy"], w["dx"]), 1.0, seed)


def displaced_target(w, seed, widths):
    """Normalised Gaussian target whose centre is drawn from U[-0.5, 0.5) per axis."""
    rng = np.random.default_rng(seed)
    ndim = 3 if w["geom"] == "3d" else 2
    center = list(rng.uniform(-0.5, 0.5, size=ndim))
    return gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                    widths=widths, center=center)


def psi0_adjoint3d_128(seed=1609):
    """exp(-(x^2 + y^2 + 3 z^2)/2) with 0.5 % phase noise on the 128^3 grid."""
    w = WORKLOADS["adjoint3d_128"]
    return gaussian("3d", w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                    widths=(1.0 / math.sqrt(3.0), 1.0, 1.0), phase_noise=0.005, seed=seed)


def batched_ensemble(count=192, seed=1606, sizes=(96, 128, 192, 256, 384, 512)):
    """Parameters of an ensemble of independent quasi-2D instances (even index XY,
    odd index XZ), drawn with PCG64 from `seed`."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n0 = int(rng.choice(sizes))
        n1 = int(rng.choice(sizes))
        a = float(rng.uniform(0.5, 4.0))
        h = float(rng.uniform(0.05, 0.2))
        g = float(rng.uniform(0.0, 50.0))
        gdd = float(rng.uniform(0.0, 30.0))
        if i % 2 == 0:
            out.append(dict(geom="2dxy", nx=n0, ny=n1, nz=1, dx=h, dy=h, dz=h, dt=0.001,
                            gamma=1.0, nu=a, lam=4.0, g=g, gdd=gdd, R=0.0))
        else:
            out.append(dict(geom="2dxz", nx=n0, ny=1, nz=n1, dx=h, dy=h, dz=h, dt=0.001,
                            gamma=1.0, nu=4.0, lam=a, g=g, gdd=gdd, R=0.0))
    return out


def psi0_instance(w, seed):
    """In-plane harmonic ground-state Gaussian times (1 + 0.01 u)."""
    if w["geom"] == "2dxy":
        widths = (1.0 / math.sqrt(w["nu"]), 1.0 / math.sqrt(w["gamma"]))
    else:
        widths = (1.0 / math.sqrt(w["lam"]), 1.0 / math.sqrt(w["gamma"]))
    return gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                    widths=widths, amp_noise=0.01, seed=seed)
