"""Plain FP64 CPU oracle for one split-step semi-implicit Crank-Nicolson step of
the dipolar Gross-Pitaevskii equation (2D XY, 2D XZ and 3D; imaginary and real time).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The GPU product path never imports it,
and it imports nothing from the GPU path: the two share no code, tables or constants.

What the paper fixes (Lončar et al., "CUDA programs for solving the time-dependent
dipolar Gross-Pitaevskii equation in an anisotropic trap", CPC, arXiv:1601.04640):
  * the problem: the time-dependent GP equation with contact and dipolar interactions
    in 2D or 3D in an anisotropic harmonic trap [program summary, "Nature of problem"];
  * the method: split-step Crank-Nicolson, propagation in imaginary or real time over
    small steps; the dipolar term is evaluated in momentum space by the convolution
    theorem [program summary, "Solution method"];
  * the step's structure: dipolar potential (calcpsidd2), nonlinear/potential sub-step
    (calcnu), Crank-Nicolson sweeps along x, y, z (calclux/y/z), normalisation
    (calcnorm), chemical potential/energy (calcmuen) and rms sizes (calcrms)
    ["Summary of revisions"];
  * real-to-complex / complex-to-real transforms of the (real) density ["Summary of
    revisions"].
The paper prints no equations.  Every formula below is a reading, listed with its
justification in the design notes; the readings are:
  * 3D: i dpsi/dt = [-1/2 lap + V + g|psi|^2 + g_dd Phi] psi,  V = (gamma^2 x^2 + nu^2 y^2 + lambda^2 z^2)/2,
    Phi = F^-1[U(k) F[|psi|^2]],  U(k) = (3 kz^2/k^2 - 1) b(kR)  (dipoles along z, spherical
    real-space cutoff R, prefactor 1);
  * quasi-2D: the frozen direction is a Gaussian of width d = 1/sqrt(omega_perp); contact
    coupling g/(sqrt(2 pi) d); U_XY, U_XZ are the transverse averages of the 3D kernel;
  * grid x_i = (i - N/2) dx, Dirichlet zero at i = 0 and i = N-1 on every axis, periodic FFT;
  * Lie splitting: density -> Phi -> phase with the pre-step density -> CN x -> CN y -> CN z
    -> (imaginary time) renormalise;
  * observables with forward-difference kinetic energy and plain-sum quadrature.

Parity pins (tests): brute-force DFT / direct real-space convolution, Gaussian closed
form of the dipolar energy, spherical-Bessel integral of the cutoff factor, transverse
quadrature of the quasi-2D kernels, dense solve of the CN systems, non-interacting
ground state vs. tridiagonal eigenvalues and (gamma+nu+lambda)/2, norm conservation in
real time, Kohn's theorem, the chemical potential as the imaginary-time decay rate,
monotone energy decrease in imaginary time.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg
import scipy.special

GEOMS = ("3d", "2dxy", "2dxz")


@dataclasses.dataclass
class Params:
    """Problem parameters (the quantities the paper's programs read: grid sizes and
    spacings, time step, trap frequencies, contact and dipolar couplings; cutoff R).

    geom: "3d", "2dxy" (x-y plane, z frozen with omega_perp = lam) or
          "2dxz" (x-z plane, y frozen with omega_perp = nu).
    R <= 0 means no real-space cutoff (3D only; 2D kernels have none).
    """
    geom: str
    nx: int
    ny: int = 1
    nz: int = 1
    dx: float = 0.1
    dy: float = 0.1
    dz: float = 0.1
    dt: float = 1e-3
    gamma: float = 1.0
    nu: float = 1.0
    lam: float = 1.0
    g: float = 0.0
    gdd: float = 0.0
    R: float = 0.0

    def shape(self):
        """Array shape, slowest axis first, x fastest."""
        if self.geom == "3d":
            return (self.nz, self.ny, self.nx)
        if self.geom == "2dxy":
            return (self.ny, self.nx)
        if self.geom == "2dxz":
            return (self.nz, self.nx)
        raise ValueError(self.geom)

    def spacings(self):
        """Spacings in array-axis order (slowest first)."""
        if self.geom == "3d":
            return (self.dz, self.dy, self.dx)
        if self.geom == "2dxy":
            return (self.dy, self.dx)
        return (self.dz, self.dx)

    def dV(self):
        return float(np.prod(self.spacings()))

    def d_perp(self):
        """Width of the frozen transverse Gaussian in 2D: d = 1/sqrt(omega_perp)."""
        if self.geom == "2dxy":
            return 1.0 / math.sqrt(self.lam)
        if self.geom == "2dxz":
            return 1.0 / math.sqrt(self.nu)
        raise ValueError("d_perp is defined in 2D only")


# ----------------------------------------------------------------------------- grid
def coords(n, h):
    """Grid coordinates x_i = (i - n/2) h, i = 0..n-1 (n even: the origin is a point)."""
    return (np.arange(n, dtype=np.float64) - n // 2) * h


def mesh(p: Params):
    """Coordinate arrays broadcast to the grid shape, in axis order (slowest first)."""
    axes = [coords(n, h) for n, h in zip(p.shape(), p.spacings())]
    return np.meshgrid(*axes, indexing="ij")


def harmonic_potential(p: Params):
    """Anisotropic harmonic trap V = (gamma^2 x^2 + nu^2 y^2 + lambda^2 z^2)/2
    [program summary, "Nature of problem": harmonic anisotropic trap]."""
    if p.geom == "3d":
        z, y, x = mesh(p)
        return 0.5 * (p.gamma**2 * x**2 + p.nu**2 * y**2 + p.lam**2 * z**2)
    if p.geom == "2dxy":
        y, x = mesh(p)
        return 0.5 * (p.gamma**2 * x**2 + p.nu**2 * y**2)
    z, x = mesh(p)
    return 0.5 * (p.gamma**2 * x**2 + p.lam**2 * z**2)


def wavenumbers(n, h):
    """Angular wavenumbers of an unnormalised length-n DFT on spacing h:
    k_m = 2 pi m/(n h) for m < n/2, 2 pi (m - n)/(n h) otherwise."""
    m = np.arange(n, dtype=np.float64)
    m = np.where(m < n / 2, m, m - n)
    return 2.0 * np.pi * m / (n * h)


def half_wavenumbers(n, h):
    """Wavenumbers of the non-redundant half of a real-to-complex transform (0..n/2)."""
    return 2.0 * np.pi * np.arange(n // 2 + 1, dtype=np.float64) / (n * h)


# ----------------------------------------------------------------- dipolar kernel
def cutoff_factor(s):
    """b(s) = 1 + 3 cos(s)/s^2 - 3 sin(s)/s^3: momentum-space factor of a dipolar
    interaction truncated to a sphere of radius R (s = kR).  b -> 1 for s -> inf and
    b(s) = s^2/10 - s^4/280 + ... for small s, so b(0) = 0.  The closed form cancels
    catastrophically for small s; there the alternating series
    b(s) = sum_{k>=2} (-1)^k 6k s^(2k-2)/(2k+1)! is summed instead."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    small = s < 1.0
    ss = s[small]
    acc = np.zeros_like(ss)
    for k in range(2, 16):
        acc += (-1) ** k * 6.0 * k * ss ** (2 * k - 2) / math.factorial(2 * k + 1)
    out[small] = acc
    sl = s[~small]
    out[~small] = 1.0 + 3.0 * np.cos(sl) / sl**2 - 3.0 * np.sin(sl) / sl**3
    return out


def dipolar_kernel(p: Params):
    """U(k) on the real-to-complex half grid (last axis kx = 0..nx/2), FP64.

    3D (dipoles along z): U = (3 kz^2/k^2 - 1) b(kR), U(0) = 0.
    2D XY (dipoles perpendicular to the plane):
        U = [2 - 3 sqrt(pi) xi erfcx(xi)] / (sqrt(2 pi) d),  xi = q d/sqrt(2), q = |(kx, ky)|.
    2D XZ (dipoles along z, in the plane):
        U = [-1 + 3 sqrt(pi) (kz^2/q^2) xi erfcx(xi)] / (sqrt(2 pi) d),  q = |(kx, kz)|,
        U(0) = -1/(sqrt(2 pi) d).
    Solution method: the dipolar term is evaluated in momentum space by the
    convolution theorem [program summary, "Solution method"]."""
    if p.geom == "3d":
        kz = wavenumbers(p.nz, p.dz)[:, None, None]
        ky = wavenumbers(p.ny, p.dy)[None, :, None]
        kx = half_wavenumbers(p.nx, p.dx)[None, None, :]
        k2 = kx**2 + ky**2 + kz**2
        with np.errstate(invalid="ignore", divide="ignore"):
            ang = 3.0 * kz**2 / k2 - 1.0
        ang = np.broadcast_to(ang, k2.shape).copy()
        ang[0, 0, 0] = 0.0
        if p.R > 0:
            u = ang * cutoff_factor(np.sqrt(k2) * p.R)
        else:
            u = ang
        u[0, 0, 0] = 0.0
        return u
    d = p.d_perp()
    pref = 1.0 / (math.sqrt(2.0 * math.pi) * d)
    if p.geom == "2dxy":
        ky = wavenumbers(p.ny, p.dy)[:, None]
        kx = half_wavenumbers(p.nx, p.dx)[None, :]
        q = np.sqrt(kx**2 + ky**2)
        xi = q * d / math.sqrt(2.0)
        return pref * (2.0 - 3.0 * math.sqrt(math.pi) * xi * scipy.special.erfcx(xi))
    kz = wavenumbers(p.nz, p.dz)[:, None]
    kx = half_wavenumbers(p.nx, p.dx)[None, :]
    q2 = kx**2 + kz**2
    q = np.sqrt(q2)
    xi = q * d / math.sqrt(2.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(q2 > 0, kz**2 / np.where(q2 > 0, q2, 1.0), 0.0)
    return pref * (-1.0 + 3.0 * math.sqrt(math.pi) * ratio * xi * scipy.special.erfcx(xi))


def contact_coupling(p: Params):
    """Contact coefficient multiplying |psi|^2: g in 3D, g/(sqrt(2 pi) d) in quasi-2D
    (transverse integral of a normalised Gaussian squared)."""
    if p.geom == "3d":
        return p.g
    return p.g / (math.sqrt(2.0 * math.pi) * p.d_perp())


def dipolar_potential(n, p: Params, kernel=None):
    """Phi = F^-1[U(k) F[n]] for a real field n (unnormalised forward DFT, inverse with
    1/N).  Real-to-complex and complex-to-real transforms, as the paper does for the
    real density ["Summary of revisions", calcpsidd2].  Does not include g_dd."""
    if kernel is None:
        kernel = dipolar_kernel(p)
    spec = np.fft.rfftn(n)
    return np.fft.irfftn(spec * kernel, s=n.shape, axes=tuple(range(n.ndim)))


# ------------------------------------------------------------- Crank-Nicolson sweep
def cn_sweep(psi, axis, A):
    """One Crank-Nicolson sweep along `axis` (calclux/calcluy/calcluz):
    for every line, solve  -A u_{i-1} + (1+2A) u_i - A u_{i+1}
                         =  A psi_{i-1} + (1-2A) psi_i + A psi_{i+1}
    for the interior points i = 1..N-2 with u_0 = u_{N-1} = 0 (Dirichlet).
    A = eps dt/(4 h^2) with eps = 1 (imaginary time) or i (real time).  The banded
    system is solved by LAPACK (library primitive), all lines at once."""
    psi = np.asarray(psi, dtype=np.complex128)
    a = np.moveaxis(psi, axis, 0)
    n = a.shape[0]
    rest = a.shape[1:]
    a2 = a.reshape(n, -1)
    rhs = A * a2[:-2] + (1.0 - 2.0 * A) * a2[1:-1] + A * a2[2:]
    m = n - 2
    ab = np.empty((3, m), dtype=np.complex128)
    ab[0, :] = -A
    ab[1, :] = 1.0 + 2.0 * A
    ab[2, :] = -A
    sol = scipy.linalg.solve_banded((1, 1), ab, rhs)
    out = np.zeros_like(a2)
    out[1:-1] = sol
    out = out.reshape((n,) + rest)
    return np.moveaxis(out, 0, axis)


# ---------------------------------------------------------------------- one step
def step(psi, p: Params, imag: bool, V=None, kernel=None, renormalize=True):
    """One split-step semi-implicit Crank-Nicolson step (program summary, "Solution
    method"; sub-step order calcpsidd2 -> calcnu -> calclux -> calcluy -> calcluz ->
    calcnorm, "Summary of revisions").

      S1  n     = |psi|^2
      S2  Phi   = F^-1[U F[n]]
      S3  theta = V + g_c n + g_dd Phi          (pre-step density)
      S4  psi  <- psi exp(-eps dt theta)         eps = 1 (imag) or i (real)
      S5  CN sweep along x, A = eps dt/(4 dx^2)
      S6  CN sweep along y (or z in 2D XZ)
      S7  CN sweep along z (3D)
      S8  imaginary time only: psi <- psi / sqrt(sum |psi|^2 dV)
    """
    if V is None:
        V = harmonic_potential(p)
    eps = 1.0 if imag else 1j
    psi = np.asarray(psi, dtype=np.complex128)
    n = np.abs(psi) ** 2                                          # S1
    phi = dipolar_potential(n, p, kernel)                         # S2
    theta = V + contact_coupling(p) * n + p.gdd * phi             # S3
    psi = psi * np.exp(-eps * p.dt * theta)                       # S4
    nd = psi.ndim
    for ax_from_end, h in zip(range(1, nd + 1), reversed(p.spacings())):   # S5..S7
        psi = cn_sweep(psi, nd - ax_from_end, eps * p.dt / (4.0 * h * h))
    if imag and renormalize:                                      # S8
        psi = psi / math.sqrt(float(np.sum(np.abs(psi) ** 2)) * p.dV())
    return psi


def run(psi, p: Params, imag: bool, nsteps: int, V=None, record=False):
    """nsteps steps; with record=True also returns the observables of the state at the
    start of every step (what calcmuen/calcnorm/calcrms report)."""
    if V is None:
        V = harmonic_potential(p)
    kernel = dipolar_kernel(p)
    hist = []
    for _ in range(nsteps):
        if record:
            hist.append(observables(psi, p, V=V, kernel=kernel))
        psi = step(psi, p, imag, V=V, kernel=kernel)
    return (psi, hist) if record else psi


# ------------------------------------------------------------------ observables
def observables(psi, p: Params, V=None, kernel=None):
    """Norm, energy and its parts, chemical potential and rms sizes of psi
    (calcnorm, calcmuen, calcrms), all accumulated in FP64:

      norm  = sum |psi|^2 dV
      E_kin = 1/2 sum_axes sum_{i=0}^{N-2} |psi_{i+1} - psi_i|^2 / h^2 dV
      E_pot = sum V |psi|^2 dV
      E_int = g_c/2 sum |psi|^4 dV
      E_dd  = g_dd/2 sum Phi |psi|^2 dV,  Phi from this psi
      E     = E_kin + E_pot + E_int + E_dd;  mu = E_kin + E_pot + 2 E_int + 2 E_dd
      rms_a = sqrt(sum a^2 |psi|^2 dV / norm), about the grid origin.
    rms is returned as (x, y, z); the frozen axis in 2D reports 0."""
    if V is None:
        V = harmonic_potential(p)
    psi = np.asarray(psi, dtype=np.complex128)
    dV = p.dV()
    n = np.abs(psi) ** 2
    phi = dipolar_potential(n, p, kernel)
    norm = float(np.sum(n)) * dV
    ekin = 0.0
    for ax, h in enumerate(p.spacings()):
        dif = np.diff(psi, axis=ax)
        ekin += 0.5 * float(np.sum(np.abs(dif) ** 2)) / (h * h) * dV
    epot = float(np.sum(V * n)) * dV
    eint = 0.5 * contact_coupling(p) * float(np.sum(n * n)) * dV
    edd = 0.5 * p.gdd * float(np.sum(phi * n)) * dV
    m = mesh(p)
    names = {"3d": ("z", "y", "x"), "2dxy": ("y", "x"), "2dxz": ("z", "x")}[p.geom]
    rms = {"x": 0.0, "y": 0.0, "z": 0.0}
    for nm, c in zip(names, m):
        rms[nm] = math.sqrt(float(np.sum(c * c * n)) * dV / norm)
    return {
        "norm": norm,
        "energy": ekin + epot + eint + edd,
        "mu": ekin + epot + 2.0 * eint + 2.0 * edd,
        "e_kin": ekin,
        "e_pot": epot,
        "e_int": eint,
        "e_dd": edd,
        "rms": (rms["x"], rms["y"], rms["z"]),
    }


def zero_boundary(psi):
    """Dirichlet: zero the first and last point along every axis."""
    psi = np.array(psi, dtype=np.complex128, copy=True)
    for ax in range(psi.ndim):
        idx = [slice(None)] * psi.ndim
        idx[ax] = 0
        psi[tuple(idx)] = 0
        idx[ax] = -1
        psi[tuple(idx)] = 0
    return psi
