"""Pins of the FP64 oracle against what the mathematics and the paper's problem
statement fix, independently of the oracle's own code paths.

Each test targets a plausible mistake: a wrong FFT scaling or sign convention
(direct real-space convolution), a wrong kernel prefactor, sign or cutoff (Gaussian
closed form, Bessel integral, symmetric densities), a wrong quasi-2D reduction
(transverse quadrature), a wrong CN coefficient (dense solve, tridiagonal
eigenvalues), a wrong potential or kinetic term (harmonic ground state
(gamma+nu+lambda)/2), a wrong phase sign or non-unitary step (norm conservation,
Kohn's theorem), a wrong chemical-potential formula (imaginary-time decay rate).
"""
import math

import numpy as np
import pytest
import scipy.integrate as integrate
import scipy.linalg
import scipy.special

import oracle as O
from paper_1601_04640_amd import inputs as I


# ------------------------------------------------------------------ helpers
def dft_matrix(n, sign):
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n)


def full_kernel_from_half(Uh, n_last):
    """Extend the half-grid kernel to the full grid using its evenness in kx."""
    full = np.empty(Uh.shape[:-1] + (n_last,))
    full[..., : n_last // 2 + 1] = Uh
    for m in range(n_last // 2 + 1, n_last):
        full[..., m] = Uh[..., n_last - m]
    return full


def brute_force_convolution(n, Ufull):
    """Phi_i = sum_j K(i - j) n_j with K = brute-force inverse DFT of U (explicit
    DFT matrices, no FFT), periodic indices."""
    K = Ufull.astype(np.complex128)
    for ax, N in enumerate(Ufull.shape):
        M = dft_matrix(N, +1) / N
        K = np.moveaxis(np.tensordot(M, np.moveaxis(K, ax, 0), axes=(1, 0)), 0, ax)
    assert np.max(np.abs(K.imag)) < 1e-12 * np.max(np.abs(K.real)) + 1e-15
    K = K.real
    shape = n.shape
    idx = np.indices(shape).reshape(len(shape), -1).T
    phi = np.zeros(n.size)
    nf = n.ravel()
    for a, ia in enumerate(idx):
        diff = tuple(((ia - idx) % np.array(shape)).T)
        phi[a] = np.sum(K[diff] * nf)
    return phi.reshape(shape)


def gaussian_density(p, widths):
    m = O.mesh(p)
    arg = sum(c * c / (2.0 * w * w) for c, w in zip(m, widths))
    n = np.exp(-arg)
    return n / (np.sum(n) * p.dV())


# ------------------------------------------------------------ FFT machinery
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 10, 12, 15, 16, 20, 24, 30, 40, 48, 60,
                               64, 80, 96, 120, 128, 192, 256])
def test_rfft_matches_bruteforce_dft(n):
    """The transform the oracle relies on equals the defining DFT sum."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n)
    ref = dft_matrix(n, -1) @ x
    got = np.fft.rfft(x)
    assert np.max(np.abs(got - ref[: n // 2 + 1])) <= 1e-13 * max(1.0, math.log2(n)) * np.max(np.abs(ref))


@pytest.mark.parametrize("geom,shape", [("3d", (10, 6, 8)), ("2dxy", (6, 8)), ("2dxz", (10, 8)),
                                        ("3d", (9, 7, 5)), ("2dxy", (7, 9)), ("2dxz", (9, 5))])
def test_dipolar_potential_equals_direct_circulant_sum(geom, shape):
    """S2: Phi = F^-1[U F[n]] is the periodic real-space convolution with
    K = F^-1[U]; checked against an explicit O(N^2) sum on tiny grids, even and odd (an
    odd axis has no Nyquist index: K is real only if U pairs index m with n - m, which
    a frequency map off by one at m = (n-1)/2 breaks)."""
    if geom == "3d":
        p = O.Params(geom=geom, nx=shape[2], ny=shape[1], nz=shape[0], dx=0.3, dy=0.45,
                     dz=0.25, R=0.7)
    elif geom == "2dxy":
        p = O.Params(geom=geom, nx=shape[1], ny=shape[0], dx=0.3, dy=0.4, lam=3.0)
    else:
        p = O.Params(geom=geom, nx=shape[1], nz=shape[0], dx=0.3, dz=0.2, nu=2.0)
    rng = np.random.default_rng(7)
    n = rng.uniform(0, 1, size=p.shape())
    Uh = O.dipolar_kernel(p)
    ref = brute_force_convolution(n, full_kernel_from_half(Uh, p.nx))
    got = O.dipolar_potential(n, p)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


# --------------------------------------------------------------- 3D kernel
def gaussian_edd_closed_form(sr, sz, gdd):
    """E_dd = gdd sqrt(pi)/(32 pi^2) int_{-1}^{1} (3u^2-1)/(sr^2(1-u^2)+sz^2 u^2)^{3/2} du
    for a normalised Gaussian density with rms widths (sr, sr, sz), kernel
    U = gdd (3 kz^2/k^2 - 1) without cutoff (derived from the momentum-space
    integral with |n(k)|^2 = exp(-(sr^2 (kx^2+ky^2) + sz^2 kz^2)))."""
    I1 = integrate.quad(lambda u: (3 * u * u - 1) / (sr**2 * (1 - u * u) + sz**2 * u * u) ** 1.5,
                        -1, 1, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
    return gdd * math.sqrt(math.pi) * I1 / (32.0 * math.pi**2)


@pytest.mark.parametrize("sr,sz", [(0.6, 0.45), (0.5, 0.8)])
def test_gaussian_dipolar_energy_closed_form(sr, sz):
    """Prefactor, angular form and cutoff of U: with the density compact inside the
    cutoff sphere R = L/2, the truncated periodic convolution equals the free-space
    interaction, whose energy has a one-dimensional integral closed form.  Prolate
    along z (dipole axis) -> E_dd < 0, oblate -> E_dd > 0."""
    p = O.Params(geom="3d", nx=64, ny=64, nz=64, dx=0.25, dy=0.25, dz=0.25, gdd=1.0, R=8.0)
    n = gaussian_density(p, (sz, sr, sr))
    edd = 0.5 * float(np.sum(O.dipolar_potential(n, p) * n)) * p.dV()
    ref = gaussian_edd_closed_form(sr, sz, 1.0)
    assert abs(edd - ref) <= 1e-10 * abs(ref)
    assert np.sign(edd) == (1 if sz < sr else -1)


def test_symmetric_density_has_zero_dipolar_energy():
    """A density symmetric under every permutation of the axes on a cubic grid has
    E_dd = 0 and Phi(origin) = 0 (the angular factor averages to zero)."""
    p = O.Params(geom="3d", nx=16, ny=16, nz=16, dx=0.3, dy=0.3, dz=0.3, gdd=1.0, R=2.4)
    rng = np.random.default_rng(3)
    a = rng.uniform(0, 1, size=p.shape())
    n = sum(np.transpose(a, perm) for perm in
            [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)])
    phi = O.dipolar_potential(n, p)
    edd = 0.5 * float(np.sum(phi * n)) * p.dV()
    scale = float(np.sum(np.abs(phi) * n)) * p.dV()
    assert abs(edd) <= 1e-14 * scale
    assert abs(phi[8, 8, 8]) <= 1e-14 * np.max(np.abs(phi))


@pytest.mark.parametrize("s", [1e-4, 1e-3, 0.05, 0.5, 0.99, 1.0, 1.01, 2.0, math.pi, 10.0, 55.0])
def test_cutoff_factor_is_spherical_bessel_integral(s):
    """Truncating (1 - 3cos^2)/r^3 to r < R multiplies the free kernel by
    b(kR) = 3 int_0^{kR} j_2(u)/u du (partial-wave expansion of the plane wave)."""
    ref = 3.0 * integrate.quad(lambda u: scipy.special.spherical_jn(2, u) / u, 0.0, s,
                               epsabs=1e-16, epsrel=1e-14, limit=400)[0]
    got = float(O.cutoff_factor(np.array([s]))[0])
    assert abs(got - ref) <= 2e-13 * max(abs(ref), 1e-300) + 1e-17


def test_kernel_limits_3d():
    p = O.Params(geom="3d", nx=8, ny=8, nz=8, dx=0.5, dy=0.5, dz=0.5, R=0.0)
    U = O.dipolar_kernel(p)
    assert U[0, 0, 0] == 0.0
    kz = O.wavenumbers(8, 0.5)
    assert abs(U[1, 0, 0] - 2.0) < 1e-15          # k along z: 3 - 1
    assert abs(U[0, 1, 0] + 1.0) < 1e-15          # k perpendicular: -1
    assert abs(U[0, 0, 1] + 1.0) < 1e-15
    assert kz[1] > 0


# -------------------------------------------------------------- 2D kernels
@pytest.mark.parametrize("geom", ["2dxy", "2dxz"])
def test_quasi2d_kernels_equal_transverse_quadrature_of_3d_kernel(geom):
    d = 0.5
    if geom == "2dxy":
        p = O.Params(geom=geom, nx=16, ny=12, dx=0.37, dy=0.29, lam=1.0 / d**2)
        ka = O.wavenumbers(12, 0.29)   # ky (rows)
    else:
        p = O.Params(geom=geom, nx=16, nz=12, dx=0.37, dz=0.29, nu=1.0 / d**2)
        ka = O.wavenumbers(12, 0.29)   # kz (rows)
    kx = O.half_wavenumbers(16, 0.37)
    U = O.dipolar_kernel(p)
    for r in (0, 1, 3, 6, 9):
        for c in (0, 1, 4, 8):
            if geom == "2dxy":
                q2 = kx[c] ** 2 + ka[r] ** 2

                def f(kp):
                    k2 = q2 + kp * kp
                    return (3 * kp * kp / k2 - 1.0) * math.exp(-kp * kp * d * d / 2) / (2 * math.pi)
            else:
                q2 = kx[c] ** 2 + ka[r] ** 2
                kz2 = ka[r] ** 2

                def f(kp):
                    k2 = q2 + kp * kp
                    if k2 == 0.0:
                        return -math.exp(-kp * kp * d * d / 2) / (2 * math.pi)
                    return (3 * kz2 / k2 - 1.0) * math.exp(-kp * kp * d * d / 2) / (2 * math.pi)
            ref = integrate.quad(f, -np.inf, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
            assert abs(U[r, c] - ref) <= 1e-10 * max(1.0, abs(ref)), (r, c, U[r, c], ref)
    pref = 1.0 / (math.sqrt(2 * math.pi) * d)
    if geom == "2dxy":
        assert abs(U[0, 0] - 2 * pref) < 1e-14
    else:
        assert abs(U[0, 0] + pref) < 1e-14


def test_quasi2d_contact_coupling():
    """g_2D = g int |w(z)|^4 dz for the normalised transverse Gaussian w."""
    d = 0.5
    p = O.Params(geom="2dxy", nx=8, ny=8, lam=1.0 / d**2, g=3.0)
    w2 = lambda z: math.exp(-z * z / d**2) / (math.sqrt(math.pi) * d)
    ref = 3.0 * integrate.quad(lambda z: w2(z) ** 2, -np.inf, np.inf)[0]
    assert abs(O.contact_coupling(p) - ref) < 1e-12


# --------------------------------------------------------------- CN sweeps
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("A", [0.3, 0.08j, 0.0125, 1.7j])
def test_cn_sweep_matches_dense_solve(axis, A):
    rng = np.random.default_rng(11)
    psi = rng.standard_normal((9, 7, 12)) + 1j * rng.standard_normal((9, 7, 12))
    psi = O.zero_boundary(psi)
    got = O.cn_sweep(psi, axis, A)
    n = psi.shape[axis]
    m = n - 2
    L = np.zeros((m, m), dtype=complex)
    Rm = np.zeros((m, n), dtype=complex)
    for i in range(m):
        L[i, i] = 1 + 2 * A
        if i > 0:
            L[i, i - 1] = -A
        if i < m - 1:
            L[i, i + 1] = -A
        Rm[i, i] = A
        Rm[i, i + 1] = 1 - 2 * A
        Rm[i, i + 2] = A
    a = np.moveaxis(psi, axis, 0).reshape(n, -1)
    ref = np.zeros_like(a)
    ref[1:-1] = np.linalg.solve(L, Rm @ a)
    ref = np.moveaxis(ref.reshape((n,) + np.moveaxis(psi, axis, 0).shape[1:]), 0, axis)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_real_time_cn_is_unitary():
    """The Cayley form (1 + i dt T/2)^-1 (1 - i dt T/2) preserves the discrete norm."""
    rng = np.random.default_rng(5)
    psi = O.zero_boundary(rng.standard_normal((20, 30)) + 1j * rng.standard_normal((20, 30)))
    out = O.cn_sweep(psi, 1, 0.4j)
    assert abs(np.sum(np.abs(out) ** 2) / np.sum(np.abs(psi) ** 2) - 1.0) < 1e-13


# -------------------------------------------- non-interacting ground states
def discrete_ground_energy(p):
    """Sum over axes of the lowest eigenvalue of -1/2 d^2/dx^2 + omega^2 x^2/2 on the
    interior points with Dirichlet ends (scipy's tridiagonal eigensolver)."""
    omegas = {"3d": (p.lam, p.nu, p.gamma), "2dxy": (p.nu, p.gamma),
              "2dxz": (p.lam, p.gamma)}[p.geom]
    e = 0.0
    for n, h, w in zip(p.shape(), p.spacings(), omegas):
        x = O.coords(n, h)[1:-1]
        diag = 1.0 / h**2 + 0.5 * w * w * x * x
        off = -0.5 / h**2 * np.ones(n - 3)
        e += scipy.linalg.eigh_tridiagonal(diag, off, select="i", select_range=(0, 0),
                                           eigvals_only=True)[0]
    return e


def relax(p, psi, nsteps):
    V = O.harmonic_potential(p)
    K = O.dipolar_kernel(p)
    for _ in range(nsteps):
        psi = O.step(psi, p, True, V=V, kernel=K)
    return psi, O.observables(psi, p, V=V, kernel=K)


@pytest.mark.parametrize("dt", [0.004, 0.002])
@pytest.mark.parametrize("nx,ny", [(40, 36), (41, 35)])
def test_noninteracting_2d_ground_energy_is_tridiagonal_eigenvalue_sum(dt, nx, ny):
    """g = g_dd = 0: imaginary time converges to the discrete ground state; E differs
    from the exact eigenvalue sum only by the O(dt^2) Lie-splitting offset (even and odd
    grids: an odd grid centres the trap on its middle point)."""
    p = O.Params(geom="2dxy", nx=nx, ny=ny, dx=0.3, dy=0.35, dt=dt, gamma=1.0, nu=1.7, lam=4.0)
    psi = I.gaussian("2dxy", nx, ny, 1, 0.3, 0.35, 0.3, widths=(0.8, 1.0), amp_noise=0.01, seed=1)
    psi, ob = relax(p, psi, int(16.0 / dt))
    e0 = discrete_ground_energy(p)
    err = ob["energy"] - e0
    assert 0 <= err <= 3.0 * dt * dt   # survey scale: 2.2e-6 at dt = 0.002
    assert abs(ob["norm"] - 1.0) < 1e-13


def test_noninteracting_2dxz_ground_state():
    """The x-z plane (program summaries (ii) and (v)): the trap acts with gamma along x
    and lambda along z, nu being the frozen transverse frequency.  With g = g_dd = 0 the
    relaxed energy is the sum of the two tridiagonal ground eigenvalues, x with gamma = 1
    and z with lambda = 2.5, within the O(dt^2) splitting offset; a swapped pair
    (gamma on z) gives a different sum on this non-square grid and fails.  The rms sizes
    are those of the harmonic ground state, 1/sqrt(2 omega) per axis, to O(h^2)."""
    dt = 0.002
    gam, lam = 1.0, 2.5
    p = O.Params(geom="2dxz", nx=44, nz=36, dx=0.3, dz=0.2, dt=dt, gamma=gam, nu=4.0, lam=lam)
    psi = I.gaussian("2dxz", 44, 1, 36, 0.3, 0.3, 0.2, widths=(0.8, 1.1), amp_noise=0.01,
                     seed=4)
    psi, ob = relax(p, psi, int(12.0 / dt))

    def eig(n, h, w):
        x = O.coords(n, h)[1:-1]
        return scipy.linalg.eigh_tridiagonal(1.0 / h**2 + 0.5 * w * w * x * x,
                                             -0.5 / h**2 * np.ones(n - 3), select="i",
                                             select_range=(0, 0), eigvals_only=True)[0]
    e0 = eig(44, 0.3, gam) + eig(36, 0.2, lam)
    swapped = eig(44, 0.3, lam) + eig(36, 0.2, gam)
    err = ob["energy"] - e0
    assert 0 <= err <= 3.0 * dt * dt, err
    assert abs(swapped - e0) > 100 * 3.0 * dt * dt
    # continuum (gamma + lambda)/2 to O(h^2)
    assert abs(ob["energy"] - 0.5 * (gam + lam)) < 0.02
    assert ob["rms"][1] == 0.0
    assert abs(ob["rms"][0] - 1.0 / math.sqrt(2.0 * gam)) < 0.01
    assert abs(ob["rms"][2] - 1.0 / math.sqrt(2.0 * lam)) < 0.01


def test_kohn_dipole_mode_along_z_in_2dxz():
    """The x-z plane with in-plane dipoles: a ground state displaced along z oscillates
    at lambda, the z trap frequency, whatever g and g_dd: <z>(pi/lambda) = -z0, while
    <x> stays at 0."""
    p = O.Params(geom="2dxz", nx=48, nz=64, dx=0.25, dz=0.15, dt=0.002, gamma=1.0, nu=4.0,
                 lam=2.0, g=15.0, gdd=10.0)
    psi = I.gaussian("2dxz", 48, 1, 64, 0.25, 0.25, 0.15, widths=(0.7, 1.0))
    psi, _ = relax(p, psi, 3000)
    m = 4
    z0 = m * p.dz
    f = np.roll(psi, m, axis=0)
    pr = O.Params(**{**p.__dict__, "dt": 0.0005})
    V = O.harmonic_potential(p)
    K = O.dipolar_kernel(p)
    Z, X = O.mesh(p)
    for _ in range(int(round(math.pi / p.lam / pr.dt))):
        f = O.step(f, pr, False, V=V, kernel=K)
    nrm = float(np.sum(np.abs(f) ** 2))
    zm = float(np.sum(Z * np.abs(f) ** 2) / nrm)
    xm = float(np.sum(X * np.abs(f) ** 2) / nrm)
    assert abs(zm + z0) < 2e-3 * z0, (zm, z0)
    assert abs(xm) < 1e-10


def test_noninteracting_3d_ground_energy():
    p = O.Params(geom="3d", nx=20, ny=18, nz=16, dx=0.45, dy=0.5, dz=0.4, dt=0.002,
                 gamma=1.0, nu=1.2, lam=2.0)
    psi = I.gaussian("3d", 20, 18, 16, 0.45, 0.5, 0.4, widths=(0.7, 0.9, 1.0), amp_noise=0.01, seed=2)
    psi, ob = relax(p, psi, 6000)
    e0 = discrete_ground_energy(p)
    assert 0 <= ob["energy"] - e0 <= 3e-5
    # rms of the discrete ground state ~ continuum 1/sqrt(2 omega) to O(dx^2)
    assert abs(ob["rms"][0] - 1 / math.sqrt(2.0)) < 0.02


def test_continuum_ground_energy_is_half_sum_of_frequencies():
    """(gamma + nu)/2 in 2D (the quasi-2D energy excludes the frozen direction):
    the error of the discrete scheme is O(dx^2), ratio ~4 when dx halves."""
    errs = []
    for n, h in ((24, 0.5), (48, 0.25)):
        p = O.Params(geom="2dxy", nx=n, ny=n, dx=h, dy=h, dt=0.001, gamma=1.0, nu=2.0, lam=4.0)
        psi = I.gaussian("2dxy", n, n, 1, h, h, h, widths=(0.7, 1.0))
        psi, ob = relax(p, psi, 9000)
        errs.append(ob["energy"] - 1.5)
    ratio = errs[0] / errs[1]
    assert -0.02 < errs[1] < 0
    assert 3.3 < ratio < 4.7, (errs, ratio)


# ------------------------------------------------------ interacting dynamics
def test_real_time_norm_conserved_with_interactions():
    p = O.Params(geom="3d", nx=16, ny=20, nz=18, dx=0.4, dy=0.35, dz=0.45, dt=0.002,
                 gamma=1.0, nu=1.3, lam=2.0, g=40.0, gdd=15.0, R=3.0)
    psi = I.gaussian("3d", 16, 20, 18, 0.4, 0.35, 0.45, widths=(0.8, 1.0, 1.0),
                     phase_noise=0.01, seed=9)
    V = O.harmonic_potential(p)
    K = O.dipolar_kernel(p)
    for _ in range(200):
        psi = O.step(psi, p, False, V=V, kernel=K)
    assert abs(np.sum(np.abs(psi) ** 2) * p.dV() - 1.0) < 1e-12


@pytest.fixture(scope="module")
def ground_2d():
    p = O.Params(geom="2dxy", nx=64, ny=64, dx=0.2, dy=0.2, dt=0.002, gamma=1.0, nu=1.3,
                 lam=4.0, g=10.0, gdd=5.0)
    psi = I.gaussian("2dxy", 64, 64, 1, 0.2, 0.2, 0.2, widths=(1.0, 1.0))
    psi, ob = relax(p, psi, 4000)
    return p, psi, ob


def test_kohn_dipole_mode(ground_2d):
    """Interactions are translation invariant, so a rigidly displaced ground state
    oscillates at the trap frequency: <x>(pi/gamma) = -x0, independent of g, g_dd."""
    p, psi, _ = ground_2d
    m = 3
    x0 = m * p.dx
    f = np.roll(psi, m, axis=1)
    pr = O.Params(**{**p.__dict__, "dt": 0.001})
    V = O.harmonic_potential(p)
    K = O.dipolar_kernel(p)
    X = O.mesh(p)[1]
    for _ in range(int(round(math.pi / p.gamma / pr.dt))):
        f = O.step(f, pr, False, V=V, kernel=K)
    xm = float(np.sum(X * np.abs(f) ** 2) / np.sum(np.abs(f) ** 2))
    assert abs(xm + x0) < 5e-4 * x0


def test_chemical_potential_is_imaginary_time_decay_rate(ground_2d):
    """At the stationary state one unnormalised imaginary step shrinks the norm by
    exp(-2 mu dt) up to O(dt^2): pins the factor 2 on both interaction terms in mu."""
    p, psi, ob = ground_2d
    V = O.harmonic_potential(p)
    K = O.dipolar_kernel(p)
    q = O.step(psi, p, True, V=V, kernel=K, renormalize=False)
    mu_decay = -math.log(float(np.sum(np.abs(q) ** 2)) * p.dV()) / (2 * p.dt)
    assert abs(mu_decay - ob["mu"]) < 1e-6 * ob["mu"]
    assert abs(ob["mu"] - ob["energy"]) > 0.1   # interactions present


def test_virial_theorem_3d():
    """Scaling argument: at the 3D ground state 2 E_kin - 2 E_pot + 3 E_int + 3 E_dd = 0
    (contact and dipolar energies scale as L^-3), up to discretisation error."""
    p = O.Params(geom="3d", nx=32, ny=32, nz=32, dx=0.35, dy=0.35, dz=0.35, dt=0.004,
                 gamma=1.0, nu=1.0, lam=2.0, g=20.0, gdd=6.0, R=5.6)
    psi = I.gaussian("3d", 32, 32, 32, 0.35, 0.35, 0.35, widths=(0.7, 1.0, 1.0))
    psi, ob = relax(p, psi, 1500)
    vir = 2 * ob["e_kin"] - 2 * ob["e_pot"] + 3 * ob["e_int"] + 3 * ob["e_dd"]
    assert abs(vir) < 0.02 * ob["energy"]


def test_imaginary_time_energy_decreases_monotonically():
    p = O.Params(geom="3d", nx=24, ny=24, nz=24, dx=0.35, dy=0.35, dz=0.35, dt=0.002,
                 gamma=1.0, nu=1.0, lam=2.0, g=20.0, gdd=6.0, R=4.2)
    psi = I.gaussian("3d", 24, 24, 24, 0.35, 0.35, 0.35, widths=(0.7, 1.0, 1.0),
                     amp_noise=0.01, seed=1601)
    _, hist = O.run(psi, p, True, 150, record=True)
    E = np.array([h["energy"] for h in hist])
    assert np.all(np.diff(E) <= 1e-14 * np.abs(E[1:]))
    assert all(abs(h["norm"] - 1.0) < 1e-13 for h in hist[1:])
