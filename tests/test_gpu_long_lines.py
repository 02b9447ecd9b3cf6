"""2D axes longer than one LDS line (more than 8192 points in FP32, 4096 in FP64; kind 3 of
gp_axis_kind): the x and y transforms by the four-step split n = A B through the
workspace, and the Crank-Nicolson sweeps in segments joined by their carries.  Parity with
the FP64 oracle through the C ABI at the bars of every other size: Phi rel-L2 1e-12 / 2e-6,
psi rel-L2 and element-wise 1e-10 / 2e-5, energy and mu 1e-12 / 1e-6.  Two starts: a
noisy Gaussian, whose density sits at low wavenumbers where U(k) varies (a slot holding
the wrong wavenumber shows there: for white noise U is nearly constant over most of the
spectrum, so Phi would only check that the transforms invert each other), and white
noise (every tile, segment and split column weighted)."""
import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import binding as B
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import (FP32_E_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            assert_psi_close, banner, obs_close, oparams, rel_l2)

pytestmark = pytest.mark.gpu


def grid(geom, n0, n1, dt=0.0005):
    """A 25.6-wide box along long axes, spacing 0.5 along short ones."""
    h0 = 25.6 / n0 if n0 > 100 else 0.5
    h1 = 25.6 / n1 if n1 > 100 else 0.5
    w = dict(geom=geom, nx=n0, ny=1, nz=1, dx=h0, dy=1.0, dz=1.0, dt=dt, gamma=1.0, nu=1.0,
             lam=4.0, g=10.0, gdd=5.0, R=0.0)
    if geom == "2dxy":
        w.update(ny=n1, dy=h1)
    else:
        w.update(nz=n1, dz=h1, nu=4.0, lam=1.0)
    return w


# (geometry, n0, n1, precisions); the split and segments each case exercises:
CASES = {
    # long x (A 100, B 90; 18 segments of 500), even and odd line count
    "2dxy_9000x12": ("2dxy", 9000, 12, ("fp32", "fp64")),
    "2dxy_9000x13": ("2dxy", 9000, 13, ("fp32", "fp64")),
    # long y (A 100, B 84; 20 segments of 420) in XZ
    "2dxz_10x8400": ("2dxz", 10, 8400, ("fp32", "fp64")),
    # primes 19 and 31 in the split (A 133 = 7 19, B 62 = 2 31): both factors by
    # Bluestein's algorithm (270- and 125-point stages; 19 segments of 434)
    "2dxy_8246x10": ("2dxy", 8246, 10, ("fp32",)),
    # a prime factor above 31 in the split (A 109 by Bluestein's algorithm, B 76; 19 segments
    # of 436), x and y
    "2dxy_8284x9": ("2dxy", 8284, 9, ("fp32",)),
    "2dxy_12x8284": ("2dxy", 12, 8284, ("fp32",)),
    # both axes long (FP64: A 70, B 60 along x, 10 segments of 420; A 72, B 57 along y,
    # 9 segments of 456)
    "2dxy_4200x4104": ("2dxy", 4200, 4104, ("fp64",)),
    # FP64 lengths just past the line (4098 = 2 3 683: A 683 by Bluestein, B 6; two
    # segments of 2049, 8 waves per segment line)
    "2dxz_4098x16": ("2dxz", 4098, 16, ("fp64",)),
}
PARAMS = [(name, prec) for name, c in CASES.items() for prec in c[3]]


def bars(prec):
    return (FP64_PSI_TOL, FP64_E_TOL) if prec == "fp64" else (FP32_PSI_TOL, FP32_E_TOL)


def smooth_start(w, seed):
    """Noisy Gaussian, widths 1.1 (axis 1) and 1.6 (x): most of the density at low k."""
    return I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                      widths=(1.1, 1.6), amp_noise=0.05, phase_noise=0.02, seed=seed)


@pytest.mark.parametrize("name,prec", PARAMS)
def test_long_axes_match_oracle(name, prec, gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    geom, n0, n1, _ = CASES[name]
    assert 3 in (B.gp_axis_kind(n0, prec), B.gp_axis_kind(n1, prec))
    w = grid(geom, n0, n1)
    banner("long axes", name, prec)
    p = oparams(w)
    ptol, etol = bars(prec)
    for kind, psi0 in (("gaussian", smooth_start(w, 611)),
                       ("noise", I.random_complex(p.shape(), 611, p.dV()))):
        s = Solver(w, prec=prec)
        s.set_psi(psi0)
        got = s.dipolar_potential()
        ref = O.dipolar_potential(np.abs(psi0) ** 2, p)
        err = rel_l2(got, ref)
        assert err <= (1e-12 if prec == "fp64" else 2e-6), (kind, err)
        assert not obs_close(s.energy(), O.observables(psi0, p), etol), kind
        s.close()
        for imag in (True, False):
            s = Solver(w, prec=prec)
            s.set_psi(psi0)
            s.step_imag(3) if imag else s.step_real(3)
            ref, hist = O.run(psi0, p, imag, 3, record=True)
            assert_psi_close(s.get_psi(), ref, ptol, (name, kind, imag))
            for k, (g_, r_) in enumerate(zip(s.history(3), hist)):
                bad = obs_close(g_, r_, etol)
                assert not bad, (name, kind, imag, k, bad)
            s.close()


def test_long_axes_fp32_both_long(gpu_lib):
    """Both axes past the FP32 line (8200 = A 100 x B 82 with B by Bluestein's algorithm,
    20 segments of 410; 8232 = 98 x 84, 21 segments of 392): Phi and two real-time steps."""
    from paper_1601_04640_amd.binding import Solver
    w = grid("2dxz", 8200, 8232)
    banner("long axes: both long, fp32")
    p = oparams(w)
    s = Solver(w, prec="fp32")
    psi0 = smooth_start(w, 612)
    s.set_psi(psi0)
    got = s.dipolar_potential()
    ref = O.dipolar_potential(np.abs(psi0) ** 2, p)
    assert rel_l2(got, ref) <= 2e-6, rel_l2(got, ref)
    del got, ref
    psi0 = I.random_complex(p.shape(), 612, p.dV())
    s.set_psi(psi0)
    s.step_real(2)
    assert_psi_close(s.get_psi(), O.run(psi0, p, False, 2), FP32_PSI_TOL)
    s.close()


def test_long_axes_graphs_and_direct_launches_agree(gpu_lib):
    """Graph-replayed steps (8 at a time) give bitwise the steps launched one by one."""
    from paper_1601_04640_amd.binding import Solver
    w = grid("2dxy", 9000, 12)
    banner("long axes: graph replay")
    p = oparams(w)
    psi0 = I.random_complex(p.shape(), 613, p.dV())
    out = []
    for graphs in (True, False):
        s = Solver(w, prec="fp32")
        s.use_graphs(graphs)
        s.set_psi(psi0)
        s.step_real(9)
        out.append(s.get_psi())
        s.close()
    assert np.array_equal(out[0], out[1])


def test_full_size_15000_plane_waves(gpu_lib):
    """The sweep's largest grid, 15000^2 FP32 (x and y split 125 x 120, segments of 500),
    in its own configuration.  The density is a constant plus plane waves reaching past
    row 60 of the split (kx = 130, 250: columns ka 1 and 2) and, through their images
    N - k, the rows rebuilt from conjugates; with the Dirichlet boundary zeroed it is
    compared with the oracle's Phi of the whole grid.  Then four real-time steps of a
    Gaussian conserve the norm."""
    from paper_1601_04640_amd.binding import Solver
    n = 15000
    h = 12.8 / n
    w = dict(geom="2dxy", nx=n, ny=n, nz=1, dx=h, dy=h, dz=1.0, dt=0.0005, gamma=1.0,
             nu=1.0, lam=4.0, g=20.0, gdd=6.0, R=0.0)
    banner("long axes: 15000^2 fp32 plane waves")
    assert B.gp_axis_kind(n, "fp32") == 3
    p = oparams(w)
    i = np.arange(n)
    rho = np.zeros((n, n))
    for (kx, ky, a) in [(0, 0, 1.0), (3, 5, 0.3), (130, 17, 0.2), (250, 211, 0.15),
                        (41, 0, 0.1)]:
        cx, sx = np.cos(2 * np.pi * kx * i / n), np.sin(2 * np.pi * kx * i / n)
        cy, sy = np.cos(2 * np.pi * ky * i / n), np.sin(2 * np.pi * ky * i / n)
        rho += a * (np.outer(cy, cx) - np.outer(sy, sx))
    psi = O.zero_boundary(np.sqrt(rho))
    del rho
    s = Solver(w, prec="fp32")
    s.set_psi(psi)
    got = s.dipolar_potential()
    ref = O.dipolar_potential(np.abs(psi) ** 2, p)
    del psi
    err = rel_l2(got, ref)
    mx = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print("15000^2 Phi: rel-L2", err, "max", mx, flush=True)
    assert err <= 2e-6 and mx <= 2e-5, (err, mx)
    del got, ref
    x = (i - n // 2) * h
    g1 = np.exp(-0.5 * x * x)
    g1[0] = g1[-1] = 0.0
    psi = np.outer(np.exp(-2.0 * x * x), g1).astype(np.complex64)
    s.set_psi(psi)
    del psi
    s.step_real(4)
    norms = [r["norm"] for r in s.history(4)]
    assert all(abs(v - norms[0]) <= 1e-5 * norms[0] for v in norms), norms
    s.close()


@pytest.mark.parametrize("prec,geom,n0,n1", [("fp32", "2dxy", 2560, 8192),
                                             ("fp64", "2dxz", 2048, 4000)])
def test_segmented_y_sweep_of_one_line_axes(prec, geom, n0, n1, gpu_lib):
    """A y axis that one LDS line holds but a tile does not (8192 = 16 x 512, FP32;
    4000 = 8 x 500, FP64), with enough columns for the segmented sweep in place over the
    strided columns (n0 x segments >= 40960 FP32 / 16384 FP64) instead of the transposed
    state: Phi, then imaginary and real steps against the oracle."""
    from paper_1601_04640_amd.binding import Solver
    assert B.gp_axis_kind(n1, prec) == 2
    w = grid(geom, n0, n1)
    banner("segmented y of a one-line axis", prec, geom, n0, n1)
    p = oparams(w)
    ptol, etol = bars(prec)
    psi0 = smooth_start(w, 614)
    for imag in (True, False):
        s = Solver(w, prec=prec)
        s.set_psi(psi0)
        if imag:
            err = rel_l2(s.dipolar_potential(), O.dipolar_potential(np.abs(psi0) ** 2, p))
            assert err <= (1e-12 if prec == "fp64" else 2e-6), err
        s.step_imag(2) if imag else s.step_real(2)
        ref, hist = O.run(psi0, p, imag, 2, record=True)
        assert_psi_close(s.get_psi(), ref, ptol, imag)
        for k, (g_, r_) in enumerate(zip(s.history(2), hist)):
            assert not obs_close(g_, r_, etol), (imag, k)
        s.close()
