"""Axis lengths.  Those without compile-time specialised passes run the run-time-length
kernels: every length >= 4, even or odd, whose prime factors are at most 31, up to 8192
(FP32) / 4096 (FP64) points per line; and every specialised length is run in each role
(x, y and z line).  The paper's programs take any grid and enlarge it silently for
the FFT ("Unusual features"); here each length runs as given.  Parity with the FP64
oracle through the C ABI at the same bars as the specialised sizes: psi rel-L2 and
element-wise <= 1e-10 / 2e-5, energy and mu <= 1e-12 / 1e-6."""
import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import binding as B
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import (FP32_E_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            assert_psi_close, banner, obs_close, oparams, rel_l2)

pytestmark = pytest.mark.gpu

CASES = {
    # the paper's small grid (50 = 2 5^2) with 3^3 and 2^2 3^2 axes
    "3d_50x54x36": dict(geom="3d", nx=50, ny=54, nz=36, dx=0.3, dy=0.28, dz=0.4, dt=0.002,
                        gamma=1.0, nu=1.2, lam=2.0, g=25.0, gdd=8.0, R=4.0),
    # radices 7, 11, 13 (the larger-prime kernels)
    "3d_14x22x26": dict(geom="3d", nx=14, ny=22, nz=26, dx=0.7, dy=0.5, dz=0.4, dt=0.002,
                        gamma=1.0, nu=1.0, lam=1.5, g=10.0, gdd=4.0, R=3.0),
    # specialised x (48) with run-time-length y and z
    "3d_48x34x38": dict(geom="3d", nx=48, ny=34, nz=38, dx=0.3, dy=0.4, dz=0.35, dt=0.001,
                        gamma=1.0, nu=1.1, lam=1.8, g=30.0, gdd=12.0, R=5.0),
    "2dxy_100x90": dict(geom="2dxy", nx=100, ny=90, nz=1, dx=0.15, dy=0.18, dz=1.0, dt=0.002,
                        gamma=1.0, nu=1.5, lam=4.0, g=30.0, gdd=10.0, R=0.0),
    # 62 = 2 31, 98 = 2 7^2
    "2dxz_62x98": dict(geom="2dxz", nx=62, ny=1, nz=98, dx=0.25, dy=1.0, dz=0.12, dt=0.001,
                       gamma=1.0, nu=4.0, lam=2.5, g=20.0, gdd=15.0, R=0.0),
    # the paper's 2D sizes 540 and 600 (2^2 3^3 5 and 2^3 3 5^2)
    "2dxy_540x600": dict(geom="2dxy", nx=540, ny=600, nz=1, dx=0.04, dy=0.04, dz=1.0,
                         dt=0.0005, gamma=1.0, nu=1.2, lam=4.0, g=40.0, gdd=20.0, R=0.0),
    # degenerate lengths: 4 and 6 points (two and four interior points)
    "3d_4x6x10": dict(geom="3d", nx=4, ny=6, nz=10, dx=1.0, dy=0.8, dz=0.6, dt=0.002,
                      gamma=1.0, nu=1.0, lam=1.0, g=5.0, gdd=2.0, R=2.0),
    # odd lengths on every axis (45 = 3^2 5, 27 = 3^3, 35 = 5 7): the x passes' last line
    # pair of a plane holds one line, and the odd spectra have no Nyquist row
    "3d_45x27x35": dict(geom="3d", nx=45, ny=27, nz=35, dx=0.3, dy=0.35, dz=0.3, dt=0.002,
                        gamma=1.0, nu=1.1, lam=1.6, g=20.0, gdd=8.0, R=4.0),
    "2dxy_63x49": dict(geom="2dxy", nx=63, ny=49, nz=1, dx=0.2, dy=0.25, dz=1.0, dt=0.001,
                       gamma=1.0, nu=1.3, lam=4.0, g=25.0, gdd=10.0, R=0.0),
    # odd z in XZ (the x passes pair z lines); 5 points: three interior points
    "2dxz_40x55": dict(geom="2dxz", nx=40, ny=1, nz=55, dx=0.25, dy=1.0, dz=0.2, dt=0.001,
                       gamma=1.0, nu=4.0, lam=2.0, g=15.0, gdd=12.0, R=0.0),
    "3d_5x9x7": dict(geom="3d", nx=5, ny=9, nz=7, dx=1.0, dy=0.7, dz=0.8, dt=0.002,
                     gamma=1.0, nu=1.0, lam=1.2, g=5.0, gdd=2.0, R=2.0),
    # prime factors above 31 on every axis, by Bluestein's algorithm (convolution lengths
    # 75, 147 and 81): 37 and 41 prime, 74 = 2 37
    "3d_37x74x41": dict(geom="3d", nx=37, ny=74, nz=41, dx=0.35, dy=0.2, dz=0.3, dt=0.002,
                        gamma=1.0, nu=1.1, lam=1.5, g=20.0, gdd=8.0, R=4.0),
    # 106 = 2 53 as x, 97 (prime) as the convolution axis
    "2dxy_106x97": dict(geom="2dxy", nx=106, ny=97, nz=1, dx=0.15, dy=0.16, dz=1.0, dt=0.001,
                        gamma=1.0, nu=1.2, lam=4.0, g=25.0, gdd=10.0, R=0.0),
    # 1009 (prime) x lines in XZ
    "2dxz_1009x24": dict(geom="2dxz", nx=1009, ny=1, nz=24, dx=0.02, dy=1.0, dz=0.4,
                         dt=0.0005, gamma=1.0, nu=4.0, lam=1.5, g=15.0, gdd=10.0, R=0.0),
}


def start_state(w, seed):
    widths = {"3d": (0.8, 1.0, 1.1), "2dxy": (0.9, 1.1), "2dxz": (0.8, 1.0)}[w["geom"]]
    return I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                      widths=widths, amp_noise=0.05, phase_noise=0.02, seed=seed)


def bars(prec):
    return (FP64_PSI_TOL, FP64_E_TOL) if prec == "fp64" else (FP32_PSI_TOL, FP32_E_TOL)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_dipolar_potential_and_energy(name, prec, gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    w = CASES[name]
    banner("run-time-length sizes: Phi and energy", name, prec)
    p = oparams(w)
    psi = start_state(w, 501)
    s = Solver(w, prec=prec)
    s.set_psi(psi)
    got = s.dipolar_potential()
    ref = O.dipolar_potential(np.abs(psi) ** 2, p)
    assert rel_l2(got, ref) <= (1e-12 if prec == "fp64" else 2e-6), rel_l2(got, ref)
    bad = obs_close(s.energy(), O.observables(psi, p), bars(prec)[1])
    assert not bad, bad
    s.close()


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_steps_match_oracle(name, prec, imag, gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    w = CASES[name]
    nsteps = 4 if name == "2dxy_540x600" else 12
    banner("run-time-length sizes: steps", name, prec, "imag" if imag else "real", nsteps)
    p = oparams(w)
    psi0 = start_state(w, 502)
    s = Solver(w, prec=prec)
    s.set_psi(psi0)
    s.step_imag(nsteps) if imag else s.step_real(nsteps)
    ref, hist = O.run(psi0, p, imag, nsteps, record=True)
    ptol, etol = bars(prec)
    assert_psi_close(s.get_psi(), ref, ptol)
    recs = s.history(nsteps)
    assert len(recs) == nsteps
    for k, (g_, r_) in enumerate(zip(recs, hist)):
        bad = obs_close(g_, r_, etol)
        assert not bad, (k, bad)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_random_field_start(prec, gpu_lib):
    """A white-noise start puts weight on every tile, the ragged ones included."""
    from paper_1601_04640_amd.binding import Solver
    w = CASES["3d_50x54x36"]
    banner("run-time-length sizes: random field", prec)
    p = oparams(w)
    psi0 = I.random_complex(p.shape(), 503, p.dV())
    for imag in (True, False):
        s = Solver(w, prec=prec)
        s.set_psi(psi0)
        s.step_imag(10) if imag else s.step_real(10)
        ref = O.run(psi0, p, imag, 10)
        assert_psi_close(s.get_psi(), ref, bars(prec)[0], imag)
        s.close()


@pytest.mark.parametrize("prec,n", [("fp32", 8192), ("fp64", 4096), ("fp64", 2 * 3 * 7 * 29),
                                    ("fp32", 4093), ("fp64", 2039)])
def test_longest_lines(prec, n, gpu_lib):
    """The longest x and y lines one block holds (and a 29-point radix; and the longest
    primes, by Bluestein's algorithm through 8192 / 4096-point FFTs) in 2D: Phi of a
    smooth start, then real-time steps of white noise (x sweeps of several waves per
    line, y sweeps on the transposed state)."""
    from paper_1601_04640_amd.binding import Solver
    for nx, ny in ((n, 12), (12, n)):
        h = 25.6 / n
        w = dict(geom="2dxy", nx=nx, ny=ny, nz=1, dx=h if nx == n else 0.5,
                 dy=h if ny == n else 0.5, dz=1.0, dt=0.0005, gamma=1.0, nu=1.0, lam=4.0,
                 g=10.0, gdd=5.0, R=0.0)
        banner("run-time-length sizes: longest line", prec, nx, ny)
        p = oparams(w)
        s = Solver(w, prec=prec)
        # Phi of a smooth start: its density sits where U(k) varies, so every wavenumber
        # must land in its own slot (white noise mostly checks that the transforms invert)
        smooth = I.gaussian("2dxy", nx, ny, 1, w["dx"], w["dy"], 1.0, widths=(1.1, 1.6),
                            amp_noise=0.05, seed=506)
        s.set_psi(smooth)
        err = rel_l2(s.dipolar_potential(), O.dipolar_potential(np.abs(smooth) ** 2, p))
        assert err <= (1e-12 if prec == "fp64" else 2e-6), (nx, ny, err)
        psi0 = I.random_complex(p.shape(), 504, p.dV())
        s.set_psi(psi0)
        s.step_real(3)
        assert_psi_close(s.get_psi(), O.run(psi0, p, False, 3), bars(prec)[0], (nx, ny))
        s.close()


def test_graph_replay_equals_direct_launches(gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    w = CASES["3d_50x54x36"]
    banner("run-time-length sizes: graph replay")
    psi0 = start_state(w, 505)
    out = []
    for graphs in (True, False):
        s = Solver(w, prec="fp32")
        s.use_graphs(graphs)
        s.set_psi(psi0)
        s.step_imag(17)
        s.step_real(16)
        out.append((s.get_psi(), s.history(33)))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_calls_needing_specialised_lengths_refuse(gpu_lib):
    import torch
    from paper_1601_04640_amd.binding import Solver
    w = CASES["3d_14x22x26"]
    banner("run-time-length sizes: refusals")
    s = Solver(w, prec="fp64")
    s.set_psi(start_state(w, 506))
    z = torch.zeros(s.shape, dtype=torch.complex128, device="cuda:0")
    gv = torch.zeros(s.shape, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    with pytest.raises(B.GPError) as e:
        B.gp_step_real_adjoint(s.ctx, z.data_ptr(), z.data_ptr(), gv.data_ptr(), g.data_ptr(),
                               g.data_ptr() + 8)
    assert e.value.status == B.GP_E_SIZE
    with pytest.raises(B.GPError) as e:
        B.gp_dipolar_potential_noalloc(B.make_params(**{**w, "prec": "fp64"}), z.data_ptr(),
                                       gv.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert e.value.status == B.GP_E_SIZE
    with pytest.raises(B.GPError) as e:
        B.Batch([dict(w, geom="2dxy", nz=1)], prec="fp64")
    assert e.value.status == B.GP_E_SIZE
    s.close()


SPECIALISED = (8, 10, 12, 16, 20, 24, 30, 32, 40, 48, 60, 64, 80, 96, 120, 128, 160, 192,
               240, 256, 320, 384, 480, 512)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", SPECIALISED)
def test_every_specialised_length_in_every_role(n, prec, gpu_lib):
    """Each compile-time specialised length as the x line (2D XY, n x 12), the y line
    (2D XY, 12 x n) and the z line (3D 12 x 10 x n), from a white-noise start: three
    real-time steps against the oracle."""
    from paper_1601_04640_amd.binding import Solver
    assert B.gp_axis_kind(n, prec) == 1
    h = 12.0 / n
    roles = {
        "x": dict(geom="2dxy", nx=n, ny=12, nz=1, dx=h, dy=0.9, dz=1.0),
        "y": dict(geom="2dxy", nx=12, ny=n, nz=1, dx=0.9, dy=h, dz=1.0),
        "z": dict(geom="3d", nx=12, ny=10, nz=n, dx=0.9, dy=1.0, dz=h),
    }
    for role, g in roles.items():
        w = dict(g, dt=0.001, gamma=1.0, nu=1.2, lam=2.0 if g["geom"] == "3d" else 4.0,
                 g=15.0, gdd=5.0, R=2.5 if g["geom"] == "3d" else 0.0)
        banner("specialised length", n, "as", role, prec)
        p = oparams(w)
        psi0 = I.random_complex(p.shape(), 600 + n, p.dV())
        s = Solver(w, prec=prec)
        s.set_psi(psi0)
        s.step_real(3)
        assert_psi_close(s.get_psi(), O.run(psi0, p, False, 3), bars(prec)[0], (n, role))
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(12, 1100, 10), (10, 12, 1100), (1100, 10, 12)])
def test_long_lines_3d(shape, prec, gpu_lib):
    """3D lines longer than 1024 points (1100 = 2^2 5^2 11) along each axis: sweeps of
    several waves per line over strided tiles of few lines, and the x sweep with the
    nonlinear sub-step; imaginary and real time against the oracle."""
    from paper_1601_04640_amd.binding import Solver
    nx, ny, nz = shape
    h = {a: (12.0 / n if n > 100 else 0.8) for a, n in zip("xyz", shape)}
    w = dict(geom="3d", nx=nx, ny=ny, nz=nz, dx=h["x"], dy=h["y"], dz=h["z"], dt=0.001,
             gamma=1.0, nu=1.2, lam=1.5, g=15.0, gdd=5.0, R=2.0)
    banner("run-time-length sizes: long 3D lines", shape, prec)
    p = oparams(w)
    psi0 = I.random_complex(p.shape(), 507, p.dV())
    for imag in (True, False):
        s = Solver(w, prec=prec)
        s.set_psi(psi0)
        s.step_imag(3) if imag else s.step_real(3)
        ref, hist = O.run(psi0, p, imag, 3, record=True)
        ptol, etol = bars(prec)
        assert_psi_close(s.get_psi(), ref, ptol, (shape, imag))
        for k, (g_, r_) in enumerate(zip(s.history(3), hist)):
            bad = obs_close(g_, r_, etol)
            assert not bad, (shape, imag, k, bad)
        s.close()


@pytest.mark.parametrize("prec,shape", [("fp64", (64, 1100, 512)), ("fp32", (64, 512, 1100))])
def test_long_lines_3d_by_columns(prec, shape, gpu_lib):
    """3D y or z lines longer than 1024 points with at least 32768 of them (64 x 512): the
    sweep runs one thread per line with the forward values in the scratch grid
    (kg_cn_cols); 1100 = 2^2 5^2 11.  Phi of a smooth start, then an imaginary and a
    real step against the oracle, with the record and the energy of the new state (the
    observables' z sums run the same kernel)."""
    from paper_1601_04640_amd.binding import Solver
    nx, ny, nz = shape
    h = {a: 12.0 / n for a, n in zip("xyz", shape)}
    w = dict(geom="3d", nx=nx, ny=ny, nz=nz, dx=h["x"], dy=h["y"], dz=h["z"], dt=0.001,
             gamma=1.0, nu=1.2, lam=1.5, g=15.0, gdd=5.0, R=2.0)
    banner("run-time-length sizes: 3D long lines by columns", shape, prec)
    p = oparams(w)
    psi0 = I.gaussian("3d", nx, ny, nz, h["x"], h["y"], h["z"], widths=(1.2, 1.0, 0.9),
                      amp_noise=0.05, phase_noise=0.02, seed=508)
    ptol, etol = bars(prec)
    for imag in (True, False):
        s = Solver(w, prec=prec)
        s.set_psi(psi0)
        if imag:
            err = rel_l2(s.dipolar_potential(), O.dipolar_potential(np.abs(psi0) ** 2, p))
            assert err <= (1e-12 if prec == "fp64" else 2e-6), err
        s.step_imag(1) if imag else s.step_real(1)
        ref, hist = O.run(psi0, p, imag, 1, record=True)
        assert_psi_close(s.get_psi(), ref, ptol, (shape, imag))
        assert not obs_close(s.history(1)[0], hist[0], etol), (shape, imag)
        assert not obs_close(s.energy(), O.observables(ref, p), etol), (shape, imag)
        s.close()
