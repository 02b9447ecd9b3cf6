"""The imaginary-time -> real-time hand-off through a saved state, and the output cadence,
through the C ABI, against the FP64 oracle: the records written every K steps, the saved
density, and the final state of the real-time run that starts from the loaded state
(with a quenched coupling and its own dt)."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import binding as B
from paper_1601_04640_amd import inputs as I
from paper_1601_04640_amd import pipeline as PL
from tests.gpu_util import (FP32_E_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            assert_psi_close, banner, obs_close, oparams)

pytestmark = pytest.mark.gpu

CASES = {
    "3d_24x20x16": dict(geom="3d", nx=24, ny=20, nz=16, dx=0.4, dy=0.45, dz=0.5, dt=0.002,
                        gamma=1.0, nu=1.3, lam=2.0, g=15.0, gdd=5.0, R=3.5),
    "2dxz_40x48": dict(geom="2dxz", nx=40, ny=1, nz=48, dx=0.3, dy=1.0, dz=0.25, dt=0.002,
                       gamma=1.0, nu=4.0, lam=1.5, g=12.0, gdd=8.0, R=0.0),
    # an x axis past one LDS line (four-step transforms, segmented sweeps), on a 256-wide
    # box: at the spacing of a 25.6-wide box (2.8e-3) FP32 energies sit at the 1e-6 bar on
    # one-line grids too (the kinetic differences subtract neighbours that agree to three
    # digits), and this test is about the hand-off
    "2dxy_9000x12": dict(geom="2dxy", nx=9000, ny=12, nz=1, dx=256.0 / 9000, dy=0.5, dz=1.0,
                         dt=0.002, gamma=1.0, nu=1.0, lam=4.0, g=12.0, gdd=8.0, R=0.0),
}
N_IMAG, N_REAL, EVERY = 30, 24, 8           # records at 0, 8, 16, 24 (and 30 in imag time)


def oracle_records(psi, p, imag, nsteps, every):
    recs, steps = [], list(range(0, nsteps + 1, every))
    if steps[-1] != nsteps:
        steps.append(nsteps)
    k = 0
    for s in steps:
        psi = O.run(psi, p, imag, s - k) if s > k else psi
        k = s
        recs.append((s, O.observables(psi, p), psi))
    return recs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_imag_to_real_through_state_file(case, prec, gpu_lib, tmp_path):
    w = CASES[case]
    wr = dict(w, dt=0.001, g=0.6 * w["g"])    # the real-time run: its own dt, quenched g
    banner("pipeline imag->file->real", case, prec)
    p, pr = oparams(w), oparams(wr)
    widths = (0.9, 1.0, 0.8) if w["geom"] == "3d" else (0.9, 1.0)
    psi0 = I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                      widths=widths, amp_noise=0.02, phase_noise=0.0, seed=41)
    out = str(tmp_path)
    rows_i = PL.imaginary_run(w, psi0, N_IMAG, EVERY, out, prec=prec)
    ref_i = oracle_records(psi0, p, True, N_IMAG, EVERY)
    ptol = FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL
    etol = FP64_E_TOL if prec == "fp64" else FP32_E_TOL
    keys = ("norm", "mu", "energy", "e_kin", "e_pot", "e_int", "e_dd")
    assert [r[0] for r in rows_i] == [s for s, _, _ in ref_i]
    for row, (s, ob, _) in zip(rows_i, ref_i):
        got = dict(zip(keys, row[2:9]), rms=row[9:12])
        assert row[1] == pytest.approx(s * w["dt"], rel=1e-15)
        assert not obs_close(got, ob, etol), (s, obs_close(got, ob, etol))
    # the table on disk holds the same records
    assert np.array_equal(np.array(PL.read_table(os.path.join(out, "imag-obs.txt"))),
                          np.array(rows_i, dtype=np.float64))
    ground = ref_i[-1][2]
    head, saved = B.gp_state_read(os.path.join(out, "imag-psi.gpd"))
    assert head["kind"] == B.GP_STATE_PSI and head["step"] == N_IMAG
    assert head["params"]["nx"] == w["nx"] and head["params"]["prec"] == prec
    assert_psi_close(saved, ground, ptol, "saved state")
    _, den = B.gp_state_read(os.path.join(out, "imag-den.gpd"))
    assert np.array_equal(den, saved.real ** 2 + saved.imag ** 2)
    # real time from the file, with the real-time parameters
    rows_r = PL.real_run(wr, N_REAL, EVERY, out, prec=prec, density_every=EVERY)
    ref_r = oracle_records(saved, pr, False, N_REAL, EVERY)
    assert [r[0] for r in rows_r] == [s for s, _, _ in ref_r]
    for row, (s, ob, psi_ref) in zip(rows_r, ref_r):
        got = dict(zip(keys, row[2:9]), rms=row[9:12])
        assert not obs_close(got, ob, etol), (s, obs_close(got, ob, etol))
        hd, d = B.gp_state_read(os.path.join(out, f"real-den-{s:06d}.gpd"))
        assert hd["kind"] == B.GP_STATE_DENSITY and hd["step"] == s
        dref = np.abs(psi_ref) ** 2
        assert np.max(np.abs(d - dref)) <= 2 * ptol * np.max(dref), s
    _, fin = B.gp_state_read(os.path.join(out, "real-psi.gpd"))
    assert_psi_close(fin, ref_r[-1][2], ptol, "after the real-time run")
    norms = [r[2] for r in rows_r]
    assert max(abs(n - norms[0]) for n in norms) <= (1e-13 if prec == "fp64" else 2e-6)


def test_state_round_trip_and_refusals(gpu_lib, tmp_path):
    from paper_1601_04640_amd.binding import Solver
    w = CASES["3d_24x20x16"]
    banner("pipeline state round trip")
    p = oparams(w)
    psi = I.random_complex(p.shape(), 7, p.dV())
    a = Solver(w, prec="fp64")
    a.set_psi(psi)
    path = str(tmp_path / "s.gpd")
    a.save_state(path, 5, 0.01)
    b = Solver(dict(w, g=1.0, dt=0.003), prec="fp64")   # other couplings and dt: accepted
    info = b.load_state(path)
    assert info["step"] == 5 and info["time"] == 0.01
    assert np.array_equal(b.get_psi(), a.get_psi())     # bit for bit through the file
    f = Solver(w, prec="fp32")                          # an FP32 context rounds on load
    f.load_state(path)
    assert np.array_equal(f.get_psi(), a.get_psi().astype(np.complex64).astype(np.complex128))
    other = Solver(dict(w, nx=20), prec="fp64")         # another grid: refused
    with pytest.raises(B.GPError) as e:
        other.load_state(path)
    assert e.value.status == B.GP_E_ARG
    spacing = Solver(dict(w, dx=0.41), prec="fp64")
    with pytest.raises(B.GPError) as e:
        spacing.load_state(path)
    assert e.value.status == B.GP_E_ARG
    a.save_density(str(tmp_path / "d.gpd"))
    with pytest.raises(B.GPError) as e:                 # a density is not a state
        b.load_state(str(tmp_path / "d.gpd"))
    assert e.value.status == B.GP_E_ARG
    raw = bytearray(open(path, "rb").read())
    raw[-3] ^= 4
    open(str(tmp_path / "bad.gpd"), "wb").write(bytes(raw))
    with pytest.raises(B.GPError) as e:
        b.load_state(str(tmp_path / "bad.gpd"))
    assert e.value.status == B.GP_E_IO
    for s in (a, b, f, other, spacing):
        s.close()


def test_evolve_stops_when_asked_and_matches_plain_steps(gpu_lib):
    from paper_1601_04640_amd.binding import Solver
    w = CASES["2dxz_40x48"]
    banner("pipeline evolve early stop")
    p = oparams(w)
    psi = I.random_complex(p.shape(), 8, p.dV())
    s = Solver(w, prec="fp64")
    s.set_psi(psi)
    seen = []
    done = s.evolve(True, 40, 8, lambda k, ob: seen.append(k) or k >= 16)
    assert done == 16 and seen == [0, 8, 16]
    t = Solver(w, prec="fp64")
    t.set_psi(psi)
    t.step_imag(16)
    assert np.array_equal(s.get_psi(), t.get_psi())     # the loop is the plain steps
    assert s.evolve(False, 5, 0) == 5                    # no callback: the steps only
    s.close()
    t.close()
