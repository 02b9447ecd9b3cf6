"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded
inputs.  Sizes are chosen so the oracle finishes in seconds while spanning several tiles
with ragged tails (x lines are processed 16 (or 8) per block, strided columns 16 (or 8)
per block).  Tolerances: psi rel-L2 <= 1e-10 (FP64) / 2e-5 (FP32); energy and mu
relative <= 1e-12 (FP64) / 1e-6 (FP32)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import (FP32_E_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            assert_psi_close, banner, obs_close, oparams, rel, rel_l2)

pytestmark = pytest.mark.gpu

CASES = {
    # 3D: ragged x-line tiles (ny = 20, 40 not multiples of 16), ragged column tiles
    "3d_24x20x16": dict(geom="3d", nx=24, ny=20, nz=16, dx=0.35, dy=0.4, dz=0.45, dt=0.002,
                        gamma=1.0, nu=1.3, lam=2.0, g=25.0, gdd=8.0, R=2.8),
    "3d_40x30x48": dict(geom="3d", nx=40, ny=30, nz=48, dx=0.3, dy=0.35, dz=0.25, dt=0.001,
                        gamma=1.0, nu=1.1, lam=1.8, g=30.0, gdd=12.0, R=5.0),
    "3d_64x48x20": dict(geom="3d", nx=64, ny=48, nz=20, dx=0.25, dy=0.3, dz=0.5, dt=0.002,
                        gamma=1.0, nu=1.0, lam=2.0, g=20.0, gdd=6.0, R=0.0),
    "2dxy_48x40": dict(geom="2dxy", nx=48, ny=40, nz=1, dx=0.25, dy=0.3, dz=1.0, dt=0.002,
                       gamma=1.0, nu=1.5, lam=4.0, g=30.0, gdd=10.0, R=0.0),
    "2dxz_30x64": dict(geom="2dxz", nx=30, ny=1, nz=64, dx=0.4, dy=1.0, dz=0.2, dt=0.001,
                       gamma=1.0, nu=4.0, lam=2.5, g=20.0, gdd=15.0, R=0.0),
    "2dxy_120x96": dict(geom="2dxy", nx=120, ny=96, nz=1, dx=0.15, dy=0.15, dz=1.0, dt=0.001,
                        gamma=1.0, nu=1.2, lam=4.0, g=40.0, gdd=20.0, R=0.0),
    # 256-point z lines: the z convolution runs as two 16-point stages held in registers
    # (FP64: real and imaginary parts exchanged in turn); ny = 20 leaves a ragged
    # 4-column tile, ny = 10 a single tile of 10 of its 16 columns
    "3d_12x20x256": dict(geom="3d", nx=12, ny=20, nz=256, dx=0.5, dy=0.45, dz=0.04,
                         dt=0.0005, gamma=1.0, nu=1.0, lam=1.0, g=15.0, gdd=6.0, R=2.0),
    "3d_16x10x256": dict(geom="3d", nx=16, ny=10, nz=256, dx=0.5, dy=0.55, dz=0.04,
                         dt=0.0005, gamma=1.0, nu=1.2, lam=1.0, g=12.0, gdd=5.0, R=2.2),
    # 256-point x lines: FP64 R2C tiles of 16 lines (ny = 20: one full, one of 4), with
    # their own count of x-difference partials in the energy
    "3d_256x20x12": dict(geom="3d", nx=256, ny=20, nz=12, dx=0.05, dy=0.5, dz=0.55,
                         dt=0.0005, gamma=1.0, nu=1.0, lam=1.2, g=15.0, gdd=6.0, R=2.0),
    # 256-point y lines: the FP32 y FFT runs 16 x 16 with one LDS exchange; 7 x 20 = 140
    # lines leave a ragged last block of 16
    "3d_12x256x20": dict(geom="3d", nx=12, ny=256, nz=20, dx=0.5, dy=0.04, dz=0.45,
                         dt=0.0005, gamma=1.0, nu=1.0, lam=1.0, g=15.0, gdd=6.0, R=2.0),
    # 2048 x-line tiles: the FP64 finalisation runs in two stages (pre-reduced slices)
    "3d_16x64x512": dict(geom="3d", nx=16, ny=64, nz=512, dx=0.45, dy=0.12, dz=0.02,
                         dt=0.0005, gamma=1.0, nu=1.0, lam=1.0, g=10.0, gdd=4.0, R=1.5),
}


def start_state(w, seed, noise=True):
    shape_axes = {"3d": (0.8, 1.0, 1.1), "2dxy": (0.9, 1.1), "2dxz": (0.8, 1.0)}[w["geom"]]
    return I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                      widths=shape_axes, amp_noise=0.05 if noise else 0.0,
                      phase_noise=0.02 if noise else 0.0, seed=seed)


def make_solver(w, prec):
    from paper_1601_04640_amd.binding import Solver
    return Solver(w, prec=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_dipolar_potential(name, prec, gpu_lib):
    w = CASES[name]
    banner("dipolar_potential", name, prec)
    psi = start_state(w, 101)
    s = make_solver(w, prec)
    s.set_psi(psi)
    got = s.dipolar_potential()
    ref = O.dipolar_potential(np.abs(psi) ** 2, oparams(w))
    err = rel_l2(got, ref)
    assert err <= (1e-12 if prec == "fp64" else 2e-6), err
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_energy_observables(name, prec, gpu_lib):
    w = CASES[name]
    banner("energy", name, prec)
    psi = start_state(w, 102)
    s = make_solver(w, prec)
    s.set_psi(psi)
    got = s.energy()
    ref = O.observables(psi, oparams(w))
    bad = obs_close(got, ref, FP64_E_TOL if prec == "fp64" else FP32_E_TOL)
    assert not bad, bad
    s.close()


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_steps_match_oracle(name, prec, imag, gpu_lib):
    w = CASES[name]
    nsteps = 12
    banner("steps", name, prec, "imag" if imag else "real", nsteps)
    psi0 = start_state(w, 103)
    p = oparams(w)
    s = make_solver(w, prec)
    s.set_psi(psi0)
    s.step_imag(nsteps) if imag else s.step_real(nsteps)
    got = s.get_psi()
    ref, hist = O.run(psi0, p, imag, nsteps, record=True)
    assert_psi_close(got, ref, FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL)
    # per-step records: observables of the state each step started from, at the bars
    recs = s.history(nsteps)
    assert len(recs) == nsteps
    etol = (dict(tol=FP64_E_TOL) if prec == "fp64"
            else dict(tol=FP32_E_TOL))
    for k, (g_, r_) in enumerate(zip(recs, hist)):
        bad = obs_close(g_, r_, **etol)
        assert not bad, (k, bad)
    s.close()


# one case per geometry plus the ragged 3D tiles: a white-noise start, which puts weight
# on every tile (boundary tiles and ragged tails included) instead of a localised cloud
RANDOM_CASES = ["3d_24x20x16", "3d_40x30x48", "2dxy_48x40", "2dxz_30x64", "2dxy_120x96"]


@pytest.mark.parametrize("imag", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", RANDOM_CASES)
def test_random_field_steps_match_oracle(name, prec, imag, gpu_lib):
    w = CASES[name]
    nsteps = 12
    banner("random-field steps", name, prec, "imag" if imag else "real", nsteps)
    p = oparams(w)
    psi0 = I.random_complex(p.shape(), 401, p.dV())
    s = make_solver(w, prec)
    s.set_psi(psi0)
    s.step_imag(nsteps) if imag else s.step_real(nsteps)
    got = s.get_psi()
    ref, hist = O.run(psi0, p, imag, nsteps, record=True)
    assert_psi_close(got, ref, FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL)
    etol = (dict(tol=FP64_E_TOL) if prec == "fp64"
            else dict(tol=FP32_E_TOL))
    for k, (g_, r_) in enumerate(zip(s.history(nsteps), hist)):
        bad = obs_close(g_, r_, **etol)
        assert not bad, (k, bad)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_set_potential_and_quench(prec, gpu_lib):
    """Arbitrary grid V through gp_set_potential, then a coupling quench."""
    w = CASES["2dxy_48x40"]
    banner("set_potential+quench", prec)
    p = oparams(w)
    V = O.harmonic_potential(p) + 0.3 * I.smooth_random_field(p.shape(), p.spacings(), 1.0, 7)
    psi0 = start_state(w, 104)
    s = make_solver(w, prec)
    s.set_psi(psi0)
    s.set_potential(V)
    s.step_imag(10)
    s.step_real(9)
    s.set_couplings(12.0, 3.0)      # captured graphs must pick up the new couplings
    s.step_real(9)
    got = s.get_psi()
    ref = O.run(psi0, p, True, 10, V=V)
    ref = O.run(ref, p, False, 9, V=V)
    p2 = oparams({**w, "g": 12.0, "gdd": 3.0})
    ref = O.run(ref, p2, False, 9, V=V)
    assert_psi_close(got, ref, FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL)
    s.close()


def test_device_io_roundtrip(gpu_lib):
    import torch
    w = CASES["3d_24x20x16"]
    banner("device io roundtrip")
    psi = start_state(w, 105)
    for prec in ("fp64", "fp32"):
        s = make_solver(w, prec)
        t = torch.from_numpy(psi).to("cuda:0")
        s.set_psi(t)
        back = s.get_psi_device().cpu().numpy()
        tol = 1e-15 if prec == "fp64" else 1e-7
        assert rel_l2(back.astype(np.complex128), psi) < tol
        s.close()


def test_state_and_nonfinite_errors(gpu_lib):
    from paper_1601_04640_amd import binding as B
    w = CASES["2dxy_48x40"]
    banner("state errors / nonfinite flag")
    s = make_solver(w, "fp64")
    with pytest.raises(B.GPError) as e:
        s.step_real(1)
    assert e.value.status == B.GP_E_STATE
    with pytest.raises(B.GPError) as e:
        s.energy()
    assert e.value.status == B.GP_E_STATE
    psi = start_state(w, 106)
    psi[10, 10] = np.nan
    s.set_psi(psi)
    s.step_imag(2)
    with pytest.raises(B.GPError) as e:
        s.sync()
    assert e.value.status == B.GP_E_NONFINITE
    s.close()


def test_zero_steps_and_boundary_zeroing(gpu_lib):
    w = CASES["3d_24x20x16"]
    banner("zero steps / boundary")
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((16, 20, 24)) + 1j * rng.standard_normal((16, 20, 24))
    s = make_solver(w, "fp64")
    s.set_psi(psi)
    s.step_real(0)
    got = s.get_psi()
    assert np.array_equal(got, O.zero_boundary(psi))
    s.close()


def test_history_ring_wraps(gpu_lib):
    """Past the ring's capacity the history holds the latest records, oldest first: the
    records read before the wrap reappear bit for bit, followed by the new ones."""
    from paper_1601_04640_amd import binding as B
    cap = B.load().gp_history_capacity()
    w = dict(CASES["2dxy_48x40"], nx=32, ny=32)
    banner("history ring wrap", cap)
    s = make_solver(w, "fp64")
    s.set_psi(start_state(w, seed=12))
    first = cap - 6
    s.step_imag(first)
    h1 = s.history(first)
    assert len(h1) == first
    s.step_imag(20)
    h2 = s.history(cap + 100)
    assert len(h2) == cap
    key = lambda h: [h[k] for k in sorted(h)]
    assert [key(h) for h in h2[:cap - 20]] == [key(h) for h in h1[20 - 6:]]
    tail = s.history(20)
    assert [key(h) for h in h2[cap - 20:]] == [key(h) for h in tail]
    # every record left in the wrapped ring is of a state the previous step renormalised
    assert all(abs(h["norm"] - 1.0) < 1e-12 for h in h2)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_equals_direct_launches(prec, gpu_lib):
    """Steps replayed from captured HIP graphs are bitwise equal to direct launches, for
    every replay, with host synchronisation and eager work between replays."""
    w = CASES["3d_40x30x48"]
    banner("graph vs direct", prec)
    psi0 = start_state(w, 107)
    runs = []
    for graphs in (True, False):
        s = make_solver(w, prec)
        s.use_graphs(graphs)
        s.set_psi(psi0)
        states = []
        s.step_imag(16)                       # two replays of the imaginary-time graph
        states.append(s.get_psi())
        for _ in range(3):                    # three separate replays of the real-time graph
            s.step_real(8)
            states.append(s.get_psi())        # synchronises; eager copy kernel in between
            states.append(s.dipolar_potential())
        runs.append((states, s.history(40)))
        s.close()
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)
    assert runs[0][1] == runs[1][1]


@pytest.mark.parametrize("name", ["3d_24x20x16", "2dxy_48x40"])
def test_imag_then_real_graphs_match_oracle(name, gpu_lib):
    """Imaginary-time graphs leave a pending renormalisation factor (lazy scale); the
    real-time steps and graph replays that follow must apply it.  FP64 against the
    oracle, per-step records included."""
    w = CASES[name]
    banner("imag then real graphs", name)
    p = oparams(w)
    psi0 = start_state(w, 111)
    s = make_solver(w, "fp64")
    s.set_psi(psi0)
    s.step_imag(8)
    s.step_real(25)                           # 1 direct + 3 graph replays
    got = s.get_psi()
    recs = s.history(33)
    mid, hist_i = O.run(psi0, p, True, 8, record=True)
    ref, hist_r = O.run(mid, p, False, 25, record=True)
    assert_psi_close(got, ref, FP64_PSI_TOL)
    for k, (g_, r_) in enumerate(zip(recs, hist_i + hist_r)):
        bad = obs_close(g_, r_, FP64_E_TOL)
        assert not bad, (k, bad)
    s.close()


def test_timing_counts_launches(gpu_lib):
    w = CASES["3d_24x20x16"]
    banner("timing")
    s = make_solver(w, "fp32")
    s.set_psi(start_state(w, 108))
    s.timing_enable(["c2r_nl_cnx", "cn_z"])
    s.step_real(10)
    t = s.timing_read()
    assert t["c2r_nl_cnx"][1] == 10 and t["cn_z"][1] == 10 and t["r2c_x"][1] == 0
    assert t["c2r_nl_cnx"][0] > 0
    s.close()


def test_timing_burst(gpu_lib):
    """gp_timing_burst: positive per-launch time for the supported passes, argument and
    state errors otherwise; the state stays finite (real-time partial steps)."""
    from paper_1601_04640_amd import binding as B
    w = CASES["3d_24x20x16"]
    banner("timing burst")
    s = make_solver(w, "fp32")
    with pytest.raises(B.GPError) as e:
        s.timing_burst("c2r_nl_cnx", 4)
    assert e.value.status == B.GP_E_STATE
    s.set_psi(start_state(w, 109))
    for name in ("r2c_x", "c2r_nl_cnx", "cn_y", "cn_z"):
        assert s.timing_burst(name, 16) > 0
    for name, reps in (("fft_y_fwd", 4), ("c2r_nl_cnx", 0), ("c2r_nl_cnx", 5000)):
        with pytest.raises(B.GPError) as e:
            s.timing_burst(name, reps)
        assert e.value.status == B.GP_E_ARG
    assert np.all(np.isfinite(s.get_psi()))
    s.close()


def test_timing_span(gpu_lib):
    """gp_timing_span: one span per timed c2r launch inside steps, shorter than the event
    pair around the same launch; nothing recorded when the pass is not timed."""
    from paper_1601_04640_amd import binding as B
    w = CASES["3d_40x30x48"]
    banner("timing span")
    s = make_solver(w, "fp32")
    s.set_psi(start_state(w, 110))
    s.timing_enable(["c2r_nl_cnx"])
    s.step_real(10)
    ms, n = s.timing_span("c2r_nl_cnx")
    ev_ms, ev_n = s.timing_read()["c2r_nl_cnx"]
    assert n == 10 and ev_n == 10
    assert 0 < ms <= ev_ms
    s.timing_enable(["cn_z"])
    s.step_real(3)
    assert s.timing_span("c2r_nl_cnx") == (0.0, 0)
    with pytest.raises(B.GPError) as e:
        s.timing_span("cn_z")
    assert e.value.status == B.GP_E_ARG
    s.timing_enable([])
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["3d_24x20x16", "2dxy_48x40", "3d_16x64x512"])
def test_deferred_finalisation_bit_exact(name, prec, gpu_lib):
    """Steps fold each step's finalisation into the next step's first pass (two-stage on
    3d_16x64x512: first stage in the x pass, second in the forward y FFT), through
    graphs and direct launches, in imaginary time (which renormalises) and real time.
    With per-pass timing on, every step finalises in its own launch instead: psi, every
    history record and the energy are the same bit for bit, across the switches between
    the two time directions."""
    from paper_1601_04640_amd.binding import PASS_NAMES
    w = CASES[name]
    banner("deferred finalisation", name, prec)
    psi0 = start_state(w, 301)

    def run(timed):
        s = make_solver(w, prec)
        s.set_psi(psi0)
        if timed:
            s.timing_enable(list(PASS_NAMES))
        s.step_imag(11)
        h = s.history(11)
        s.step_real(19)
        h += s.history(19)
        s.step_imag(1)
        s.step_real(10)
        h += s.history(11)
        e = s.energy()
        psi = s.get_psi()
        s.close()
        return psi, h, e

    psi_a, h_a, e_a = run(False)
    psi_b, h_b, e_b = run(True)
    assert np.array_equal(psi_a, psi_b)
    assert len(h_a) == len(h_b) == 41
    for ra, rb in zip(h_a, h_b):
        assert ra == rb, (ra, rb)
    assert e_a == e_b
