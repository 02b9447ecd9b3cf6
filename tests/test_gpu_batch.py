"""Batched ensemble (one persistent launch per pass and size class) against the FP64
oracle per instance and against each instance run alone through the single-grid path."""
import numpy as np
import pytest

import oracle as O
from paper_1601_04640_amd import inputs as I
from tests.gpu_util import (FP32_E_TOL, FP32_PSI_TOL, FP64_E_TOL, FP64_PSI_TOL,
                            assert_psi_close, banner, obs_close, oparams, rel_l2)

pytestmark = pytest.mark.gpu


def small_ensemble(count=12, seed=77):
    """Mixed XY/XZ instances, sizes from {32, 48, 64, 96} (both classes: 384 added once)."""
    return I.batched_ensemble(count=count, seed=seed, sizes=(32, 48, 64, 96))


def start(w, i):
    return I.psi0_instance(w, seed=[1606, i])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_oracle_per_instance(prec, gpu_lib):
    from paper_1601_04640_amd.binding import Batch
    ens = small_ensemble()
    ens[3] = dict(ens[3], nx=384)            # one large-class x axis
    banner("batch vs oracle", prec, len(ens))
    b = Batch(ens, prec=prec)
    psis = [start(w, i) for i, w in enumerate(ens)]
    for i, p in enumerate(psis):
        b.set_psi(i, p)
    b.step_imag(12)
    b.step_real(9)
    tol = FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL
    energies = b.energy()
    for i, w in enumerate(ens):
        p = oparams(w)
        ref = O.run(O.run(psis[i], p, True, 12), p, False, 9)
        assert_psi_close(b.get_psi(i), ref, tol, (i, w["geom"], w["nx"]))
        if prec == "fp64":
            bad = obs_close(energies[i], O.observables(ref, p), FP64_E_TOL)
        else:
            bad = obs_close(energies[i], O.observables(ref, p), FP32_E_TOL)
        assert not bad, (i, bad)
    b.close()


SAME_PATH_TOL = 1e-6  # same tile bodies and partial-sum order; allows for contraction choices


def test_batch_equals_single_grid_path(gpu_lib):
    """Same tile bodies, same partial-sum order as running each instance alone."""
    from paper_1601_04640_amd.binding import Batch, Solver
    ens = small_ensemble(count=6, seed=78)
    banner("batch vs single path")
    b = Batch(ens, prec="fp32")
    for i, w in enumerate(ens):
        b.set_psi(i, start(w, i))
    b.step_imag(10)
    for i, w in enumerate(ens):
        s = Solver(w, prec="fp32")
        s.set_psi(start(w, i))
        s.step_imag(10)
        a, c = s.get_psi(), b.get_psi(i)
        print("instance", i, "bitwise" if np.array_equal(a, c) else f"rel {rel_l2(c, a):.2e}")
        assert rel_l2(c, a) <= SAME_PATH_TOL, i
        for ha, hb in zip(s.history(10), b.history(i, 10)):
            assert abs(ha["energy"] - hb["energy"]) <= SAME_PATH_TOL * abs(ha["energy"])
        s.close()
    b.close()


@pytest.mark.parametrize("shape", [("2dxy", 48, 64), ("2dxz", 384, 32)])
def test_single_instance_batch(shape, gpu_lib):
    """An ensemble of one instance (each pass then has a single size class, and the
    384-point x axis puts the x passes in the large class alone) against the oracle."""
    from paper_1601_04640_amd.binding import Batch
    geom, nx, n1 = shape
    w = small_ensemble(count=2, seed=80)[0 if geom == "2dxy" else 1]
    w = dict(w, nx=nx, **({"ny": n1} if geom == "2dxy" else {"nz": n1}))
    banner("single-instance batch", geom, nx, n1)
    b = Batch([w], prec="fp64")
    psi0 = start(w, 0)
    b.set_psi(0, psi0)
    b.step_imag(6)
    b.step_real(5)
    p = oparams(w)
    ref = O.run(O.run(psi0, p, True, 6), p, False, 5)
    assert_psi_close(b.get_psi(0), ref, FP64_PSI_TOL)
    assert not obs_close(b.energy()[0], O.observables(ref, p), FP64_E_TOL)
    b.close()


def test_full_ensemble_sampled(gpu_lib):
    """The 192-instance ensemble (sizes 96..512): a few steps; sampled instances against
    the single-grid path (bitwise) and the oracle (FP32 tolerance)."""
    from paper_1601_04640_amd.binding import Batch, Solver
    ens = I.batched_ensemble()
    banner("full ensemble", len(ens))
    b = Batch(ens, prec="fp32")
    for i, w in enumerate(ens):
        b.set_psi(i, start(w, i))
    b.step_imag(8)
    rng = np.random.default_rng(5)
    for i in rng.choice(len(ens), size=4, replace=False):
        i = int(i)
        w = ens[i]
        s = Solver(w, prec="fp32")
        s.set_psi(start(w, i))
        s.step_imag(8)
        assert rel_l2(b.get_psi(i), s.get_psi()) <= SAME_PATH_TOL, i
        s.close()
        ref = O.run(start(w, i), oparams(w), True, 8)
        assert_psi_close(b.get_psi(i), ref, FP32_PSI_TOL, i)
    b.close()


def test_autotuner_keeps_results(tmp_path, gpu_lib):
    from paper_1601_04640_amd import autotune
    from paper_1601_04640_amd.binding import Batch
    ens = small_ensemble(count=8, seed=79)
    banner("autotune")
    b = Batch(ens, prec="fp32")
    for i, w in enumerate(ens):
        b.set_psi(i, start(w, i))
    b.step_imag(8)
    ref = [b.get_psi(i) for i in range(len(ens))]
    plan = autotune.tune(b, steps=8, cache_path=str(tmp_path / "tune.json"))
    assert plan and all(v["blocks"] >= 1 and v["shape"] in (0, 1) for v in plan.values())
    assert (tmp_path / "tune.json").exists()
    b.close()
    # the cached plan is applied as it was chosen; block counts change only which block
    # runs a tile, so with the default shapes the results are bitwise those of the default
    # plan, and with the tuned shapes they stay at the FP32 bars against the oracle
    b2 = Batch(ens, prec="fp32")
    autotune.tune(b2, steps=8, cache_path=str(tmp_path / "tune.json"))  # cached plan
    assert {f"{p}:{c}": v for (p, c), v in b2.tile_shapes().items()
            if f"{p}:{c}" in plan} == {k: v["shape"] for k, v in plan.items()}
    for i, w in enumerate(ens):
        b2.set_psi(i, start(w, i))
    b2.step_imag(8)
    for i, w in enumerate(ens):
        assert_psi_close(b2.get_psi(i), O.run(start(w, i), oparams(w), True, 8),
                         FP32_PSI_TOL, i)
    for (p, c) in b2.tile_shapes():
        b2.set_shape(p, c, 0)
    for i, w in enumerate(ens):
        b2.set_psi(i, start(w, i))
    b2.step_imag(8)
    for i in range(len(ens)):
        assert np.array_equal(b2.get_psi(i), ref[i])
    b2.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tile_shapes_match_oracle(prec, gpu_lib):
    """Every pass and class with the alternative tile shape (8-line x and column tiles,
    twice the line-FFT block), imaginary and real time, against the oracle; the energies
    and per-instance records through the batch finalisation."""
    from paper_1601_04640_amd.binding import Batch
    ens = small_ensemble(count=6, seed=83)
    ens[1] = dict(ens[1], nx=384)            # a class-1 x axis
    banner("batch tile shapes", prec)
    b = Batch(ens, prec=prec)
    for (p, c) in b.tile_shapes():
        b.set_shape(p, c, 1)
    assert set(b.tile_shapes().values()) == {1}
    for i, w in enumerate(ens):
        b.set_psi(i, start(w, i))
    b.step_imag(9)
    b.step_real(7)
    tol = FP64_PSI_TOL if prec == "fp64" else FP32_PSI_TOL
    etol = FP64_E_TOL if prec == "fp64" else FP32_E_TOL
    energies = b.energy()
    for i, w in enumerate(ens):
        p = oparams(w)
        ref = O.run(O.run(start(w, i), p, True, 9), p, False, 7)
        assert_psi_close(b.get_psi(i), ref, tol, i)
        assert not obs_close(energies[i], O.observables(ref, p), etol), i
        # the record of the state the last step started from, reduced by the batch
        rec = b.history(i, 16)[-1]
        prev = O.run(O.run(start(w, i), p, True, 9), p, False, 6)
        assert not obs_close(rec, O.observables(prev, p), etol), i
    b.close()


def test_batch_rejects_bad_params(gpu_lib):
    from paper_1601_04640_amd import binding as B
    banner("batch errors")
    ens = small_ensemble(count=3)
    with pytest.raises(B.GPError) as e:
        B.Batch([dict(ens[0], nx=80)] + ens[1:])
    assert e.value.status == B.GP_E_SIZE
    with pytest.raises(B.GPError) as e:
        B.Batch([dict(geom="3d", nx=32, ny=32, nz=32)])
    assert e.value.status == B.GP_E_ARG
    b = B.Batch(ens)
    with pytest.raises(B.GPError) as e:
        b.step_imag(1)
    assert e.value.status == B.GP_E_STATE
    b.close()


def test_batch_state_io_and_streams(gpu_lib):
    """gp_batch_set_psi / gp_batch_get_psi address the instances by index (out of range:
    GP_E_ARG); an instance context stepped on its own is brought up to date by the next
    batch step; the two-stream launch order gives bitwise the same results as one
    stream."""
    from paper_1601_04640_amd import binding as B
    from paper_1601_04640_amd.binding import Batch
    ens = small_ensemble(count=5, seed=81)
    ens[2] = dict(ens[2], nx=384)            # both size classes present
    banner("batch io / streams")
    runs = []
    for streams in (False, True):
        b = Batch(ens, prec="fp64")
        b.use_streams(streams)
        for i, w in enumerate(ens):
            b.set_psi(i, start(w, i))
        B.gp_step_imag(b.ctxs[1], 3)           # instance 1 alone: leaves a deferred step
        b.step_imag(9)
        runs.append([b.get_psi(i) for i in range(len(ens))])
        for bad in (-1, len(ens)):
            with pytest.raises(B.GPError) as e:
                b.get_psi(bad)
            assert e.value.status == B.GP_E_ARG
        b.close()
    for a, c in zip(*runs):
        assert np.array_equal(a, c)
    for i, w in enumerate(ens):
        p = oparams(w)
        ref = O.run(start(w, i), p, True, 12 if i == 1 else 9)
        assert_psi_close(runs[0][i], ref, FP64_PSI_TOL, i)
