"""Helpers shared by the GPU parity tests: oracle parameters from a workload dict, relative
errors, and a case banner printed (and flushed) before every GPU step."""
import sys

import numpy as np

import oracle as O

FP64_PSI_TOL = 1e-10     # rel-L2 of psi, FP64 mode
FP32_PSI_TOL = 2e-5      # rel-L2 of psi, FP32 mode (FP64 reductions)
FP64_E_TOL = 1e-12       # relative energy / mu, FP64 mode
FP32_E_TOL = 1e-6        # relative energy / mu, FP32 mode


def banner(*parts):
    print("[gpu case]", *parts, flush=True)
    sys.stdout.flush()


def oparams(w):
    keys = ("geom", "nx", "ny", "nz", "dx", "dy", "dz", "dt", "gamma", "nu", "lam", "g", "gdd", "R")
    return O.Params(**{k: w[k] for k in keys if k in w})


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def psi_errors(got, ref):
    """(rel-L2, element-wise max |got - ref| / max |ref|) of two wave functions."""
    got = np.asarray(got).ravel()
    ref = np.asarray(ref).ravel()
    return rel_l2(got, ref), float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def assert_psi_close(got, ref, tol, what=""):
    """Both the relative L2 error and the largest element-wise error (relative to the
    largest |ref|) within tol: a wrong tile where the state is small cannot hide in the
    global norm."""
    l2, mx = psi_errors(got, ref)
    assert l2 <= tol and mx <= tol, (what, l2, mx, tol)
    return l2, mx


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def energy_scale(ob):
    """Magnitude of the terms of the energy functional, |e_kin| + |e_pot| + |e_int| + |e_dd|."""
    return abs(ob["e_kin"]) + abs(ob["e_pot"]) + abs(ob["e_int"]) + abs(ob["e_dd"])


def obs_close(got, ref, tol, keys=("norm", "energy", "mu", "e_kin", "e_pot", "e_int", "e_dd"),
              per_particle=False):
    """Observables against reference values.  The stated bar is relative on the energy.
    The chemical potential and the parts (kinetic, trap, contact, dipolar) are sums of the
    energy functional's terms, so they are held at the same bar relative to the larger of
    their own size and the energy scale S = |e_kin| + |e_pot| + |e_int| + |e_dd|: a part's
    error enters E and mu one to one (twice for the interaction parts in mu), and a bar
    relative to mu alone is ill-conditioned where the interaction terms cancel the rest.
    per_particle: E, mu and the parts of each state are divided by its norm first, and the
    norm itself is left to a separate conservation check (long FP32 real-time runs, whose
    norm drifts by rounding while the exact evolution conserves it).
    The rms sizes are moments of |psi|^2, first order in the state's error: for a
    Gaussian-like cloud d(rms)/rms <= about sqrt(3) ||d psi||/||psi||, so they are held at
    the psi bar of the same precision (1e-10 FP64, 2e-5 FP32)."""
    bad = {}
    rms_tol = {FP64_E_TOL: FP64_PSI_TOL, FP32_E_TOL: FP32_PSI_TOL}.get(tol, tol)
    gn = got["norm"] if per_particle else 1.0
    rn = ref["norm"] if per_particle else 1.0
    scale = energy_scale(ref) / rn
    for k in keys:
        if k == "norm":
            if not per_particle and abs(got[k] - ref[k]) > tol * abs(ref[k]):
                bad[k] = (got[k], ref[k])
            continue
        g_, r_ = got[k] / gn, ref[k] / rn
        den = abs(r_) if k == "energy" else max(abs(r_), scale)
        if abs(g_ - r_) > tol * max(den, 1e-300):
            bad[k] = (got[k], ref[k])
    for a in range(3):
        if abs(got["rms"][a] - ref["rms"][a]) > rms_tol * max(abs(ref["rms"][a]), 1e-3):
            bad[f"rms{a}"] = (got["rms"][a], ref["rms"][a])
    return bad
