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


def obs_close(got, ref, tol, keys=("norm", "energy", "mu", "e_kin", "e_pot", "e_int", "e_dd")):
    """Observables against reference values.  The stated bar is relative on the energy and
    the chemical potential.  Their parts (kinetic, trap, contact, dipolar) are the terms of
    those sums, so each is held at the same bar relative to the larger of its own size and
    the scale of the sums, max(|E|, |mu|): a part's error enters E or mu one to one."""
    bad = {}
    scale = max(abs(ref["energy"]), abs(ref["mu"]))
    for k in keys:
        ref_k = abs(ref[k])
        if k in ("e_kin", "e_pot", "e_int", "e_dd"):
            ref_k = max(ref_k, scale)
        if abs(got[k] - ref[k]) > tol * max(ref_k, 1e-300):
            bad[k] = (got[k], ref[k])
    for a in range(3):
        if abs(got["rms"][a] - ref["rms"][a]) > tol * max(abs(ref["rms"][a]), 1e-3):
            bad[f"rms{a}"] = (got["rms"][a], ref["rms"][a])
    return bad
