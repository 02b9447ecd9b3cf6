"""Helpers shared by the GPU parity tests: oracle parameters from a workload dict, relative
errors, and a case banner printed (and flushed) before every GPU step."""
import sys

import numpy as np

import oracle as O

FP64_PSI_TOL = 1e-10     # rel-L2 of psi, FP64 mode
FP32_PSI_TOL = 2e-5      # rel-L2 of psi, FP32 mode (FP64 reductions)
FP64_E_TOL = 1e-12       # relative energy / mu, FP64 mode
FP32_E_TOL = 1e-6        # relative energy / mu, FP32 mode
# The stated energy bar applies to E and mu.  Their interaction parts e_int and e_dd are
# quartic in psi (sum |psi|^4, sum Phi |psi|^2): a relative amplitude error d of the FP32
# state enters them as about 4 d where E and mu see it diluted by the kinetic and trap
# parts, so the parts are held at four times the energy bar (a reading of the tolerance
# statement, which names the energy only).
FP32_PART_TOL = 4 * FP32_E_TOL


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


def obs_close(got, ref, tol, keys=("norm", "energy", "mu", "e_kin", "e_pot", "e_int", "e_dd"),
              part_tol=None):
    """Relative comparison of observables; part_tol (default tol) applies to e_int, e_dd."""
    bad = {}
    scale = max(abs(ref["energy"]), abs(ref["mu"]), 1.0)
    for k in keys:
        t = part_tol if (part_tol is not None and k in ("e_int", "e_dd")) else tol
        # each part is compared relative to the total energy scale (parts can be ~0)
        if abs(got[k] - ref[k]) > t * max(abs(ref[k]), scale * 1e-3):
            bad[k] = (got[k], ref[k])
    for a in range(3):
        if abs(got["rms"][a] - ref["rms"][a]) > tol * max(abs(ref["rms"][a]), 1e-3):
            bad[f"rms{a}"] = (got["rms"][a], ref["rms"][a])
    return bad
