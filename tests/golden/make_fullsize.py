"""Writes the full-size expected values used by tests/test_gpu_fullsize.py.

Every value here comes from the FP64 oracle (`oracle/`) on the seeded inputs of
`paper_1601_04640_amd/inputs.py`; nothing is read from the GPU path.

  imag3d_64_500.json      64^3, dx 0.25, dt 0.002, trap (1,1,2), g 20, g_dd 6, R 8:
                          500 imaginary-time steps from the seeded anisotropic Gaussian.
                          Stores the observables of the final state, the per-step
                          energy / mu records, and psi at 512 seeded sample points.
  ensemble_imag_1000.json 1000 imaginary-time steps (dt 0.001) of six instances of the
                          192-instance quasi-2D ensemble (the four smallest grids and the
                          two smallest with a 384/512 axis): final observables and psi at
                          256 seeded sample points each.

Usage: python tests/golden/make_fullsize.py   (about two minutes, one process)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1601_04640_amd import inputs as I  # noqa: E402

KEYS = ("geom", "nx", "ny", "nz", "dx", "dy", "dz", "dt", "gamma", "nu", "lam", "g", "gdd", "R")


def params(w):
    return O.Params(**{k: w[k] for k in KEYS})


def sample_indices(shape, count, seed):
    """Flat indices of `count` distinct interior points (PCG64, `seed`)."""
    rng = np.random.default_rng(seed)
    interior = np.ones(shape, dtype=bool)
    for ax in range(len(shape)):
        idx = [slice(None)] * len(shape)
        idx[ax] = 0
        interior[tuple(idx)] = False
        idx[ax] = -1
        interior[tuple(idx)] = False
    flat = np.flatnonzero(interior.ravel())
    return np.sort(rng.choice(flat, size=count, replace=False))


def obs_json(o):
    return {k: (list(map(float, v)) if k == "rms" else float(v)) for k, v in o.items()}


def imag3d_64():
    w = I.WORKLOADS["imag3d_64"]
    p = params(w)
    psi0 = I.psi0_imag3d_64()
    t0 = time.time()
    psi, hist = O.run(psi0, p, True, w["steps"], record=True)
    final = O.observables(psi, p)
    idx = sample_indices(psi.shape, 512, 7001)
    out = {
        "workload": "imag3d_64", "steps": w["steps"], "params": {k: w[k] for k in KEYS},
        "psi0": "inputs.psi0_imag3d_64(seed=1601)",
        "final": obs_json(final),
        "history_energy": [float(h["energy"]) for h in hist],
        "history_mu": [float(h["mu"]) for h in hist],
        "sample_index": idx.tolist(),
        "psi_re": psi.ravel()[idx].real.tolist(),
        "psi_im": psi.ravel()[idx].imag.tolist(),
    }
    print(f"imag3d_64: {time.time() - t0:.1f} s, E = {final['energy']:.12f}", flush=True)
    return out


def pick_instances(ens):
    area = [(w["nx"] * (w["ny"] if w["geom"] == "2dxy" else w["nz"]), i) for i, w in enumerate(ens)]
    area.sort()
    small = [i for _, i in area[:4]]
    big = [i for _, i in area
           if max(ens[i]["nx"], ens[i]["ny"] if ens[i]["geom"] == "2dxy" else ens[i]["nz"]) > 256]
    return small + big[:2]


def ensemble():
    ens = I.batched_ensemble()
    picks = pick_instances(ens)
    recs = []
    for i in picks:
        w = ens[i]
        p = params(w)
        t0 = time.time()
        psi = O.run(I.psi0_instance(w, seed=[1606, i]), p, True, 1000)
        o = O.observables(psi, p)
        idx = sample_indices(psi.shape, 256, 7002 + i)
        recs.append({"index": i, "params": {k: w[k] for k in KEYS}, "final": obs_json(o),
                     "sample_index": idx.tolist(),
                     "psi_re": psi.ravel()[idx].real.tolist(),
                     "psi_im": psi.ravel()[idx].imag.tolist()})
        print(f"instance {i} {w['geom']} {psi.shape}: {time.time() - t0:.1f} s", flush=True)
    return {"ensemble": "inputs.batched_ensemble(count=192, seed=1606)",
            "psi0": "inputs.psi0_instance(w, seed=[1606, i])", "steps": 1000,
            "instances": recs}


def main():
    with open(os.path.join(HERE, "imag3d_64_500.json"), "w") as f:
        json.dump(imag3d_64(), f)
    with open(os.path.join(HERE, "ensemble_imag_1000.json"), "w") as f:
        json.dump(ensemble(), f)


if __name__ == "__main__":
    main()
