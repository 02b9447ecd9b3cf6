"""Imaginary-time -> real-time hand-off through a saved state, with output every K steps.

The paper's real-time programs start from the stationary state an imaginary-time run
wrote to a file, and both kinds of run write the chemical potential, energy and rms sizes
(calcmuen, calcrms) and density profiles at chosen steps; only the wave function comes
back to the host, for output ("Summary of revisions").  This module strings the library's
calls together for that flow (argument marshalling and text formatting only: the steps,
the observables, the state files and the density run in the library):

  imaginary time: gp_set_psi, gp_evolve (records every K steps), gp_save_state,
                  gp_save_density
  real time:      gp_load_state into a context with the real-time parameters (dt, a
                  quenched coupling, another precision), gp_evolve (records every K steps,
                  a density file at each record), gp_save_state

Outputs in `outdir`: imag-obs.txt / real-obs.txt (one row per record: step, time, norm,
mu, energy, e_kin, e_pot, e_int, e_dd, rms_x, rms_y, rms_z), imag-psi.gpd, imag-den.gpd,
real-den-<step>.gpd (when density_every > 0) and real-psi.gpd, in the state-file layout
of include/gp.h.
"""
from __future__ import annotations

import os

from .binding import Solver

COLUMNS = ("step", "time", "norm", "mu", "energy", "e_kin", "e_pot", "e_int", "e_dd",
           "rms_x", "rms_y", "rms_z")


def _row(step, dt, ob):
    return [step, step * dt, ob["norm"], ob["mu"], ob["energy"], ob["e_kin"], ob["e_pot"],
            ob["e_int"], ob["e_dd"], *ob["rms"]]


def write_table(path, rows, title):
    with open(path, "w") as f:
        f.write(f"# {title}\n# " + " ".join(COLUMNS) + "\n")
        for r in rows:
            f.write(f"{r[0]:d} " + " ".join(f"{v:.17e}" for v in r[1:]) + "\n")


def read_table(path):
    rows = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = line.split()
            rows.append([int(v[0])] + [float(x) for x in v[1:]])
    return rows


def imaginary_run(params, psi0, nsteps, every, outdir, prec="fp64"):
    """Relax psi0 for nsteps imaginary-time steps; writes imag-obs.txt, imag-psi.gpd and
    imag-den.gpd.  Returns the records (rows)."""
    os.makedirs(outdir, exist_ok=True)
    s = Solver(params, prec=prec)
    try:
        s.set_psi(psi0)
        rows = []
        s.evolve(True, nsteps, every, lambda k, ob: rows.append(_row(k, params["dt"], ob)))
        write_table(os.path.join(outdir, "imag-obs.txt"), rows,
                    f"imaginary time, dt {params['dt']}, {nsteps} steps, {prec}")
        t = nsteps * params["dt"]
        s.save_state(os.path.join(outdir, "imag-psi.gpd"), nsteps, t)
        s.save_density(os.path.join(outdir, "imag-den.gpd"), nsteps, t)
    finally:
        s.close()
    return rows


def real_run(params, nsteps, every, outdir, prec="fp64", state=None, density_every=0):
    """Real-time run from a saved state (default: outdir/imag-psi.gpd) with the real-time
    parameters `params`; records every `every` steps in real-obs.txt, a density file at
    every record whose step is a multiple of density_every (> 0), and the final state in
    real-psi.gpd.  Returns the records."""
    os.makedirs(outdir, exist_ok=True)
    s = Solver(params, prec=prec)
    try:
        s.load_state(state or os.path.join(outdir, "imag-psi.gpd"))
        rows = []

        def out(k, ob):
            rows.append(_row(k, params["dt"], ob))
            if density_every > 0 and k % density_every == 0:
                s.save_density(os.path.join(outdir, f"real-den-{k:06d}.gpd"), k, k * params["dt"])

        s.evolve(False, nsteps, every, out)
        write_table(os.path.join(outdir, "real-obs.txt"), rows,
                    f"real time, dt {params['dt']}, {nsteps} steps, {prec}")
        s.save_state(os.path.join(outdir, "real-psi.gpd"), nsteps, nsteps * params["dt"])
    finally:
        s.close()
    return rows
