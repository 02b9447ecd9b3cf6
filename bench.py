#!/usr/bin/env python3
"""Benchmark: grid-point-steps/s of one full split-step Crank-Nicolson step of the 3D
dipolar GP equation on one MI355X.

Headline: the large real-time workload, 256^3 (dx 0.1, dt 0.0005, g 50, g_dd 25, trap
(1,1,3), R 12.8) in FP64, the precision of the paper's programs; the FP32 mode (FP32 bulk
arithmetic, FP64 reductions) is timed beside it, and both are paired with their error
against the FP64 oracle (500 steps, oracle-written fixture) and against each other.  The
dominant pass's HBM roofline is measured live; the FP64 CPU oracle is timed on the host
cores (one thread, and one process per core) on a bounded sample of the same workload.
The other workloads (the 128x96x80 quench, the 64^3 imaginary-time run, the 192-instance
quasi-2D ensemble, the 128^3 adjoint) are reported beside the headline.

Each timed step runs every pass of the hot path: |psi|^2 -> R2C -> y/z FFT, U(k)
product, inverse -> C2R -> nonlinear phase -> CN sweeps x, y, z -> FP64 norm / energy /
mu / rms reductions.  Inputs are resident in HBM before the timed region starts, and the
step graphs are captured before it.

Prints ONE JSON line (or one per grid with --sweep).
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
       python bench.py --sweep [--sweep-dims 3 2] [--sweep-prec fp32 fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid-point-steps/s (3D dipolar CN step), %HBM peak, FP32 vs FP64 at stated err"
WORKLOAD = "real3d_256"
DOMINANT = "c2r_nl_cnx"
GRAPH_STEPS = 8          # steps per captured graph in the library
KEYS = ("geom", "nx", "ny", "nz", "dx", "dy", "dz", "dt", "gamma", "nu", "lam", "g", "gdd", "R")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pass_bytes(name, npts, nspec, esz, ktab=0):
    """Algorithmic HBM bytes of one launch of a pass: each input read once, each output
    written once (complex values are 2*esz bytes; ktab = kernel-table values read)."""
    c = 2 * esz
    return {
        "r2c_x": npts * c + nspec * c,
        "fft_y_fwd": 2 * nspec * c,
        "conv_z": 2 * nspec * c + ktab * esz,
        "fft_y_inv": 2 * nspec * c,
        "c2r_nl_cnx": nspec * c + npts * c + npts * esz + npts * c,
        "cn_y": 2 * npts * c,
        "cn_z": 2 * npts * c,
    }[name]


def step_bytes_3d(n0, n1, n2, esz):
    """Algorithmic bytes of one 3D step (pencil model): the sum over the seven passes."""
    npts = n0 * n1 * n2
    nspec = (n0 // 2 + 1) * n1 * n2
    ktab = (n0 // 2 + 1) * (n1 // 2 + 1) * (n2 // 2 + 1)
    return sum(pass_bytes(p, npts, nspec, esz, ktab) for p in
               ("r2c_x", "fft_y_fwd", "conv_z", "fft_y_inv", "c2r_nl_cnx", "cn_y", "cn_z"))


def step_bytes_2d(n0, n1, esz):
    """Algorithmic HBM bytes of one quasi-2D step (r2c, y convolution, c2r + phase + CN x,
    CN y), each pass reading its inputs once and writing its outputs once."""
    npts = n0 * n1
    nspec = (n0 // 2 + 1) * n1
    c = 2 * esz
    return ((npts * c + nspec * c) + (2 * nspec * c + nspec * esz)
            + (nspec * c + npts * c + npts * esz + npts * c) + 2 * npts * c)


def read_traffic(kernel, workload, prec):
    """Counter-measured HBM bytes per launch from a committed rocprofv3 PMC summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}_{prec}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    from paper_1601_04640_amd.profile_run import kernel_hash
    if kv.get("kernel_source_hash") != kernel_hash():
        return None
    try:
        fetch = float(kv["FETCH_SIZE_KiB_per_dispatch"]) * float(kv["fetch_scale"])
        write = float(kv["WRITE_SIZE_KiB_per_dispatch"]) * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0


# ------------------------------------------------------------------- CPU oracle
def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_CPU = {}


def _oracle_setup():
    import oracle as O
    from paper_1601_04640_amd import inputs as I
    w = I.WORKLOADS[WORKLOAD]
    p = O.Params(**{k: w[k] for k in KEYS})
    _CPU.update(p=p, psi=I.psi0_real3d_256(), V=O.harmonic_potential(p),
                K=O.dipolar_kernel(p), npts=w["nx"] * w["ny"] * w["nz"])


def _oracle_steps(budget_s, min_steps=2):
    """Real-time steps of the oracle (step + the step's observables) for about
    budget_s seconds in this process, one thread: (steps, seconds)."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    p, psi, V, K = _CPU["p"], _CPU["psi"], _CPU["V"], _CPU["K"]
    n = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            O.observables(psi, p, V=V, kernel=K)      # the step's reductions
            psi = O.step(psi, p, False, V=V, kernel=K)
            n += 1
            el = time.perf_counter() - t0
            if n >= min_steps and el > budget_s:
                break
    return n, el


def _worker(budget_s):
    return _oracle_steps(budget_s)


def cpu_baseline(budget_s=15.0):
    """The FP64 oracle (as is: numpy/scipy, one thread per process) on the headline
    workload, 256^3 real time, on this machine's host cores, in two legs: one thread
    (the paper's single-core comparison) and one process per available core, each
    stepping its own copy of the same state (aggregate throughput).  Runs before the
    GPU is touched (the all-core leg forks)."""
    import multiprocessing as mp
    _oracle_setup()
    npts = _CPU["npts"]
    n1, el1 = _oracle_steps(budget_s)
    one = npts * n1 / el1
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(int(cores or 1), 16))
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_worker, [budget_s] * cores)
    allv = sum(npts * n / el for n, el in res)
    steps = [n for n, _ in res]
    return {"value": allv, "unit": "grid-point-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{WORKLOAD} real-time steps (step + observables, FP64 numpy/scipy "
                      f"oracle) for about {budget_s:.0f} s: {cores} processes of one thread "
                      f"each on {cores} host cores ({min(steps)}-{max(steps)} steps each), "
                      f"aggregate pt-steps/s",
            "cpu_model": _cpu_model(),
            "one_thread": {"value": one, "steps": n1, "seconds": round(el1, 2), "cores": 1},
            "all_cores": {"value": allv, "processes": cores, "threads_per_process": 1}}


# ------------------------------------------------------------------------ GPU
def time_gpu(workload, prec, psi_start, steps, warmup, solver_params=None, host=()):
    """Two live timed regions of `steps` full steps from the same start, on the solver's
    stream: (1) steps replayed from captured HIP graphs, no instrumentation -> value;
    (2) the same steps launched directly with the dominant pass's launches timed by their
    own dispatch timestamps -> its mean launch time for the roofline.  Before timing, the
    warm-up runs max(warmup, GRAPH_STEPS + 1) steps and then the timed call once, so every
    graph the timed call replays is captured outside the timed region."""
    import torch
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Solver
    w = solver_params or I.WORKLOADS[workload]
    s = Solver(w, prec=prec, host=host)
    # the start state is kept on the device: resetting it between runs is a device copy,
    # so the GPU does not sit idle (and clock down) behind a host transfer just before a
    # timed region
    psi_dev = (psi_start.to(s.device, s.cdtype) if torch.is_tensor(psi_start)
               else torch.from_numpy(psi_start).to(s.device, s.cdtype))
    s.set_psi(psi_dev)
    s.step_real(max(warmup, GRAPH_STEPS + 1))
    s.set_psi(psi_dev)
    s.step_real(steps)
    s.sync()
    res = {}
    for region in ("graph", "events"):
        s.set_psi(psi_dev)                   # every timed run starts afresh
        if region == "events":
            s.timing_enable([DOMINANT])
        else:
            s.timing_enable([])
            s.use_graphs(True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(s.stream)
        s.step_real(steps)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res[region] = dict(wall=wall, gpu_ms=ev0.elapsed_time(ev1))
        if region == "events":
            res["timing"] = s.timing_read()
            res["span"] = s.timing_span(DOMINANT)
            s.timing_enable([])
        else:
            res["hist"] = s.history(steps)
    res["npts"] = w["nx"] * w["ny"] * w["nz"]
    res["nspec"] = (w["nx"] // 2 + 1) * w["ny"] * w["nz"]
    res["dims"] = (w["nx"], w["ny"], w["nz"])
    s.close()
    return res


def roofline(r, esz):
    """Dominant pass: algorithmic bytes per launch / mean launch duration over the timed
    steps.  Each launch of the pass is timed by HIP events that the launch itself fills
    from its dispatch start/end timestamps (hipExtLaunchKernelGGL, on the solver's
    stream); the blocks' own wall-clock span (first start to last end) is reported beside
    it."""
    tot_ms, nl = r["timing"][DOMINANT]
    avg_ms = tot_ms / max(nl, 1)
    span_ms, ns = r["span"]
    alg = pass_bytes(DOMINANT, r["npts"], r["nspec"], esz)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": DOMINANT,
            "avg_launch_ms": round(avg_ms, 5), "launches": nl,
            "avg_block_span_ms": round(span_ms / max(ns, 1), 5),
            "algorithmic_bytes_per_launch": alg}


def summary(r, steps, esz):
    n0, n1, n2 = r["dims"]
    wall = r["graph"]["wall"]
    byts = step_bytes_3d(n0, n1, n2, esz)
    return {"value": r["npts"] * steps / wall, "ms_per_step": wall * 1e3 / steps,
            "gpu_event_ms_per_step": r["graph"]["gpu_ms"] / steps,
            "step_algorithmic_bytes": byts,
            "step_hbm_frac": round(byts / (wall / steps) / 1e9 / HBM_PEAK_GBS, 4)}


def accuracy_256():
    """FP64 and FP32 runs of the headline workload, 500 steps from its seeded start,
    against the oracle's fixture of the same run (psi at 4096 sampled points, final
    energy), and FP32 against FP64 on the whole grid."""
    import numpy as np
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Solver
    path = os.path.join(ROOT, "tests", "golden", "real3d_256_500.json")
    if not os.path.exists(path):
        return {"note": "oracle fixture missing: run tests/golden/make_fullsize.py real3d_256"}
    with open(path) as f:
        g = json.load(f)
    idx = np.asarray(g["sample_index"])
    ref = np.asarray(g["psi_re"]) + 1j * np.asarray(g["psi_im"])
    psi0 = I.psi0_real3d_256()
    out, psis = {}, {}
    for prec in ("fp64", "fp32"):
        s = Solver(I.WORKLOADS[WORKLOAD], prec=prec)
        s.set_psi(psi0)
        s.step_real(g["steps"])
        psi = s.get_psi()
        e = s.energy()["energy"]
        s.close()
        got = psi.ravel()[idx]
        out[prec] = {"psi_rel_l2_vs_oracle": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                     "psi_max_rel_vs_oracle": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))),
                     "energy_rel_vs_oracle": abs(e - g["final"]["energy"]) / abs(g["final"]["energy"])}
        psis[prec] = psi
    out["fp32_vs_fp64_psi_rel_l2"] = float(np.linalg.norm(psis["fp32"] - psis["fp64"]) /
                                           np.linalg.norm(psis["fp64"]))
    out["steps"] = g["steps"]
    out["note"] = ("oracle: FP64 numpy/scipy, psi at 4096 sampled points and the final "
                   "energy after the same 500 steps (tests/golden/real3d_256_500.json)")
    return out


def quench_128x96x80(steps, warmup):
    """The 128x96x80 quench (from the FP64 imaginary-time ground state at g = 20, then
    g = 15) in FP32 and FP64."""
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Solver
    w = dict(I.WORKLOADS["real3d_128x96x80"])
    gs = Solver(dict(w, g=w["g_ground"], dt=0.002), prec="fp64")
    gs.set_psi(I.psi0_real3d_128x96x80())
    gs.step_imag(1500)
    psi_g = gs.get_psi()
    gs.close()
    out = {}
    for prec, esz in (("fp32", 4), ("fp64", 8)):
        r = time_gpu("real3d_128x96x80", prec, psi_g, steps, warmup)
        out[prec] = dict(summary(r, steps, esz), roofline=dict(
            roofline(r, esz), traffic=read_traffic(DOMINANT, "real3d_128x96x80", prec)))
    return out


def host_resident_256(steps, warmup):
    """The headline workload with the trap potential and the dipolar kernel table in
    pinned host memory (read over the host link every step), FP32 and FP64: step time and
    the device memory it saves."""
    from paper_1601_04640_amd import binding as B
    from paper_1601_04640_amd import inputs as I
    psi5 = I.psi0_real3d_256()
    out = {}
    for prec in ("fp32", "fp64"):
        r = time_gpu(WORKLOAD, prec, psi5, steps, warmup, host=("V", "ktab"))
        prm = B.make_params(**{**I.WORKLOADS[WORKLOAD], "prec": prec})
        out[prec] = {"ms_per_step": r["graph"]["wall"] * 1e3 / steps,
                     "value": r["npts"] * steps / r["graph"]["wall"],
                     "workspace_bytes": B.gp_workspace_bytes_ex(prm, B.GP_HOST_V | B.GP_HOST_KTAB),
                     "workspace_bytes_resident": B.gp_workspace_bytes(prm)}
    out["note"] = "V and the kernel table in pinned host memory (gp_init_ex), 256^3 real time"
    return out


def imag3d_64(steps):
    """The 64^3 imaginary-time workload (FP64): graph-replayed steps from its start."""
    import torch
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Solver
    w = I.WORKLOADS["imag3d_64"]
    s = Solver(w, prec="fp64")
    psi0 = torch.from_numpy(I.psi0_imag3d_64()).to(s.device)   # reset by a device copy
    s.set_psi(psi0)
    s.step_imag(steps)
    s.set_psi(psi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_imag(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    npts = 64 ** 3
    return {"value": npts * steps / wall, "ms_per_step": wall * 1e3 / steps, "dtype": "f64",
            "steps": steps}


def time_batch(steps, tune_steps=16, two_streams=False):
    """The 192-instance quasi-2D ensemble (sizes from {96..512}^2, mixed XY/XZ), FP32 with
    FP64 reductions, imaginary time: the default launch plan, the autotuned plan, and the
    autotuned plan with the two size classes on two streams; each timed region runs
    `steps` steps from the same seeded start (graph replay, captured beforehand)."""
    import torch
    from paper_1601_04640_amd import autotune
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Batch
    ens = I.batched_ensemble()
    b = Batch(ens, prec="fp32")
    # start states kept on the device: resets are device copies, not host transfers
    starts = [torch.from_numpy(I.psi0_instance(w, seed=[1606, i])).to(b.device, torch.complex64)
              for i, w in enumerate(ens)]

    def reset():
        for i, p in enumerate(starts):
            b.set_psi(i, p)

    def timed():
        reset()
        b.step_imag(GRAPH_STEPS)             # graph capture outside the timed region
        reset()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(b.stream)
        b.step_imag(steps)
        ev1.record(b.stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev0.elapsed_time(ev1)

    wall0, _ = timed()
    reset()
    plan = autotune.tune(b, steps=tune_steps)
    wall1, gpu1 = timed()
    wall2 = None
    if two_streams:
        b.use_streams(True)
        wall2, _ = timed()
        b.use_streams(False)
    npts = b.points()
    byts = sum(step_bytes_2d(w["nx"], w["ny"] if w["geom"] == "2dxy" else w["nz"], 4)
               for w in ens)
    energies = [e["energy"] for e in b.energy()]
    out = {"workload": "imag2d ensemble: 192 XY/XZ instances, sizes {96..512}^2, dt 0.001",
           "instances": len(ens), "points": npts, "steps": steps,
           "value": npts * steps / wall1, "unit": "grid-point-steps/s",
           "ms_per_step": wall1 * 1e3 / steps, "gpu_event_ms_per_step": gpu1 / steps,
           "ms_per_step_default_plan": wall0 * 1e3 / steps,
           "ms_per_step_two_streams": None if wall2 is None else wall2 * 1e3 / steps,
           "step_algorithmic_bytes": byts,
           "step_achieved_GBs": round(byts / (wall1 / steps) / 1e9, 1),
           "tuned_plan": plan,
           "energy_range": [min(energies), max(energies)]}
    b.close()
    return out


def adjoint_128(nsteps=200, K=20):
    """The 128^3 adjoint workload (overlap loss, checkpoints every K): forward with
    checkpoints, then backward (segment recompute + one adjoint step per step), FP32."""
    import numpy as np
    import torch
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.adjoint import evolve_real, overlap_loss
    from paper_1601_04640_amd.binding import Solver
    w = I.WORKLOADS["adjoint3d_128"]
    out = {}
    for prec in ("fp32", "fp64"):
        s = Solver(w, prec=prec)
        dev = "cuda:0"
        x = I.grid_axes("3d", w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"])
        Z, Y, X = np.meshgrid(*x, indexing="ij")
        V = 0.5 * (X ** 2 + Y ** 2 + 9.0 * Z ** 2)
        psi0 = torch.from_numpy(I.psi0_adjoint3d_128()).to(dev, s.cdtype)
        target = torch.from_numpy(I.displaced_target(w, 1611, widths=(3 ** -0.5, 1.0, 1.0))
                                  ).to(dev, s.cdtype)
        dV = w["dx"] * w["dy"] * w["dz"]

        def run():
            p0 = psi0.clone().requires_grad_(True)
            Vt = torch.from_numpy(V).to(dev).requires_grad_(True)
            gt = torch.tensor(w["g"], dtype=torch.float64, device=dev, requires_grad=True)
            gdt = torch.tensor(w["gdd"], dtype=torch.float64, device=dev, requires_grad=True)
            L = overlap_loss(evolve_real(s, p0, Vt, gt, gdt, nsteps, K), target, dV)
            L.backward()
            torch.cuda.synchronize()
        run()
        t0 = time.perf_counter()
        run()
        wall = time.perf_counter() - t0
        s.close()
        out[prec] = {"ms_per_step_forward_and_backward": wall * 1e3 / nsteps,
                     "grid_point_steps_per_s": 128 ** 3 * nsteps / wall}
    out["workload"] = f"adjoint3d_128: {nsteps} real-time steps, checkpoints every {K}"
    return out


def adjoint_2d_256(nsteps=400, K=50):
    """The 256^2 adjoint workload's rate (overlap loss against the displaced target,
    checkpoints every K; the trap (x^2 + 1.5^2 y^2)/2 plus its seeded perturbation):
    forward with checkpoints, then backward, over nsteps real-time steps."""
    import numpy as np
    import torch
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.adjoint import evolve_real, overlap_loss
    from paper_1601_04640_amd.binding import Solver
    w = I.WORKLOADS["real2dxy_256"]
    out = {}
    y, x = I.grid_axes("2dxy", w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"])
    Y, X = np.meshgrid(y, x, indexing="ij")
    V = 0.5 * (X ** 2 + (w["nu"] * Y) ** 2) + I.trap_perturbation_real2dxy_256()
    for prec in ("fp32", "fp64"):
        s = Solver(w, prec=prec)
        dev = "cuda:0"
        psi0 = torch.from_numpy(I.psi0_real2dxy_256()).to(dev, s.cdtype)
        target = torch.from_numpy(I.displaced_target(w, 1610, widths=(1.0 / np.sqrt(1.5), 1.0))
                                  ).to(dev, s.cdtype)
        dV = w["dx"] * w["dy"]

        def run():
            p0 = psi0.clone().requires_grad_(True)
            Vt = torch.from_numpy(V).to(dev).requires_grad_(True)
            gt = torch.tensor(w["g"], dtype=torch.float64, device=dev, requires_grad=True)
            gdt = torch.tensor(w["gdd"], dtype=torch.float64, device=dev, requires_grad=True)
            L = overlap_loss(evolve_real(s, p0, Vt, gt, gdt, nsteps, K), target, dV)
            L.backward()
            torch.cuda.synchronize()
        run()
        t0 = time.perf_counter()
        run()
        wall = time.perf_counter() - t0
        s.close()
        out[prec] = {"ms_per_step_forward_and_backward": wall * 1e3 / nsteps,
                     "grid_point_steps_per_s": 256 ** 2 * nsteps / wall}
    out["workload"] = (f"real2dxy_256 adjoint: {nsteps} real-time steps (of the workload's "
                       f"4000), checkpoints every {K}")
    return out


# ---------------------------------------------------------------------- sweep
# to the paper's 600^3 and 15000^2, then to the largest grids the run-time-length passes
# address (fewer than 2^31 points: 1280^3, 46000^2)
SWEEP3 = (48, 50, 64, 80, 96, 100, 120, 128, 150, 160, 192, 200, 240, 250, 256, 300, 320, 360,
          384, 400, 450, 480, 500, 512, 540, 600, 700, 800, 1000, 1280)
SWEEP2 = (256, 384, 512, 1000, 1024, 1500, 2000, 2048, 3000, 4000, 4096, 5000, 6000, 8000, 8192,
          10000, 12000, 13000, 15000, 20000, 30000, 40000, 46000)
PASSES = {1: "specialised", 2: "run-time length", 3: "four-step, segmented"}


def sweep(args):
    """Throughput against grid size (one JSON line per grid and precision), the axis of the
    paper's Fig. 2 (3D cubes 50^3 -> 600^3, 2D squares from 1000^2): real-time steps of
    cubes and squares (trap (1,1,2), g 20, g_dd 6, R half the box in 3D; box 12.8),
    graph-replayed.  Lengths with specialised passes report the dominant pass's HBM
    fraction; the run-time-length kernels (other lengths) report null there.  2D squares
    past one LDS line (8192 FP32, 4096 FP64) run the four-step transforms and segmented
    sweeps.  Past the paper's 600^3 and 15000^2 the sweep goes on to the largest grids the
    run-time-length passes address (1280^3, 46000^2), as far as the GPU's memory holds
    them."""
    import torch
    from paper_1601_04640_amd import binding as B
    cases = []
    if 3 in args.sweep_dims:
        cases += [("3d", n) for n in SWEEP3 if args.sweep_min <= n <= args.sweep_max3]
    if 2 in args.sweep_dims:
        cases += [("2dxy", n) for n in SWEEP2 if args.sweep_min <= n <= args.sweep_max2]
    for geom, n in cases:
        for prec in args.sweep_prec:
            esz = 8 if prec == "fp64" else 4
            kind = B.gp_axis_kind(n, prec)
            if kind == 0:
                continue
            h = 12.8 / n
            w = dict(geom=geom, nx=n, ny=n, nz=n if geom == "3d" else 1, dx=h, dy=h, dz=h,
                     dt=0.0005, gamma=1.0, nu=1.0, lam=2.0 if geom == "3d" else 4.0, g=20.0,
                     gdd=6.0, R=6.4 if geom == "3d" else 0.0)
            npts = n ** (3 if geom == "3d" else 2)
            need = B.gp_workspace_bytes(B.make_params(**{**w, "prec": prec}))
            if need + 4 * esz * npts > 0.85 * torch.cuda.mem_get_info()[0]:
                continue
            # the separable Gaussian start, built on the device in the step's precision and
            # normalised from its factors (no host grid for the largest cases)
            rd = torch.float64 if prec == "fp64" else torch.float32
            x = (torch.arange(n, dtype=torch.float64, device="cuda") - n // 2) * h
            g1 = torch.exp(-0.5 * x * x)
            g1[0] = g1[-1] = 0.0
            if geom == "3d":
                gz = torch.exp(-0.5 * 2.0 * x * x)
                gz[0] = gz[-1] = 0.0
                norm = torch.sqrt((gz * gz).sum() * (g1 * g1).sum() ** 2 * h ** 3)
                gz, g1 = (gz / norm).to(rd), g1.to(rd)
                psi = (gz[:, None, None] * g1[None, :, None]) * g1[None, None, :]
            else:
                norm = torch.sqrt((g1 * g1).sum() ** 2 * h ** 2)
                psi = (g1 / norm).to(rd)[:, None] * g1.to(rd)[None, :]
            steps = max(GRAPH_STEPS, min(400, int(2e9 / npts) // GRAPH_STEPS * GRAPH_STEPS))
            r = time_gpu(None, prec, psi, steps, GRAPH_STEPS + 1, solver_params=w)
            wall = r["graph"]["wall"]
            byts = (step_bytes_3d(n, n, n, esz) if geom == "3d" else step_bytes_2d(n, n, esz))
            line = {"sweep": "grid size", "geom": geom, "n": n, "points": npts,
                    "dtype": "f64" if prec == "fp64" else "f32",
                    "passes": PASSES[kind],
                    "steps": steps, "value": npts * steps / wall, "unit": "grid-point-steps/s",
                    "ms_per_step": wall * 1e3 / steps, "step_algorithmic_bytes": byts,
                    "step_hbm_frac": round(byts / (wall / steps) / 1e9 / HBM_PEAK_GBS, 4),
                    "dominant_kernel_frac": roofline(r, esz)["frac"] if kind == 1 else None}
            print(json.dumps(line), flush=True)
            del psi, x, g1
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload (FP64 and FP32)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 2D ensemble")
    ap.add_argument("--batch-steps", type=int, default=400)
    ap.add_argument("--two-streams", action="store_true",
                    help="also time the ensemble with its two size classes on two streams")
    ap.add_argument("--sweep", action="store_true", help="throughput against grid size")
    ap.add_argument("--sweep-dims", type=int, nargs="*", default=[3, 2])
    ap.add_argument("--sweep-prec", nargs="*", default=["fp32", "fp64"])
    ap.add_argument("--sweep-max3", type=int, default=1280)
    ap.add_argument("--sweep-max2", type=int, default=46000)
    ap.add_argument("--sweep-min", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus}); sharding "
              "across GPUs is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle), before the GPU is used")
        cpu = cpu_baseline(args.cpu_budget)
        log(f"cpu: {cpu['one_thread']['value']:.3e} pt-steps/s on one thread, "
            f"{cpu['value']:.3e} on {cpu['cores']} cores")
    from paper_1601_04640_amd import inputs as I
    psi5 = I.psi0_real3d_256()
    log(f"{WORKLOAD}: fp64 then fp32, {args.steps} steps, {args.warmup} warmup")
    r64 = time_gpu(WORKLOAD, "fp64", psi5, args.steps, args.warmup)
    log(f"fp64: {r64['graph']['wall'] * 1e3 / args.steps:.4f} ms/step")
    r32 = time_gpu(WORKLOAD, "fp32", psi5, args.steps, args.warmup)
    log(f"fp32: {r32['graph']['wall'] * 1e3 / args.steps:.4f} ms/step")
    s64 = summary(r64, args.steps, 8)
    s32 = summary(r32, args.steps, 4)
    roof = dict(roofline(r64, 8), traffic=read_traffic(DOMINANT, WORKLOAD, "fp64"))
    log("accuracy: 500 steps, fp64 and fp32, against the oracle fixture")
    acc = accuracy_256()
    line = {
        "metric": METRIC,
        "value": s64["value"],
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: 256^3 real time, dx 0.1, dt 0.0005, g 50, "
                               "g_dd 25, trap (1,1,3), cutoff R 12.8, seeded Gaussian start "
                               "with 0.5% phase noise",
                   "grid": [256, 256, 256], "points": 256 ** 3},
        "roofline": roof,
        "step_hbm_frac": s64["step_hbm_frac"],
        "gpu_event_ms_per_step": s64["gpu_event_ms_per_step"],
        "fp32": dict(s32, dtype="f32", reductions_dtype="f64", roofline=dict(
            roofline(r32, 4), traffic=read_traffic(DOMINANT, WORKLOAD, "fp32"))),
        "accuracy": acc,
    }
    if not args.no_extra:
        log("128x96x80 quench")
        line["real3d_128x96x80"] = quench_128x96x80(args.steps, args.warmup)
        log("256^3 with V and the kernel table in host memory")
        line["host_resident_256"] = host_resident_256(args.steps, args.warmup)
        log("64^3 imaginary time")
        line["imag3d_64"] = imag3d_64(args.steps)
        log("128^3 adjoint")
        line["adjoint3d_128"] = adjoint_128()
        log("256^2 adjoint")
        line["adjoint2d_256"] = adjoint_2d_256()
        if not args.no_batch:
            line["batched_2d"] = time_batch(args.batch_steps, two_streams=args.two_streams)
            log(f"batched 2d: {line['batched_2d']['ms_per_step']:.4f} ms/step "
                f"(default plan {line['batched_2d']['ms_per_step_default_plan']:.4f})")
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
