"""Profiling workloads and summaries for rocprofv3.

Run modes (each is one small program to put after `rocprofv3 ... --`):

  python3 paper_1601_04640_amd/profile_run.py steps W PREC N
      N direct-launch (no graph) real-time steps of workload W (a key of inputs.WORKLOADS)
      in precision PREC (fp32 / fp64) from its seeded Gaussian start.
  python3 paper_1601_04640_amd/profile_run.py grid GEOM N PREC STEPS
      STEPS direct-launch real-time steps of the grid-size sweep's N^3 cube (GEOM 3d) or
      N^2 square (2dxy), any supported length.
  python3 paper_1601_04640_amd/profile_run.py batch N
      N imaginary-time steps of the 192-instance quasi-2D ensemble (FP32), direct launches.
  python3 paper_1601_04640_amd/profile_run.py copy MIB
      three plain device-to-device copies of MIB MiB: the reference for scaling the HBM
      counters (a copy reads and writes exactly MIB MiB).

Summaries (no GPU):

  python3 paper_1601_04640_amd/profile_run.py pmc KERNEL OUT FETCH_DIR WRITE_DIR
          COPY_FETCH_DIR COPY_WRITE_DIR COPY_MIB COMMAND...
      averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the dispatches whose name
      contains KERNEL, and the scales (copy bytes / copy counter) measured by the copy
      runs, into a key = value text file.
  python3 paper_1601_04640_amd/profile_run.py stats OUT DIR COMMAND...
      the per-kernel duration table of a `--kernel-trace --stats` run.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = "paper_1601_04640_amd/csrc"


def kernel_hash():
    """Hash of every device and launch source the counters depend on (all of csrc/:
    the kernels, the finalisation folded into them, the launch shapes and the host
    schedule that orders the passes)."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, CSRC))):
        if f.endswith((".hpp", ".hip", ".h")):
            with open(os.path.join(ROOT, CSRC, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def run_steps(workload, prec, n):
    sys.path.insert(0, ROOT)
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Solver
    w = I.WORKLOADS[workload]
    s = Solver(w, prec=prec)
    s.use_graphs(False)
    if workload == "real3d_256":
        psi0 = I.psi0_real3d_256()
    elif workload == "real3d_128x96x80":
        psi0 = I.psi0_real3d_128x96x80()
    else:
        psi0 = I.gaussian(w["geom"], w["nx"], w["ny"], w["nz"], w["dx"], w["dy"], w["dz"],
                          widths=(0.7, 1.0, 1.0))
    s.set_psi(psi0)
    print(f"[profile] {workload} {prec}: {n} steps", flush=True)
    s.step_real(n)
    s.sync()
    s.close()


def run_grid(geom, n, prec, steps):
    """Real-time steps of the grid-size sweep's n^3 cube or n^2 square (trap (1,1,2),
    g 20, g_dd 6, box 12.8), launched pass by pass."""
    sys.path.insert(0, ROOT)
    import numpy as np
    from paper_1601_04640_amd.binding import Solver
    h = 12.8 / n
    w = dict(geom=geom, nx=n, ny=n, nz=n if geom == "3d" else 1, dx=h, dy=h, dz=h,
             dt=0.0005, gamma=1.0, nu=1.0, lam=2.0 if geom == "3d" else 4.0, g=20.0,
             gdd=6.0, R=6.4 if geom == "3d" else 0.0)
    s = Solver(w, prec=prec)
    s.use_graphs(False)
    x = (np.arange(n) - n // 2) * h
    g1 = np.exp(-0.5 * x * x)
    g1[0] = g1[-1] = 0.0
    psi = (g1[:, None, None] * g1[None, :, None] * g1[None, None, :] if geom == "3d"
           else g1[:, None] * g1[None, :]).astype(np.complex128)
    s.set_psi(psi / np.sqrt(np.sum(np.abs(psi) ** 2) * h ** psi.ndim))
    print(f"[profile] {geom} {n} {prec}: {steps} steps", flush=True)
    s.step_real(steps)
    s.sync()
    s.close()


def run_batch(n):
    sys.path.insert(0, ROOT)
    from paper_1601_04640_amd import inputs as I
    from paper_1601_04640_amd.binding import Batch
    ens = I.batched_ensemble()
    b = Batch(ens, prec="fp32")
    b.use_graphs(False)
    for i, w in enumerate(ens):
        b.set_psi(i, I.psi0_instance(w, seed=[1606, i]))
    print(f"[profile] batch {len(ens)} instances: {n} steps", flush=True)
    b.step_imag(n)
    b.torch.cuda.synchronize()
    b.close()


def run_copy(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.ones_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        a.copy_(b)
    torch.cuda.synchronize()
    print(f"[profile] copy {mib} MiB x3", flush=True)


def _rows(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _counter(d, counter, name_has, biggest=False):
    vals = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in _rows(d, "counter_collection.csv")
            if r["Counter_Name"] == counter and name_has in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no {counter} rows for '{name_has}' under {d}")
    if biggest:  # the copy of known size: its largest-grid dispatches
        g = max(v[0] for v in vals)
        vals = [v for v in vals if v[0] == g]
    return sum(v[1] for v in vals) / len(vals), len(vals)


def summarize_pmc(kernel, out, fdir, wdir, cfdir, cwdir, copy_mib, command):
    f, nf = _counter(fdir, "FETCH_SIZE", kernel)
    w, nw = _counter(wdir, "WRITE_SIZE", kernel)
    cf, _ = _counter(cfdir, "FETCH_SIZE", "copyBuffer", biggest=True)
    cw, _ = _counter(cwdir, "WRITE_SIZE", "copyBuffer", biggest=True)
    kib = copy_mib * 1024.0
    lines = [
        f"# HBM counters of {kernel} (rocprofv3 --pmc, one counter per run), KiB per dispatch,",
        "# and the scale that maps each counter onto bytes, from a plain device copy of",
        f"# {copy_mib} MiB (reads and writes {copy_mib} MiB) profiled the same way.",
        "# command: " + command,
        f"kernel = {kernel}",
        f"kernel_source_hash = {kernel_hash()}",
        f"dispatches_fetch = {nf}",
        f"dispatches_write = {nw}",
        f"FETCH_SIZE_KiB_per_dispatch = {f:.3f}",
        f"WRITE_SIZE_KiB_per_dispatch = {w:.3f}",
        f"copy_FETCH_SIZE_KiB = {cf:.3f}",
        f"copy_WRITE_SIZE_KiB = {cw:.3f}",
        f"fetch_scale = {kib / cf:.4f}",
        f"write_scale = {kib / cw:.4f}",
        f"hbm_bytes_per_dispatch = {(f * kib / cf + w * kib / cw) * 1024.0:.0f}",
    ]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_stats(out, d, command):
    rows = _rows(d, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 --kernel-trace --stats; command: {command}",
             f"# {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}  kernel"]
    for r in rows:
        name = r["Name"]
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"  {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):6.2f}  {short}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv):
    if not argv:
        raise SystemExit(__doc__)
    mode = argv[0]
    if mode == "steps":
        run_steps(argv[1], argv[2], int(argv[3]))
    elif mode == "grid":
        run_grid(argv[1], int(argv[2]), argv[3], int(argv[4]))
    elif mode == "batch":
        run_batch(int(argv[1]))
    elif mode == "copy":
        run_copy(int(argv[1]))
    elif mode == "pmc":
        summarize_pmc(argv[1], argv[2], argv[3], argv[4], argv[5], argv[6], int(argv[7]),
                      " ".join(argv[8:]))
    elif mode == "stats":
        summarize_stats(argv[1], argv[2], " ".join(argv[3:]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
