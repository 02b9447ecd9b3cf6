"""Build libgpdbec.so (HIP, gfx950) in-tree: one object per (precision, pass family)
plus the C-ABI translation unit, compiled in parallel with hipcc, linked shared."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgpdbec.so")
ARCH = os.environ.get("GPDBEC_ARCH", "gfx950")

HIPCC = "/opt/rocm/bin/hipcc"
GXX = "g++"
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra"]
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _jobs(build_dir=BUILD, extra=()):
    jobs = []
    for real in ("float", "double"):
        for fam in (0, 1, 2):
            obj = os.path.join(build_dir, f"inst_{real}_{fam}.o")
            cmd = [HIPCC, *FLAGS, *extra, f"-DGP_REAL={real}", f"-DGP_FAMILY={fam}", "-c",
                   os.path.join(CSRC, "gp_inst.hip"), "-o", obj]
            jobs.append((obj, cmd))
    for real in ("float", "double"):
        obj = os.path.join(build_dir, f"generic_{real}.o")
        jobs.append((obj, [HIPCC, *FLAGS, *extra, f"-DGP_REAL={real}", "-c",
                           os.path.join(CSRC, "gp_generic_inst.hip"), "-o", obj]))
    for real in ("float", "double"):
        obj = os.path.join(build_dir, f"batch_{real}.o")
        jobs.append((obj, [HIPCC, *FLAGS, *extra, f"-DGP_REAL={real}", "-c",
                           os.path.join(CSRC, "gp_batch_inst.hip"), "-o", obj]))
    obj = os.path.join(build_dir, "capi.o")
    jobs.append((obj, [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, "gp_capi.hip"), "-o", obj]))
    # host-only code over the public C ABI (saved states, output cadence)
    obj = os.path.join(build_dir, "state.o")
    jobs.append((obj, [GXX, *HOST_FLAGS, "-c", os.path.join(CSRC, "gp_state.cpp"), "-o", obj]))
    return jobs


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                    and "not a recognized feature" not in l)
    return r.returncode, err


def build(verbose: bool = True, out: str = LIB, build_dir: str = BUILD, extra=()) -> str:
    """Compile and link the library to `out`; `extra` adds hipcc flags (e.g. -D tile
    thresholds) to every translation unit."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = _jobs(build_dir, tuple(extra))
    workers = min(len(jobs), max(1, min(os.cpu_count() or 1, 8)))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: (j[0], _run(j[1])), jobs))
    failed = [(o, e) for o, (rc, e) in results if rc != 0]
    if failed:
        msg = "\n\n".join(f"{o}:\n{e}" for o, e in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = out + ".tmp"
    rc, err = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
                    *[o for o, _ in jobs]])
    if rc != 0:
        raise RuntimeError(f"link failed:\n{err}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}", file=sys.stderr)
    return out


if __name__ == "__main__":
    build()
