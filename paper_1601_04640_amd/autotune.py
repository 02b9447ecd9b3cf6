"""Autotuner for the batched ensemble's launch plan.

For every (pass, size class) of a `binding.Batch` it chooses the tile shape (the default
tiles, or x and CN column tiles of 8 lines and line-FFT blocks of twice the points:
`gp_batch_set_shape`) and the number of persistent blocks, timing a few graph-replayed
steps for each candidate and keeping the fastest, one coordinate at a time.  Results are
cached in a JSON file keyed by the ensemble's size multiset, precision and device name, so
a later run with the same ensemble reuses the plan.
"""
from __future__ import annotations

import hashlib
import json
import os

CANDIDATES = (128, 256, 384, 512, 768, 1024, 1536, 2048, 4096)
SHAPES = (0, 1)


def ensemble_key(batch, device_name: str) -> str:
    sizes = sorted(tuple(s) for s in batch.shapes)
    h = hashlib.sha256(json.dumps([sizes, batch.prec, device_name]).encode()).hexdigest()
    return h[:24]


def _time_steps(batch, steps, imag):
    torch = batch.torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    (batch.step_imag if imag else batch.step_real)(8)  # capture/warm the graph
    torch.cuda.synchronize()
    ev0.record(batch.stream)
    (batch.step_imag if imag else batch.step_real)(steps)
    ev1.record(batch.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def apply(batch, plan):
    """Set a plan {"pass:class": {"shape": s, "blocks": g}} on a batch."""
    for name, v in plan.items():
        p, c = name.split(":")
        batch.set_shape(p, int(c), v["shape"])
        batch.set_blocks(p, int(c), v["blocks"])


def tune(batch, steps=16, imag=True, cache_path=None, verbose=False):
    """Choose a tile shape and a persistent block count per (pass, size class); returns
    {"pass:class": {"shape": s, "blocks": g}}.  The instances' wave functions must be set
    (tuning steps evolve them)."""
    torch = batch.torch
    dev_name = torch.cuda.get_device_name(batch.device)
    key = ensemble_key(batch, dev_name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        apply(batch, cache[key])
        return cache[key]
    best_plan = {}
    base = _time_steps(batch, steps, imag)
    for (p, c), (items, _) in batch.plan().items():
        if items == 0:
            continue
        best = None
        for shape in SHAPES:
            batch.set_shape(p, c, shape)
            n = batch.plan()[(p, c)][0]
            for g in sorted({g for g in CANDIDATES if g < n} | {n}):
                batch.set_blocks(p, c, g)
                t = _time_steps(batch, steps, imag)
                if verbose:
                    print(f"[autotune]   {p} class {c}: shape {shape}, {g} blocks "
                          f"{t:.4f} ms/step", flush=True)
                if best is None or t < best[0]:
                    best = (t, shape, g)
        _, shape, g = best
        batch.set_shape(p, c, shape)
        batch.set_blocks(p, c, g)
        best_plan[f"{p}:{c}"] = {"shape": shape, "blocks": g}
        if verbose:
            print(f"[autotune] {p} class {c}: shape {shape}, {g} blocks "
                  f"({best[0]:.4f} ms/step)", flush=True)
    if verbose:
        print(f"[autotune] default {base:.4f} ms/step -> tuned "
              f"{_time_steps(batch, steps, imag):.4f} ms/step", flush=True)
    if cache_path:
        cache[key] = best_plan
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best_plan
