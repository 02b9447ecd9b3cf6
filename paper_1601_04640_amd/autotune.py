"""Autotuner for the batched ensemble's launch plan.

For every (pass, size class) of a `binding.Batch`, it times a few graph-replayed steps
for each candidate number of persistent blocks and keeps the fastest, one coordinate at
a time.  Results are cached in a JSON file keyed by the ensemble's size multiset,
precision and device name, so a later run with the same ensemble reuses the plan.
"""
from __future__ import annotations

import hashlib
import json
import os

CANDIDATES = (128, 256, 384, 512, 768, 1024, 1536, 2048, 4096)


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


def tune(batch, steps=16, imag=True, cache_path=None, verbose=False):
    """Choose persistent block counts per (pass, size class); returns {key: blocks}.
    The instances' wave functions must be set (tuning steps evolve them)."""
    torch = batch.torch
    dev_name = torch.cuda.get_device_name(batch.device)
    key = ensemble_key(batch, dev_name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        plan = cache[key]
        for name, blocks in plan.items():
            p, c = name.split(":")
            batch.set_blocks(p, int(c), blocks)
        return plan
    best_plan = {}
    base = _time_steps(batch, steps, imag)
    for (p, c), (items, _) in batch.plan().items():
        if items == 0:
            continue
        trials = sorted({g for g in CANDIDATES if g < items} | {items})
        best_g, best_t = None, None
        for g in trials:
            batch.set_blocks(p, c, g)
            t = _time_steps(batch, steps, imag)
            if verbose:
                print(f"[autotune]   {p} class {c}: {g} blocks {t:.4f} ms/step", flush=True)
            if best_t is None or t < best_t:
                best_g, best_t = g, t
        batch.set_blocks(p, c, best_g)
        best_plan[f"{p}:{c}"] = best_g
        if verbose:
            print(f"[autotune] {p} class {c}: {items} items -> {best_g} blocks "
                  f"({best_t:.4f} ms/step)", flush=True)
    if verbose:
        print(f"[autotune] default {base:.4f} ms/step -> tuned "
              f"{_time_steps(batch, steps, imag):.4f} ms/step", flush=True)
    if cache_path:
        cache[key] = best_plan
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best_plan
