"""Tile-shape autotuner for the generation kernel.

The only free parameter of the kernels' launch is the number of waves per
workgroup (1, 2, 4 or 8): it trades LDS per workgroup against how many
workgroups share one copy of the processing-time table.  Results are
identical for every choice, so the tuner only measures speed.  It times each
candidate on a throwaway context holding the same instances (the caller's
GA trajectory is left untouched), keeps the fastest in a JSON cache keyed by
the device and the workload shape, and applies it to the caller's context.
"""
from __future__ import annotations

import json
import os

from .binding import Context

CANDIDATES = (1, 2, 4, 8)
_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "autotune.json")


def _bucket(x: int) -> int:
    b = 1
    while b < x:
        b <<= 1
    return b


def shape_key(ctx: Context) -> str:
    import torch
    props = torch.cuda.get_device_properties(ctx.device)
    arch = getattr(props, "gcnArchName", props.name)
    parts = []
    for inst in ctx.instances:
        a = inst["args"]
        kinds = "".join("c" if int(x["kind"]) == 0 else "p" for x in a["islands"])
        sizes = "/".join(str(_bucket(s)) for s in inst["sizes"])
        parts.append(f"n{_bucket(inst['n'])}-S{inst['S']}-m{int(max(a['m']))}-{kinds}-{sizes}")
    parts = sorted(set(parts))
    return arch + "|" + ";".join(parts)


def _load_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _time_tile(ctx: Context, waves: int, generations: int) -> float:
    import torch
    trial = Context(device=ctx.device.index or 0, waves_per_block=waves)
    try:
        for inst in ctx.instances:
            trial.add_instance(**inst["args"])
        trial.bind()
        trial.evolve(2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(trial.stream)
        trial.evolve(generations)
        e1.record(trial.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / generations
    finally:
        trial.close()


def autotune(ctx: Context, generations: int = 20, candidates=CANDIDATES, use_cache: bool = True,
             cache_path: str = _CACHE) -> dict:
    """Pick and apply the fastest waves-per-block for `ctx` (bound or not).

    Returns {"waves_per_block": w, "ms_per_generation": {w: ms, ...}, "cached": bool}."""
    key = shape_key(ctx)
    cache = _load_cache(cache_path) if use_cache else {}
    if key in cache:
        best = int(cache[key]["waves_per_block"])
        ctx.set_waves_per_block(best)
        return {"waves_per_block": best, "ms_per_generation": cache[key]["ms_per_generation"], "cached": True}
    times = {}
    for w in candidates:
        try:
            times[w] = _time_tile(ctx, w, generations)
        except RuntimeError:
            continue       # tile does not fit this workload's LDS
    best = min(times, key=times.get)
    ctx.set_waves_per_block(best)
    if use_cache:
        cache[key] = {"waves_per_block": best, "ms_per_generation": {str(k): v for k, v in times.items()}}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, cache_path)
    return {"waves_per_block": best, "ms_per_generation": times, "cached": False}
