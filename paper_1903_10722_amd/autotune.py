"""Tile autotuner for the generation kernels.

A tile is (mapping, waves per workgroup): the decode mapping (0: a group of
n_stages lanes per chromosome, one lane per stage; 1: one lane per
chromosome through every stage) and the number of waves a workgroup holds
(1, 2, 4 or 8), which trades LDS per workgroup against how many waves share
one copy of the processing-time table.  Results are identical for every
tile, so the tuner only measures speed.  It times each candidate on a
throwaway context (the caller's GA trajectory is left untouched), keeps the
fastest in a JSON cache keyed by the device and the shape, and applies it.

autotune():           one tile for the whole context (waves per workgroup).
autotune_instances(): one tile per group of instances with the same jobs
                      bucket and stage count, chosen by timing the whole
                      batch -- for batches of uneven instances.
"""
from __future__ import annotations

import json
import os

from .binding import Context

CANDIDATES = (1, 2, 4, 8)
TILE_CANDIDATES = ((1, 4), (1, 2), (0, 4), (0, 2))
_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "autotune.json")


def _bucket(x: int) -> int:
    b = 1
    while b < x:
        b <<= 1
    return b


def _arch(ctx: Context) -> str:
    import torch
    props = torch.cuda.get_device_properties(ctx.device)
    return getattr(props, "gcnArchName", props.name)


def instance_key(inst: dict) -> str:
    a = inst["args"]
    kinds = "".join("c" if int(x["kind"]) == 0 else "p" for x in a["islands"])
    sizes = "/".join(str(_bucket(s)) for s in inst["sizes"])
    return f"n{_bucket(inst['n'])}-S{inst['S']}-m{int(max(a['m']))}-{kinds}-{sizes}"


def shape_key(ctx: Context) -> str:
    parts = sorted(set(instance_key(inst) for inst in ctx.instances))
    return _arch(ctx) + "|" + ";".join(parts)


def _load_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(cache: dict, path: str):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, path)


def _time_trial(device: int, insts, generations: int, waves: int, mapping: int = -1) -> float:
    """Milliseconds per generation of a throwaway context holding `insts`."""
    import torch
    trial = Context(device=device, waves_per_block=waves, mapping=mapping)
    try:
        for inst in insts:
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
            times[w] = _time_trial(ctx.device.index or 0, ctx.instances, generations, w)
        except RuntimeError:
            continue       # tile does not fit this workload's LDS
    best = min(times, key=times.get)
    ctx.set_waves_per_block(best)
    if use_cache:
        cache[key] = {"waves_per_block": best, "ms_per_generation": {str(k): v for k, v in times.items()}}
        _store(cache, cache_path)
    return {"waves_per_block": best, "ms_per_generation": times, "cached": False}


def group_key(inst: dict) -> str:
    """Coarse shape of an instance for the per-group tuner: jobs bucket and stages."""
    return f"n{_bucket(inst['n'])}-S{inst['S']}"


def _time_tiles(device: int, insts, tiles: dict, generations: int) -> float:
    """Milliseconds per generation of a throwaway context holding every
    instance of `insts`, instance i on tiles.get(i) (default tile if absent)."""
    import torch
    trial = Context(device=device)
    try:
        for inst in insts:
            trial.add_instance(**{**inst["args"], "interval": 0})
        for i, t in tiles.items():
            trial.set_instance_tile(i, t[0], t[1])
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


def autotune_instances(ctx: Context, generations: int = 4, candidates=TILE_CANDIDATES, use_cache: bool = True,
                       cache_path: str = _CACHE) -> dict:
    """Pick and apply a tile per group of instances of `ctx` with the same
    jobs bucket and stage count (not yet bound).

    Greedy coordinate descent on the whole context: starting from the
    automatic tiles, each group in turn (largest work first) tries every
    candidate while the others keep their current tile, every trial timed on
    a throwaway context holding all instances, since the launches of a
    generation share the GPU.  Returns {"groups": {key: {"tile": [m, w] or
    None (automatic), "instances": count}}, "ms_per_generation": {"automatic":
    ms, "tuned": ms}, "cached": bool}."""
    key = _arch(ctx) + "|tiles|" + ";".join(sorted(instance_key(i) for i in ctx.instances))
    cache = _load_cache(cache_path) if use_cache else {}
    groups: dict[str, list[int]] = {}
    for i, inst in enumerate(ctx.instances):
        groups.setdefault(group_key(inst), []).append(i)
    if key in cache:
        chosen = {g: (tuple(t) if t else None) for g, t in cache[key]["tiles"].items()}
        ms, cached = cache[key]["ms_per_generation"], True
    else:
        dev = ctx.device.index or 0
        work = {g: sum(ctx.instances[i]["n"] * ctx.instances[i]["S"] * sum(ctx.instances[i]["sizes"]) for i in idx)
                for g, idx in groups.items()}
        chosen = {g: None for g in groups}

        def tiles_of(ch):
            return {i: t for g, t in ch.items() if t for i in groups[g]}

        best = _time_tiles(dev, ctx.instances, {}, generations)
        auto = best
        for g in sorted(groups, key=lambda x: -work[x]):
            for cand in candidates:
                trial = dict(chosen)
                trial[g] = tuple(cand)
                try:
                    t = _time_tiles(dev, ctx.instances, tiles_of(trial), generations)
                except RuntimeError:
                    continue
                if t < best:
                    best, chosen = t, trial
        ms, cached = {"automatic": auto, "tuned": best}, False
        if use_cache:
            cache[key] = {"tiles": {g: (list(t) if t else None) for g, t in chosen.items()}, "ms_per_generation": ms}
            _store(cache, cache_path)
    for g, t in chosen.items():
        if t:
            for i in groups[g]:
                ctx.set_instance_tile(i, t[0], t[1])
    return {"groups": {g: {"tile": (list(t) if t else None), "instances": len(groups[g])} for g, t in chosen.items()},
            "ms_per_generation": ms, "cached": cached}
