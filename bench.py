"""Benchmark of the island-GA hot path on one MI355X.

Headline workload: the large flexible-flow-shop configuration -- n=500 jobs,
10 stages, machines per stage uniform in [3,5], processing times uniform in
[1,99]; 8 cellular islands of 128x128 (crossover 0.9, swap mutation 0.1) and
8 pseudo islands of 16384 (crossover 0.75), ring-then-adaptive migration every
20 generations -- the largest configuration that fits one GPU.

A step is one migration epoch: 20 generations of every island (262144 exact
makespan decodes per generation, neighbourhood selection, order crossover,
swap mutation, replacement, complementary-pair mating, best-ever update) plus
the migration epoch that closes it.  The population is resident in HBM when
the timed region starts.  The medium workload (n=100, S=5, 64x64 + 4096) is
measured the same way and reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 lanes/clk x 2.4 GHz (32-bit integer VALU)
PEAK_LDS_TBS = 256 * 128 * 2.4e9 / 1e12   # 256 CUs x 128 bytes/clk x 2.4 GHz (nominal LDS bandwidth)

WORKLOADS = {
    "medium": "medium: n=100 jobs, 5 stages, machines U[1,5], p U[1,99]; cellular 64x64 (pc 0.9, pm 0.1) + "
              "pseudo 4096 (pc 0.75); adaptive migration every 20 generations; step = one 20-generation epoch",
    "tiny": "tiny: n=20 jobs, 3 stages, machines [2,2,2], p U[1,99]; cellular 8x8 + pseudo 64; migration every 10",
    "large": "large: n=500 jobs, 10 stages, machines U[3,5], p U[1,99]; 8 cellular 128x128 + 8 pseudo 16384; "
             "ring-then-adaptive migration every 20",
    "surrogate": "surrogate: n=1000 jobs, 20 stages, machines U[2,6], p U[1,99]; cellular 64x64 + pseudo 4096; "
                 "migration every 20",
    "batched": "batched: 256 instances, n in {20,50,100,200,500}, S in {5,10,20}, machines U[1,5], grids 32..128; "
               "migration every 10",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["medium", "tiny", "large", "surrogate", "batched"],
                    help="workload of the timed steps (default: the large workload, the largest single-GPU one)")
    ap.add_argument("--secondary", default="medium", choices=["", "medium", "tiny", "large", "surrogate", "batched"],
                    help="a second workload measured the same way and reported beside the headline ('' = none)")
    ap.add_argument("--prescreen-k", type=int, default=0,
                    help="run the timed steps with the learned pre-screen (k candidates per cell)")
    ap.add_argument("--waves-per-block", type=int, default=None)
    ap.add_argument("--mapping", type=int, default=-1, choices=[-1, 0, 1],
                    help="decode mapping: -1 automatic, 0 one lane per stage, 1 one lane per chromosome")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workload: skip the per-shape tile autotuner (outside the timed region)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--surrogate-seconds", type=float, default=8.0,
                    help="wall-clock budget of each side of the plain vs pre-screen comparison (0 = skip)")
    ap.add_argument("--experiment", default="", choices=["", "islands", "tardiness", "decode", "surrogate"],
                    help="islands: island-layout ablation and migration-gap sweep; tardiness: Section 5 on the "
                         "paper-faithful variant (each prints one JSON line)")
    ap.add_argument("--decode-count", type=int, default=1_000_000,
                    help="random permutations per workload shape of --experiment decode")
    ap.add_argument("--runs", type=int, default=20, help="seeds per configuration of --experiment")
    ap.add_argument("--ga-seed0", type=int, default=101, help="first GA seed of --experiment surrogate")
    ap.add_argument("--generations", type=int, default=2000, help="generations per run of --experiment")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times), to calibrate HBM counters")
    return ap.parse_args()


KERNEL_SOURCES = ("ffs_kernels.h", "ffs_lane.h", "philox.h")
TT_KERNEL_SOURCES = ("ffs_tt.hip", "philox.h")   # the paper-faithful variant's kernels


def source_digest(read=None, sources=KERNEL_SOURCES) -> str:
    """SHA-256 of the device-code sources: traffic counters are only reported
    for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_10722_amd", "csrc")
    for f in sources:
        if read is None:
            with open(os.path.join(csrc, f), "rb") as fh:
                data = fh.read()
        else:
            data = read(f)
        h.update(f.encode() + b"\0" + data)
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str, sources=KERNEL_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the summary is missing or was taken on different sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_digest(sources=sources):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy(mib: int):
    import torch
    src = torch.ones(mib * 1024 * 1024 // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": mib * 1024 * 1024,
                      "bytes_written": mib * 1024 * 1024, "launches": 5}), flush=True)


# Island sides of the oracle's sample are divided by this factor (the same
# instance, operators and schedule, fewer individuals per generation), so
# that a generation of the single-threaded oracle takes about a second.
CPU_SCALE = {"tiny": 1, "medium": 1, "large": 4, "surrogate": 2, "batched": 8}

_CPU_CHILD = r"""
import json, os, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1903_10722_amd import inputs
name, seed, scale, seconds = sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), float(sys.argv[5])
ws = inputs.batched_workloads(count=256, batch_seed=7, scale=scale) if name == "batched" else \
     [inputs.workload(name, seed=seed, scale=scale)]
t0 = time.perf_counter()
gas = [oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], theta=w["theta"],
                 topology=w["topology"], seed=101, inst=i) for i, w in enumerate(ws)]
t_init = time.perf_counter() - t0
per_gen = sum(sum(x["size"] for x in w["islands"]) for w in ws)
gens = 0
t1 = time.perf_counter()
while time.perf_counter() - t1 < seconds:
    for ga in gas:
        ga.evolve(1)
    gens += 1
dt = time.perf_counter() - t1
print(json.dumps({"per_gen": per_gen, "gens": gens, "seconds": dt, "init_s": t_init,
                  "affinity": sorted(os.sched_getaffinity(0))}))
"""


def cpu_baseline(name: str, seed: int, seconds: float) -> dict:
    """The oracle (single-threaded C) on a bounded sample of the same
    workload: the same instance(s) with island sides divided by CPU_SCALE,
    generation 0 then whole generations for about `seconds`, in a child
    process pinned to one host core (taskset)."""
    import subprocess
    core = min(os.sched_getaffinity(0))
    scale = CPU_SCALE[name]
    args = [sys.executable, "-c", _CPU_CHILD, ROOT, name, str(seed), str(scale), str(seconds)]
    try:
        res = subprocess.run(["taskset", "-c", str(core)] + args, capture_output=True, text=True, check=True)
        pinned = "taskset -c %d" % core
    except (OSError, subprocess.CalledProcessError):
        res = subprocess.run(args, capture_output=True, text=True, check=True)
        pinned = "not pinned (taskset unavailable)"
    r = json.loads(res.stdout.strip().splitlines()[-1])
    sides = "full size" if scale == 1 else f"island sides / {scale}"
    return {"value": r["per_gen"] * r["gens"] / r["seconds"], "unit": "decodes/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle GA on the {name} workload ({sides}, {r['per_gen']} individuals per generation): "
                      f"generation 0 ({r['init_s']:.2f} s) then {r['gens']} generations in {r['seconds']:.1f} s, "
                      f"one thread, {pinned}",
            "generations_per_s": r["gens"] / r["seconds"], "host_cpu": host_cpu(),
            "host_threads": len(os.sched_getaffinity(0)), "affinity": r["affinity"]}


def lds_peak(repeats: int = 3) -> dict:
    """Achievable LDS read bandwidth of this GPU: the probe kernel of
    csrc/lds_probe.hip (conflict-free 16-byte reads on every CU), best of
    `repeats` launches timed with HIP events."""
    import ctypes

    import torch
    from paper_1903_10722_amd.build import PROBE_LIB
    lib = ctypes.CDLL(PROBE_LIB)
    lib.lds_probe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                              ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
    blocks, iters = 256 * 16, 4096
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    best = 0.0
    for _ in range(repeats):
        ms, nbytes = ctypes.c_float(), ctypes.c_double()
        rc = lib.lds_probe(ctypes.c_void_p(st.cuda_stream), blocks, iters, ctypes.c_void_p(out.data_ptr()),
                           ctypes.byref(ms), ctypes.byref(nbytes))
        if rc != 0:
            raise RuntimeError(f"lds_probe failed with HIP error {rc}")
        best = max(best, nbytes.value / (ms.value / 1e3))
    return {"kernel": "k_lds_probe", "bytes_per_s": best, "TB_per_s": best / 1e12, "blocks": blocks,
            "reads_per_thread": iters, "nominal_TB_per_s": PEAK_LDS_TBS}


def host_cpu() -> str:
    """Model name of the host CPU (first entry of /proc/cpuinfo), or ''."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _finite_or_none(x):
    x = float(x)
    return x if x == x and abs(x) != float("inf") else None


def surrogate_compare(seconds: float, seed: int = 101) -> dict:
    """Best makespan at equal wall-clock: the plain GA and the GA with the
    learned pre-screen (k = 8 candidates per cell) on the surrogate workload
    (n=1000 jobs, 20 stages, machines U[2,6], p U[1,99]; cellular 64x64 +
    pseudo 4096; migration every 20).  Both start from the same generation 0
    (GA seed `seed`)."""
    import numpy as np
    import torch
    from scipy.stats import spearmanr

    from paper_1903_10722_amd import Context, inputs
    w = inputs.workload("surrogate", seed=1)
    p64, m64 = w["p"].astype(np.int64), w["m"].astype(np.int64)
    lb = max(int(p64.sum(axis=1).max()), max(int(-(-p64[:, k].sum() // m64[k])) for k in range(p64.shape[1])))
    out = {"workload": "surrogate: n=1000 jobs, 20 stages, machines U[2,6], p U[1,99]; cellular 64x64 + "
                       "pseudo 4096; migration every 20; k=8 candidates per cell, warm-up 5",
           "budget_s": seconds, "lower_bound": lb}
    for name, k in (("plain", 0), ("prescreen", 8)):
        ctx = Context(device=0)
        ctx.add_instance(w["m"], w["p"], w["islands"], interval=w["interval"], theta=w["theta"],
                         topology=w["topology"], seed=seed, surrogate_k=k, surrogate_warmup=5)
        ctx.bind()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            ctx.evolve(w["interval"])   # whole epochs, replayed from a captured graph
            torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = {"best_makespan": ctx.best(0)["makespan"], "generations": ctx.generation, "seconds": dt}
        if k:
            cand = ctx.surrogate_candidates(exact=True)
            ex, pred = cand["exact"].astype(np.float64), cand["pred"].astype(np.float64)
            chosen = ex[np.arange(ex.shape[0]), cand["choice"]]
            spread = [i for i in range(ex.shape[0]) if np.ptp(ex[i]) > 0]
            # rank correlations are undefined (null) once every candidate of
            # every cell decodes to the same makespan (a converged population)
            res.update({"spearman": _finite_or_none(spearmanr(pred.reshape(-1), ex.reshape(-1)).correlation)
                        if np.ptp(ex) > 0 else None,
                        "spearman_within_cell": _finite_or_none(np.nanmean([spearmanr(pred[i], ex[i]).correlation
                                                                           for i in spread])) if spread else None,
                        "cells_with_distinct_candidates": len(spread),
                        "mae": float(np.abs(pred - ex).mean()),
                        "chosen_minus_candidate0": float(chosen.mean() - ex[:, 0].mean())})
        out[name] = res
        ctx.close()
        print(f"[surrogate] seed {seed} {name}: best {res['best_makespan']} after {res['generations']} "
              f"generations", file=sys.stderr, flush=True)
    return out


def surrogate_experiment(seconds: float, seeds) -> dict:
    """The learned pre-screen against the plain GA at equal wall-clock on the
    surrogate workload, one pair of runs per GA seed: per-seed pairs, mean and
    standard deviation of the best makespans and of their difference."""
    import numpy as np
    pairs = [surrogate_compare(seconds, seed=sd) for sd in seeds]
    plain = np.array([x["plain"]["best_makespan"] for x in pairs], dtype=np.float64)
    pre = np.array([x["prescreen"]["best_makespan"] for x in pairs], dtype=np.float64)
    sd = (lambda a: float(a.std(ddof=1)) if len(a) > 1 else 0.0)
    return {"experiment": "surrogate", "budget_s": seconds, "seeds": list(seeds),
            "workload": pairs[0]["workload"], "lower_bound": pairs[0]["lower_bound"],
            "plain_mean": float(plain.mean()), "plain_sd": sd(plain),
            "prescreen_mean": float(pre.mean()), "prescreen_sd": sd(pre),
            "prescreen_minus_plain_mean": float((pre - plain).mean()), "prescreen_minus_plain_sd": sd(pre - plain),
            "pairs": [{"seed": sd_, "plain": x["plain"], "prescreen": x["prescreen"]} for sd_, x in zip(seeds, pairs)]}


def islands_experiment(runs: int, generations: int) -> dict:
    """Island-layout ablation and migration-gap sweep in Section 5's setting
    (300 jobs, 4 stages, 2 machines per stage, p uniform in [1, 5], 512
    individuals; makespan objective): the dual heterogeneous layout, a single
    cellular torus, a single pseudo population, two islands of one kind, and
    the dual layout at migration gaps 10 ... 800, and the cellular parent
    selection variants (self + best neighbour, binary tournaments) on the
    layouts with cellular islands, and sixteen islands with ring-then-pairs
    against the rule on every ring edge.  `runs` GA seeds run as
    instances of one batched context; best makespans are read at checkpoints."""
    import numpy as np
    import torch

    from paper_1903_10722_amd import Context, inputs
    w0 = inputs.paper_setting("dual")
    p64, m64 = w0["p"].astype(np.int64), w0["m"].astype(np.int64)
    lb = max(int(p64.sum(axis=1).max()), max(int(-(-p64[:, k].sum() // m64[k])) for k in range(p64.shape[1])))
    configs = [(v, 500, 0, 0) for v in inputs.ISLAND_VARIANTS] + \
              [("dual", i, 0, 0) for i in (10, 20, 50, 100, 200, 300, 800)] + \
              [(v, 500, sel, 0) for sel in (1, 2) for v in ("dual", "cellular", "cellular2")] + \
              [("ring16", i, 0, top) for top in (1, 2) for i in (50, 500)]
    checkpoints = [c for c in (50, 100, 200, 500, 1000, 2000) if c < generations] + [generations]
    rows = []
    for variant, interval, sel, top in configs:
        w = inputs.paper_setting(variant, interval=interval, sel=sel, topology=top)
        ctx = Context(device=0)
        for r in range(runs):
            ctx.add_instance(w["m"], w["p"], w["islands"], interval=interval, theta=w["theta"],
                             topology=w["topology"], seed=1000 + r)
        ctx.bind()
        curve = []
        ms, done = 0.0, 0
        for c in checkpoints:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            ctx.evolve(c - done)
            e1.record(ctx.stream)
            best = np.array([ctx.best(i)["makespan"] for i in range(runs)], dtype=np.float64)
            ms += e0.elapsed_time(e1)
            done = c
            curve.append({"generation": c, "best_mean": float(best.mean())})
        found = [ctx.best(i)["generation"] for i in range(runs)]
        ctx.close()
        rows.append({"layout": variant, "selection": sel, "topology": w["topology"],
                     "islands": [f"cellular {x['rows']}x{x['cols']}" if x["kind"] == 0 else f"pseudo {x['size']}"
                                 for x in w["islands"]],
                     "interval": interval if len(w["islands"]) > 1 else None,
                     "best_mean": float(best.mean()), "best_std": float(best.std(ddof=1)) if runs > 1 else 0.0,
                     "best_min": int(best.min()), "best_max": int(best.max()),
                     "gap_to_lb_mean": float((best.mean() - lb) / lb),
                     "found_generation_mean": float(np.mean(found)), "curve": curve,
                     "ms_per_generation_all_runs": ms / generations})
        print(f"[islands] {variant} interval={interval} selection={sel}: mean {best.mean():.2f}", file=sys.stderr,
              flush=True)
    return {"experiment": "islands",
            "setting": "300 jobs, 4 stages, 2 machines per stage, p U[1,5]; 512 individuals; cellular rates "
                       "1.00/0.05, pseudo crossover 0.75; theta 1; makespan objective",
            "generations": generations, "runs": runs, "ga_seeds": f"1000..{1000 + runs - 1}",
            "lower_bound": lb, "rows": rows}


def tardiness_experiment(runs: int, generations: int) -> dict:
    """Section 5 on the paper-faithful variant (Table 1's data: 300 jobs, 4
    stages, 2 unrelated machines per stage, P U[1,5], release and due dates,
    WT = 100; objective WT * sum T + C_max; machine-assignment genotype):
    Table 2's comparison of the heterogeneous GA (16x16 cellular + pseudo
    256, migration gap 500) with a cellular GA (16x32) and a pseudo GA (512),
    Fig. 4's gap sweep of the heterogeneous GA, and the asynchronous
    line-sweep update of the cellular islands (an alternative reading); all
    of it again on a loaded shop whose releases span an eighth of the range.  `runs` seeds run as the
    batched runs of one context per configuration; objectives are reported in
    time units (the library works in hundredths)."""
    import numpy as np
    import torch

    from paper_1903_10722_amd import inputs
    from paper_1903_10722_amd.tardiness import TtContext
    # (layout, gap, line sweep, release scale): Table 1 read literally, then
    # a loaded shop with the release range compressed by sum_s M_s = 8
    configs = [(v, 500, False, 1.0) for v in ("dual", "cellular", "pseudo")] + \
              [("dual", g, False, 1.0) for g in (10, 50, 100, 200, 800)] + \
              [(v, 500, True, 1.0) for v in ("dual", "cellular")] + \
              [(v, 500, False, 0.125) for v in ("dual", "cellular", "pseudo")] + \
              [("dual", g, False, 0.125) for g in (10, 100, 800)] + \
              [(v, 500, True, 0.125) for v in ("dual", "cellular")]
    checkpoints = [c for c in (100, 500, 1000) if c < generations] + [generations]
    rows, kernel = [], None
    for variant, interval, sweep, rscale in configs:
        w = inputs.tardiness_setting(variant, seed=1, interval=interval, release_scale=rscale)
        inst, isl = w["inst"], w["islands"]
        ctx = TtContext(inst, isl, interval=interval if len(isl) > 1 else 0, theta=w["theta"], seed=1000, runs=runs,
                        sweep=sweep)
        curve, ms, done = [], 0.0, 0
        for c in checkpoints:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            ctx.evolve(c - done)
            e1.record(ctx.stream)
            best = np.array([ctx.best(r)["objective"] for r in range(runs)], dtype=np.float64) / 100.0
            ms += e0.elapsed_time(e1)
            done = c
            curve.append({"generation": c, "best_mean": float(best.mean())})
        found = [ctx.best(r)["generation"] for r in range(runs)]
        if kernel is None:
            ctx.set_timing(True)
            ctx.evolve(200)
            k_ms, launches = ctx.kernel_time()
            ctx.set_timing(False)
            J, S = inst["P"].shape[:2]
            per_decode = sum(J * (6 + (int(m) - 1) * int(np.ceil(np.log2(J)))) for m in inst["M"])
            n_ind = sum(x["size"] for x in isl) * runs
            avg_s = k_ms / launches / 1e3
            achieved = per_decode * n_ind / avg_s / 1e12
            kernel = {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                      "frac": achieved / PEAK_INT_TOPS,
                      "traffic": recorded_traffic("k_tt_generation", "section5", TT_KERNEL_SOURCES),
                      "kernel": "k_tt_generation",
                      "avg_launch_us": avg_s * 1e6, "launches": launches,
                      "timing": "HIP events around each generation launch (eager launches)",
                      "ops_per_decode": per_decode, "decodes_per_launch": n_ind}
        ctx.close()
        n_ind = sum(x["size"] for x in isl) * runs
        rows.append({"layout": variant, "cellular_update": "line sweep" if sweep else "synchronous",
                     "release_scale": rscale,
                     "islands": [f"cellular {x['rows']}x{x['cols']}" if x["kind"] == 0 else f"pseudo {x['size']}"
                                 for x in isl],
                     "interval": interval if len(isl) > 1 else None,
                     "best": float(best.min()), "average": float(best.mean()),
                     "variance": float(best.var(ddof=1)) if runs > 1 else 0.0,
                     "found_generation_mean": float(np.mean(found)), "curve": curve,
                     "ms_per_generation_all_runs": ms / generations,
                     "decodes_per_s": n_ind * generations / (ms / 1e3)})
        print(f"[tardiness] {variant} gap={interval} sweep={sweep} release_scale={rscale}: average "
              f"{best.mean():.2f}", file=sys.stderr, flush=True)
    # the oracle on the heterogeneous layout, one run, about 5 s
    from oracle import tardiness as ot
    w = inputs.tardiness_setting("dual", seed=1, interval=500)
    ga = ot.GA(w["inst"], w["islands"], interval=500, seed=1000)
    t1, gens = time.perf_counter(), 0
    while time.perf_counter() - t1 < 5.0:
        ga.evolve(1)
        gens += 1
    dt = time.perf_counter() - t1
    per_gen = sum(x["size"] for x in w["islands"])
    return {"experiment": "tardiness",
            "setting": "Table 1 data: 300 jobs, 4 stages, 2 unrelated machines per stage, P U[1,5], R U[0,Pbar], "
                       "D = R + Pbar_j (1 + U[0,2]), WT 100; 512 individuals; cellular 1.00/0.05, pseudo 0.75; "
                       "theta 1; objective WT * sum T + C_max in time units; synthetic instance (seed 1)",
            "generations": generations, "runs": runs, "rows": rows, "roofline": kernel,
            "cpu_baseline": {"value": per_gen * gens / dt, "unit": "decodes/s", "cores": 1, "kind": "oracle",
                             "sample": f"oracle GA of the variant, heterogeneous layout, one run: {gens} "
                                       f"generations of {per_gen} decodes in {dt:.1f} s, one thread"},
            "paper_table2_context": {"heterogeneous": [306500.03, 309885.90, 2003059.14],
                                     "cellular": [314467.50, 320648.18, 6792896.04],
                                     "pseudo": [314636.59, 317683.23, 2963668.96],
                                     "columns": ["best", "average", "variance"],
                                     "note": "the paper's own instance (not published) on its hardware; context, "
                                             "not a target"}}


def decode_experiment(count: int) -> dict:
    """The exact makespan decode alone, through ffs_evaluate: `count` uniformly
    random permutations per workload shape (tiny, medium, large, surrogate),
    generated on the device (argsort of seeded uniform keys) and resident in
    HBM before the timed region; HIP events on the library's stream bracket
    each call, median of three.  Work per decode as for the generation
    kernel: n * sum_k (m_k + 6) integer operations.  The oracle decodes a
    sample of the same shape on one host thread."""
    import numpy as np
    import torch

    import oracle
    from paper_1903_10722_amd import Context, inputs
    rows = []
    for name in ("tiny", "medium", "large", "surrogate"):
        w = inputs.workload(name, seed=1)
        n, S = w["p"].shape
        m = [int(x) for x in w["m"]]
        ctx = Context(device=0)
        ctx.add_instance(w["m"], w["p"], w["islands"], interval=0, theta=w["theta"], topology=w["topology"],
                         seed=101)
        ctx.bind()
        g = torch.Generator(device="cuda").manual_seed(1000 + n)
        perms = torch.empty((count, n), dtype=torch.int32, device="cuda")
        chunk = max(1, (1 << 27) // n)   # keys of at most 512 MB at a time
        for r0 in range(0, count, chunk):
            r1 = min(count, r0 + chunk)
            perms[r0:r1] = torch.argsort(torch.rand((r1 - r0, n), device="cuda", generator=g), dim=1).to(torch.int32)
        torch.cuda.synchronize()
        ctx.evaluate(0, perms[:4096])   # warm-up
        times = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            out = ctx.evaluate(0, perms)
            e1.record(ctx.stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        ops = n * sum(x + 6 for x in m)
        achieved = ops * count / (ms / 1e3) / 1e12
        # the oracle on a sample of the same shape, about 2 s
        sample = inputs.random_perms(64, n, seed=7)
        t0, done = time.perf_counter(), 0
        while time.perf_counter() - t0 < 2.0:
            oracle.decode(w["m"], w["p"], sample[done % len(sample)])
            done += 1
        cpu = done / (time.perf_counter() - t0)
        rows.append({"workload": WORKLOADS[name], "n": n, "S": S, "machines": m, "decodes": count,
                     "ms": ms, "decodes_per_s": count / (ms / 1e3),
                     "job_stage_steps_per_s": count * n * S / (ms / 1e3),
                     "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                                  "frac": achieved / PEAK_INT_TOPS, "ops_per_decode": ops},
                     "cpu_baseline": {"value": cpu, "unit": "decodes/s", "cores": 1, "kind": "oracle",
                                      "sample": f"oracle decode of {done} random permutations of this shape "
                                                f"in about 2 s, one thread"},
                     "makespan_min": int(out.min().item())})
        print(f"[decode] {name}: {count / (ms / 1e3) / 1e6:.1f} M decodes/s", file=sys.stderr, flush=True)
        del perms, out
        ctx.close()
    return {"experiment": "decode", "count_per_shape": count,
            "timing": "HIP events around ffs_evaluate on the library's stream, median of 3; inputs resident",
            "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the island GA of this "
              f"build keeps every island on a single MI355X.", file=sys.stderr)
        sys.exit(2)
    if args.experiment == "islands":
        print(json.dumps(islands_experiment(args.runs, args.generations)), flush=True)
        return
    if args.experiment == "tardiness":
        print(json.dumps(tardiness_experiment(args.runs, args.generations)), flush=True)
        return
    if args.experiment == "decode":
        print(json.dumps(decode_experiment(args.decode_count)), flush=True)
        return
    if args.experiment == "surrogate":
        print(json.dumps(surrogate_experiment(args.surrogate_seconds,
                                              list(range(args.ga_seed0, args.ga_seed0 + args.runs)))),
              flush=True)
        return
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
        return
    import torch  # noqa: F401

    from paper_1903_10722_amd.binding import library_path
    if not os.path.exists(library_path()):
        from paper_1903_10722_amd.build import build_library
        build_library()

    head = measure(args.workload, args.seed, args.steps, args.warmup, args)
    out = {
        "metric": "makespan decodes/sec and generations/sec at 1 GPU; best makespan at fixed time budget",
        "value": head["value"],
        "unit": "decodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": head["config"],
        "generations_per_s": head["generations_per_s"],
        "best_makespan": head["best_makespan"],
        "best_found_generation": head["best_found_generation"],
        "generations_run": head["generations_run"],
        "wall_s_timed": head["wall_s_timed"],
        "bind_and_generation0_s": head["bind_and_generation0_s"],
        "roofline": head["roofline"],
    }
    try:
        peak = lds_peak()
        lm = out["roofline"]["lds_model"]
        lm["probe_TB_per_s"] = peak["TB_per_s"]
        lm["frac_of_probe"] = lm["achieved_TB_per_s"] / peak["TB_per_s"]
        lm["frac_of_nominal"] = lm["achieved_TB_per_s"] / PEAK_LDS_TBS
    except (OSError, RuntimeError) as e:
        print(f"[bench] LDS probe unavailable: {e}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.seed, args.cpu_seconds)
    if args.secondary and args.secondary != args.workload:
        sec = measure(args.secondary, args.seed, max(1, min(args.steps, 25)), min(args.warmup, 2), args)
        out["secondary"] = {args.secondary: {k: sec[k] for k in ("value", "ms_per_step", "generations_per_s",
                                                                  "config", "roofline", "best_makespan")}}
    if args.surrogate_seconds > 0:
        out["best_makespan_at_fixed_budget"] = surrogate_compare(args.surrogate_seconds)
    print(json.dumps(out), flush=True)


def measure(name: str, seed: int, steps: int, warmup: int, args) -> dict:
    """Time `steps` migration epochs of workload `name` (after `warmup`
    epochs) and the generation kernel's average launch."""
    import torch

    from paper_1903_10722_amd import Context, inputs
    if name == "batched":
        ws = inputs.batched_workloads(count=256, batch_seed=7)
    else:
        ws = [inputs.workload(name, seed=seed)]
    w = ws[0]
    m = w["m"]
    I = w["interval"]
    decodes_per_gen = sum(sum(x["size"] for x in v["islands"]) for v in ws)
    ctx = Context(device=0, waves_per_block=args.waves_per_block, mapping=args.mapping)
    for v in ws:
        ctx.add_instance(v["m"], v["p"], v["islands"], interval=I, theta=v["theta"], topology=v["topology"], seed=101,
                         surrogate_k=args.prescreen_k, surrogate_warmup=5)
    tiles = None
    if name == "batched" and not args.no_autotune and args.mapping < 0 and args.waves_per_block is None:
        from paper_1903_10722_amd.autotune import autotune_instances
        t_tune = time.perf_counter()
        tiles = autotune_instances(ctx)
        t_tune = time.perf_counter() - t_tune
        print(f"[bench] batched tiles tuned in {t_tune:.1f} s: " +
              ", ".join(f"{k}: {v['tile']}" for k, v in tiles["groups"].items()) +
              f"; ms per generation {tiles['ms_per_generation']}", file=sys.stderr, flush=True)
    t_bind = time.perf_counter()
    ctx.bind()
    t_bind = time.perf_counter() - t_bind
    stream = ctx.stream
    used = ctx.mapping()
    chains = ctx.chains()
    kernel = {0: "k_generation", 1: "k_generation_lane", 2: "k_generation_lane+k_generation"}[used]

    for _ in range(warmup):
        ctx.evolve(I)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        ctx.evolve(I)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    gens = I * steps
    decodes = decodes_per_gen * gens
    best = ctx.best(0)
    generations_run = ctx.generation

    # dominant kernel (the generation kernel): its average launch duration
    if args.prescreen_k:
        # the pre-screened path runs eagerly: HIP events around every launch
        ctx.set_timing(True)
        for _ in range(max(1, min(steps, 25))):
            ctx.evolve(I)
        k_ms, launches = ctx.kernel_time()
        ctx.set_timing(False)
        timing = "HIP events around each launch (eager launches)"
        ctx.close()
    else:
        ctx.close()
        # back to back as in the timed region: a context of the same instances
        # without migration replays graphs whose every node is a generation
        # launch; HIP events bracket the replays on the library's stream
        ctx2 = Context(device=0, waves_per_block=args.waves_per_block, mapping=args.mapping)
        for v in ws:
            ctx2.add_instance(v["m"], v["p"], v["islands"], interval=0, theta=v["theta"], topology=v["topology"],
                              seed=101)
        if tiles:
            from paper_1903_10722_amd.autotune import group_key
            for i, inst in enumerate(ctx2.instances):
                t = tiles["groups"][group_key(inst)]["tile"]
                if t:
                    ctx2.set_instance_tile(i, t[0], t[1])
        ctx2.bind()
        L = 16
        ctx2.evolve(L)
        torch.cuda.synchronize()
        epochs = max(1, min(steps, 25))
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(ctx2.stream)
        ctx2.evolve(L * epochs)
        k1.record(ctx2.stream)
        torch.cuda.synchronize()
        k_ms, launches = k0.elapsed_time(k1), L * epochs
        ctx2.close()
        timing = "HIP events around back-to-back graph replays of generation launches only"
        if chains == 2:
            timing += ("; one launch = one generation of every island: two concurrent dispatches (launch chains), "
                       "each over half of the islands")
    avg_s = k_ms / max(1, launches) / 1e3
    ops_per_launch = sum(int(v["p"].shape[0]) * int(sum(int(x) + 6 for x in v["m"])) *
                         sum(x["size"] for x in v["islands"]) for v in ws)
    achieved = ops_per_launch / avg_s / 1e12
    # the decode's LDS traffic in the model of its algorithmic bytes:
    # 4 n (2 S + sum m) bytes per decode (processing-time reads, machine-free
    # scans and writes), against the probe's achievable LDS bandwidth
    lds_bytes = sum(4 * int(v["p"].shape[0]) * (2 * int(v["p"].shape[1]) + int(sum(int(x) for x in v["m"]))) *
                    sum(x["size"] for x in v["islands"]) for v in ws)
    return {
        "value": decodes / (ms / 1e3),
        "ms_per_step": ms / steps,
        "config": {"workload": WORKLOADS[name] + ("" if not args.prescreen_k else
                                                  f"; learned pre-screen k={args.prescreen_k}"),
                   "machines": [int(x) for x in m] if len(ws) == 1 else "per instance",
                   "decodes_per_generation": decodes_per_gen, "generations_per_step": I,
                   "mapping": {0: "per stage", 1: "per lane", 2: "per instance (autotuned)"}[used],
                   "launch_chains": chains,
                   **({"tiles": {k: v["tile"] for k, v in tiles["groups"].items()},
                       "tuning_ms_per_generation": tiles["ms_per_generation"]} if tiles else {})},
        "generations_per_s": gens / (ms / 1e3),
        "best_makespan": best["makespan"],
        "best_found_generation": best["generation"],
        "generations_run": generations_run,
        "wall_s_timed": wall,
        "bind_and_generation0_s": t_bind,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_INT_TOPS, "traffic": recorded_traffic(kernel, name),
                     "kernel": kernel, "avg_launch_us": avg_s * 1e6, "launches": launches, "timing": timing,
                     "ops_per_launch": ops_per_launch,
                     "lds_model": {"bytes_per_launch": lds_bytes, "achieved_TB_per_s": lds_bytes / avg_s / 1e12}},
    }


if __name__ == "__main__":
    main()
