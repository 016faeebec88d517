"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import os
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ensure_built():
    from paper_1903_10722_amd.binding import library_path
    if not os.path.exists(library_path()):
        from paper_1903_10722_amd.build import build_library
        build_library()


def make_ctx(workloads, waves_per_block=None, seed=101, mapping=None):
    """One context holding every workload (instance i gets RNG instance id i)."""
    from paper_1903_10722_amd import Context
    ctx = Context(device=0, waves_per_block=waves_per_block, mapping=mapping)
    for w in workloads:
        ctx.add_instance(w["m"], w["p"], w["islands"], interval=w["interval"], theta=w.get("theta", 1.0),
                         topology=w.get("topology", 0), seed=w.get("seed", seed))
    ctx.bind()
    return ctx


def oracle_ga(w, inst=0, seed=101):
    import oracle
    return oracle.GA(w["m"], w["p"], w["islands"], interval=w["interval"], theta=w.get("theta", 1.0),
                     topology=w.get("topology", 0), seed=w.get("seed", seed), inst=inst)


def assert_same_state(ctx, ga, inst, n_islands, what=""):
    for isl in range(n_islands):
        g1, m1 = ctx.population(inst, isl)
        g2, m2 = ga.population(isl)
        if not np.array_equal(m1, m2):
            bad = np.nonzero(m1 != m2)[0]
            raise AssertionError(f"{what} island {isl}: makespans differ at {bad[:10]} "
                                 f"gpu={m1[bad[:5]]} oracle={m2[bad[:5]]}")
        if not np.array_equal(g1, g2):
            bad = np.nonzero((g1 != g2).any(axis=1))[0]
            raise AssertionError(f"{what} island {isl}: genes differ in slots {bad[:10]}")
