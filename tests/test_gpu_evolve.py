"""GPU parity of the whole generation loop (ffs_evolve / ffs_migrate /
ffs_best / ffs_get_population) against the oracle: same seed, same
trajectory, bit-exact genes and makespans of every island."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_state, ensure_built, make_ctx, oracle_ga, say
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("inst_seed", [1, 2])
def test_tiny_trajectory(inst_seed):
    """Tiny workload at its full size: 8x8 cellular + 64 pseudo, n=20, S=3,
    100 generations, migration every 10; compared after every chunk."""
    ensure_built()
    w = inputs.workload("tiny", seed=inst_seed)
    say(f"[evolve] tiny inst_seed={inst_seed}")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    assert_same_state(ctx, ga, 0, 2, "generation 0")
    done = 0
    for chunk in [1, 4, 5, 10, 7, 13, 20, 40]:
        ctx.evolve(chunk)
        ga.evolve(chunk)
        done += chunk
        assert ctx.generation == done
        assert_same_state(ctx, ga, 0, 2, f"generation {done}")
        b1, b2 = ctx.best(0), ga.best()
        assert b1["makespan"] == b2["makespan"] and b1["generation"] == b2["generation"]
        assert b1["perm"].tolist() == b2["perm"].tolist()
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


def test_medium_scaled_trajectory():
    """Medium instance (n=100, S=5, m in [1,5]) on 32x32 + 1024 islands,
    60 generations with adaptive migration every 20."""
    ensure_built()
    w = inputs.workload("medium", seed=1, scale=2)
    say("[evolve] medium scale=2")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for g in (19, 1, 20, 20):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"generation {ctx.generation}")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


def test_medium_full_size_generations():
    """The benchmarked medium workload at full size (64x64 + 4096): the GPU
    state after 19 generations is loaded into the oracle, then generation 20
    (with its migration epoch) and 21 are compared exactly."""
    ensure_built()
    w = inputs.workload("medium", seed=1)
    say("[evolve] medium full size")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    # generation 0 must already agree (initialisation + decode of 8192 individuals)
    assert_same_state(ctx, ga, 0, 2, "generation 0")
    ctx.evolve(19)
    for isl in range(2):
        genes, mk = ctx.population(0, isl)
        ga.set_population(isl, genes, mk)
    ga.set_generation(19)
    for g in (20, 21):
        ctx.evolve(1)
        ga.evolve(1)
        assert_same_state(ctx, ga, 0, 2, f"generation {g}")
    ctx.close()


def test_surrogate_size_full_generations():
    """The plain GA on the longest instance (n=1000, S=20, m in [2,6]) at
    full size (64x64 + 4096): generation 0 whole, then the GPU state after
    19 generations loaded into the oracle and generations 20 (with its
    migration epoch) and 21 compared exactly.  At n=1000 the crossover chunk
    per lane exceeds the register path, so this covers the longer paths."""
    ensure_built()
    w = inputs.workload("surrogate", seed=2)
    say("[evolve] n=1000 S=20 full size")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    assert_same_state(ctx, ga, 0, 2, "generation 0")
    ctx.evolve(19)
    for isl in range(2):
        genes, mk = ctx.population(0, isl)
        ga.set_population(isl, genes, mk)
    ga.set_generation(19)
    for g in (20, 21):
        ctx.evolve(1)
        ga.evolve(1)
        assert_same_state(ctx, ga, 0, 2, f"generation {g}")
    # the best-so-far record holds at most the current populations' minimum
    cur = min(int(ga.population(i)[1].min()) for i in range(2))
    assert ctx.best(0)["makespan"] <= cur
    ctx.close()


def test_sixteen_islands_ring_then_adaptive():
    """Large instance (n=500, S=10, m in [3,5]) on 16 islands (8 cellular
    8x8, 8 pseudo 64), ring-then-adaptive migration every 20, 40 generations,
    plus one forced epoch."""
    ensure_built()
    w = inputs.workload("large", seed=1, scale=16)
    say("[evolve] large scale=16, 16 islands, topology 1")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for g in (20, 20):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 16, f"generation {ctx.generation}")
    ctx.migrate(0)
    ga.migrate()
    assert_same_state(ctx, ga, 0, 16, "forced epoch")
    ctx.evolve(3)
    ga.evolve(3)
    assert_same_state(ctx, ga, 0, 16, "after forced epoch")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    ctx.close()


def test_large_full_size_one_generation_sampled():
    """The large workload at full size (16 islands of 16384, n=500, S=10):
    generation 0 of two islands, then generation 1 of one cellular and one
    pseudo island recomputed by the oracle from the GPU's generation-0 state."""
    ensure_built()
    w = inputs.workload("large", seed=1)
    say("[evolve] large full size")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for isl in (0, 8):
        g1, m1 = ctx.population(0, isl)
        g2, m2 = ga.population(isl)
        assert np.array_equal(m1, m2) and np.array_equal(g1, g2), f"generation 0 island {isl}"
    ctx.evolve(1)
    for isl in (3, 12):
        ga.step_island(isl)
        g1, m1 = ctx.population(0, isl)
        g2, m2 = ga.population(isl)
        assert np.array_equal(m1, m2) and np.array_equal(g1, g2), f"generation 1 island {isl}"
    ctx.close()


def test_batched_uneven_instances():
    """Eight instances of the uneven batch (n in {20..500}, S in {5,10,20},
    grids shrunk 8x) in one context: each matches its own oracle run."""
    ensure_built()
    ws = inputs.batched_workloads(count=8, batch_seed=7, scale=8)
    say("[evolve] batched 8 instances " + str([(w["p"].shape, w["islands"][0]["rows"]) for w in ws]))
    ctx = make_ctx(ws)
    gas = [oracle_ga(w, inst=i) for i, w in enumerate(ws)]
    for g in (10, 15):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, 2, f"instance {i} generation {ctx.generation}")
            assert ctx.best(i)["makespan"] == ga.best()["makespan"]
    ctx.close()


def test_tile_shapes_give_identical_trajectories():
    ensure_built()
    w = inputs.workload("tiny", seed=3)
    ref = None
    for wpb in (1, 2, 8):
        say(f"[evolve] tiny waves_per_block={wpb}")
        ctx = make_ctx([w], waves_per_block=wpb)
        ctx.evolve(30)
        st = [ctx.population(0, i) for i in range(2)]
        ctx.close()
        if ref is None:
            ga = oracle_ga(w)
            ga.evolve(30)
            ref = [ga.population(i) for i in range(2)]
        for a, b in zip(st, ref):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("variant", ["no_operators", "always_mutate", "n2_S1", "theta0", "odd_shapes"])
def test_edge_workloads(variant):
    ensure_built()
    if variant == "no_operators":
        m, p = inputs.make_instance(15, 3, 1, 3, seed=3)
        isl = [inputs.cellular(3, 4, 0.0, 0.0), inputs.pseudo(10, 0.0, 0.0)]
        w = dict(m=m, p=p, islands=isl, interval=5)
    elif variant == "always_mutate":
        m, p = inputs.make_instance(25, 4, 1, 4, seed=4)
        isl = [inputs.cellular(5, 3, 1.0, 1.0), inputs.pseudo(12, 1.0, 1.0)]
        w = dict(m=m, p=p, islands=isl, interval=3)
    elif variant == "n2_S1":
        m, p = inputs.make_instance(2, 1, 1, 1, seed=5, machines=[1])
        isl = [inputs.cellular(3, 3, 0.9, 0.5), inputs.pseudo(4, 0.75, 0.5)]
        w = dict(m=m, p=p, islands=isl, interval=2)
    elif variant == "theta0":
        m, p = inputs.make_instance(30, 5, 1, 5, seed=6)
        isl = [inputs.cellular(4, 4, 0.9, 0.1), inputs.pseudo(16, 0.75, 0.0)]
        w = dict(m=m, p=p, islands=isl, interval=4, theta=0.0)
    else:
        m, p = inputs.make_instance(33, 7, 1, 6, seed=7)
        isl = [inputs.cellular(3, 11, 0.9, 0.1), inputs.pseudo(130, 0.75, 0.05)]
        w = dict(m=m, p=p, islands=isl, interval=6)
    say(f"[evolve] edge {variant}")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for g in (1, 6, 13):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"{variant} generation {ctx.generation}")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    ctx.close()


def test_stored_makespans_match_redecode():
    """Invariant on the GPU's own state: every stored makespan equals the
    oracle's decode of the stored permutation, which is a permutation."""
    ensure_built()
    w = inputs.workload("medium", seed=2, scale=4)
    say("[evolve] redecode medium scale=4")
    ctx = make_ctx([w])
    ctx.evolve(25)
    for isl in range(2):
        genes, mk = ctx.population(0, isl)
        rows = np.arange(0, len(mk), 7)
        for r in rows:
            assert sorted(genes[r].tolist()) == list(range(w["p"].shape[0]))
        assert np.array_equal(mk[rows], oracle.decode_many(w["m"], w["p"], genes[rows]))
    ctx.close()


def test_graph_replay_and_eager_agree():
    """Epoch graphs (default) and eager launches give the oracle's trajectory;
    replays are checked after every epoch, with host work in between."""
    ensure_built()
    w = inputs.workload("tiny", seed=4)
    for graphs in (True, False):
        say(f"[evolve] tiny graphs={graphs}")
        ctx = make_ctx([w])
        ctx.set_graphs(graphs)
        ga = oracle_ga(w)
        for _ in range(5):
            ctx.evolve(10)
            ga.evolve(10)
            assert_same_state(ctx, ga, 0, 2, f"graphs={graphs} generation {ctx.generation}")
        ctx.close()


def test_tile_change_after_bind_and_autotuner():
    """Changing the tile shape mid-run (also through the autotuner) keeps the
    trajectory."""
    ensure_built()
    from paper_1903_10722_amd.autotune import autotune
    w = inputs.workload("medium", seed=3, scale=4)
    say("[evolve] tile change after bind")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for wpb in (2, 8, 1):
        ctx.set_waves_per_block(wpb)
        ctx.evolve(7)
        ga.evolve(7)
        assert_same_state(ctx, ga, 0, 2, f"waves_per_block={wpb}")
    res = autotune(ctx, generations=10, use_cache=False)
    assert res["waves_per_block"] in (1, 2, 4, 8)
    ctx.evolve(13)
    ga.evolve(13)
    assert_same_state(ctx, ga, 0, 2, "after autotune")
    ctx.close()


def _parallel(fn, items, workers=None):
    """Run independent oracle calls on worker threads (the C oracle releases
    the GIL inside ctypes calls; every item has its own oracle object)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


@pytest.mark.timeout(900)
def test_batched_full_size_256_instances():
    """The uneven batch at full size: 256 instances (n in {20..500}, S in
    {5,10,20}, grids 32x32 .. 128x128) in one context, migration every 10.
    The GPU state after 9 generations is loaded into one oracle run per
    instance; generation 10 and its migration epoch are then compared exactly
    on every island of every instance."""
    ensure_built()
    ws = inputs.batched_workloads(count=256, batch_seed=7)
    say("[evolve] batched full size, 256 instances, all compared at generation 10")
    ctx = make_ctx(ws)
    ctx.evolve(9)
    states = [[ctx.population(i, isl) for isl in range(2)] for i in range(len(ws))]
    ctx.evolve(1)
    assert ctx.generation == 10

    import threading
    done = [0]
    lock = threading.Lock()

    def oracle_gen10(i):
        ga = oracle_ga(ws[i], inst=i)
        for isl in range(2):
            ga.set_population(isl, *states[i][isl])
        ga.set_generation(9)
        ga.evolve(1)
        out = [ga.population(isl) for isl in range(2)]
        del ga
        with lock:
            done[0] += 1
            if done[0] % 32 == 0:
                say(f"[evolve] batched: oracle done for {done[0]} of {len(ws)} instances")
        return out

    want = _parallel(oracle_gen10, range(len(ws)))
    say("[evolve] batched: oracle generation 10 done")
    for i in range(len(ws)):
        for isl in range(2):
            g1, m1 = ctx.population(i, isl)
            g2, m2 = want[i][isl]
            assert np.array_equal(m1, m2), f"instance {i} island {isl}: makespans differ"
            assert np.array_equal(g1, g2), f"instance {i} island {isl}: genes differ"
    ctx.close()


@pytest.mark.timeout(300)
def test_medium_full_trajectory_every_epoch():
    """The benchmarked medium workload (n=100, S=5, 64x64 + 4096, migration
    every 20) over its whole 500 generations, compared with the oracle at the
    end of every migration epoch, with the best-ever record and counters."""
    ensure_built()
    w = inputs.workload("medium", seed=1)
    say("[evolve] medium full size, 500 generations")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for e in range(25):
        ctx.evolve(20)
        ga.evolve(20)
        assert_same_state(ctx, ga, 0, 2, f"generation {ctx.generation}")
        b1, b2 = ctx.best(0), ga.best()
        assert (b1["makespan"], b1["generation"]) == (b2["makespan"], b2["generation"])
        assert b1["perm"].tolist() == b2["perm"].tolist()
    assert ctx.generation == 500
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


@pytest.mark.timeout(600)
def test_large_full_size_epoch_all_islands():
    """The large workload at full size (8 cellular 128x128 + 8 pseudo 16384,
    n=500, S=10, ring-then-adaptive every 20): the GPU state after 19
    generations is loaded into the oracle; generation 20 with its migration
    epoch (the ring over 16 islands, then the adaptive rule on each pair,
    sorting 16384 slots per island) is compared on all 16 islands, and so is
    one more forced epoch."""
    ensure_built()
    w = inputs.workload("large", seed=1)
    say("[evolve] large full size, generation 20 epoch on 16 islands")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    ctx.evolve(19)
    for isl in range(16):
        ga.set_population(isl, *ctx.population(0, isl))
    ga.set_generation(19)
    ctx.evolve(1)
    ga.evolve(1)
    say("[evolve] large: oracle generation 20 done")
    assert_same_state(ctx, ga, 0, 16, "generation 20")
    ctx.migrate(0)
    ga.migrate()
    assert_same_state(ctx, ga, 0, 16, "forced epoch")
    ctx.close()


def test_best_record_with_eight_waves_and_wide_stages():
    """Forty stages leave one chromosome per wave, so a workgroup's LDS is
    smaller than the best-ever fold's scratch at eight waves per workgroup;
    the best record (makespan, generation, permutation) must still match."""
    ensure_built()
    m, p = inputs.make_instance(20, 40, 1, 3, seed=12)
    isl = [inputs.cellular(3, 4, 0.9, 0.2), inputs.pseudo(12, 0.75, 0.1)]
    w = dict(m=m, p=p, islands=isl, interval=4)
    say("[evolve] n=20 S=40, 8 waves per workgroup")
    ctx = make_ctx([w], waves_per_block=8)
    ga = oracle_ga(w)
    for g in (1, 3, 6, 10):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"generation {ctx.generation}")
        b1, b2 = ctx.best(0), ga.best()
        assert (b1["makespan"], b1["generation"]) == (b2["makespan"], b2["generation"])
        assert b1["perm"].tolist() == b2["perm"].tolist()
    ctx.close()
