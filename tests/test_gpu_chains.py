"""Launch chains: the islands of each instance split into two groups whose
generations of a migration epoch run as two launch sequences side by side in
the captured epoch graph.  Every state is compared whole with the oracle
(which runs the islands of a generation one after the other), and the
best-ever record (makespan, generation, permutation) with the oracle's."""
import numpy as np
import pytest

from gpu_util import assert_same_state, ensure_built, make_ctx, oracle_ga, say
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu


def _check_best(ctx, ga, inst, what):
    b, o = ctx.best(inst), ga.best()
    assert b["makespan"] == o["makespan"], what
    assert b["generation"] == o["generation"], what
    assert np.array_equal(np.asarray(b["perm"]), np.asarray(o["perm"])), what


@pytest.mark.parametrize("chains", [2, 1])
def test_sixteen_islands_epochs_in_chains(chains):
    """The large workload's layout at 1/16 of the side, ring-then-adaptive
    migration every 5 generations: whole epochs from the graph, an odd
    eager stretch, and epochs again."""
    ensure_built()
    w = inputs.workload("large", seed=4, scale=16)
    w["interval"] = 5
    say(f"[chains] sixteen islands, chains={chains}")
    ctx = make_ctx([w])
    ctx.set_chains(chains)
    assert ctx.chains() == chains
    ga = oracle_ga(w)
    for g in (5, 10, 3, 2, 10):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 16, f"chains {chains} generation {ctx.generation}")
        _check_best(ctx, ga, 0, f"chains {chains} generation {ctx.generation}")
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


def test_two_instances_medium_in_chains_and_switches():
    """Two medium-shaped instances (1/4 side) in one context, two chains by
    default, switched to one chain and back between epochs."""
    ensure_built()
    a = inputs.workload("medium", seed=6, scale=4)
    b = inputs.workload("medium", seed=7, scale=4)
    a["interval"] = b["interval"] = 10
    say("[chains] two instances, switching")
    ctx = make_ctx([a, b])
    assert ctx.chains() == 1           # automatic: small contexts keep one chain
    gas = [oracle_ga(a, inst=0), oracle_ga(b, inst=1)]
    for g, chains in ((10, 2), (10, 1), (7, 1), (3, 2), (20, 2)):
        ctx.set_chains(chains)
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, 2, f"instance {i} generation {ctx.generation}")
            _check_best(ctx, ga, i, f"instance {i} generation {ctx.generation}")
    ctx.close()


def test_automatic_chains():
    """Two chains for the large workload's 262144 individuals, one for the
    medium one's 8192, for a batch of several launch classes and with a
    swept island."""
    ensure_built()
    big = inputs.workload("large", seed=1)
    ctx = make_ctx([big])
    assert ctx.chains() == 2
    ctx.close()
    ctx = make_ctx([inputs.workload("medium", seed=1)])
    assert ctx.chains() == 1
    ctx.close()
    swept = inputs.workload("large", seed=1)
    swept["islands"][0]["sweep"] = 1
    ctx = make_ctx([swept])
    assert ctx.chains() == 1
    ctx.close()


def test_chains_checkpoint_restore():
    """A checkpoint of a two-chain context (both chains' records) restored
    into a fresh context continues exactly as the uninterrupted run."""
    ensure_built()
    w = inputs.workload("large", seed=8, scale=16)
    w["interval"] = 5
    say("[chains] checkpoint and restore")
    a = make_ctx([w])
    a.set_chains(2)
    a.evolve(10)
    image = a.checkpoint()
    a.evolve(10)
    b = make_ctx([w])
    b.set_chains(2)
    b.restore(image)
    b.evolve(10)
    ga = oracle_ga(w)
    ga.evolve(20)
    assert_same_state(a, ga, 0, 16, "uninterrupted generation 20")
    assert_same_state(b, ga, 0, 16, "restored generation 20")
    _check_best(b, ga, 0, "restored generation 20")
    assert a.checkpoint() == b.checkpoint()
    a.close()
    b.close()


@pytest.mark.parametrize("concurrent", [True, False])
def test_class_groups_epoch_branches(concurrent):
    """Twelve uneven batched instances (grids shrunk eightfold) with tiles
    that put them in several launch classes: with the classes side by side,
    each class's generations of an epoch are one branch of the epoch graph
    (the classes run out of step between migrations) and fold their own
    best-ever records.  Whole epochs, an eager stretch and epochs again,
    every instance compared with its oracle run and its best record."""
    ensure_built()
    ws = inputs.batched_workloads(count=12, batch_seed=11, scale=8)
    for w in ws:
        w["interval"] = 5
    say(f"[chains] class groups, concurrent={concurrent}")
    ctx = make_ctx(ws, mapping=1)
    for i in range(len(ws)):
        ctx.set_instance_tile(i, i % 2, (1, 2, 4)[i % 3])
    ctx.set_concurrent(concurrent)
    gas = [oracle_ga(w, inst=i) for i, w in enumerate(ws)]
    for g in (5, 10, 3, 2, 10):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, 2, f"instance {i} generation {ctx.generation}")
            _check_best(ctx, ga, i, f"instance {i} generation {ctx.generation}")
        for i, ga in enumerate(gas):
            assert ctx.migration_counters(i) == ga.counters()
    ctx.close()


def test_class_groups_small_class_fold_scratch():
    """Two launch classes; the second holds an instance whose own LDS is
    smaller than the best-ever workgroup's scratch at 8 waves per workgroup
    (n = 20, S = 40, per-stage mapping: 3104 bytes against 6144).  With one
    fold group per class that class's launch folds its own best-ever record,
    so its LDS must cover the scratch.  Every instance, its best makespan,
    generation and permutation against the oracle."""
    ensure_built()
    ws = []
    for j, (n, S) in enumerate([(20, 40), (500, 10)]):
        m, p = inputs.make_instance(n, S, 1, 3, seed=30 + j)
        ws.append(dict(m=m, p=p, islands=[inputs.cellular(4, 4, 0.9, 0.2), inputs.pseudo(16, 0.75, 0.05)],
                       interval=4, theta=1.0, topology=0))
    say("[chains] class groups with a small class at 8 waves per workgroup")
    ctx = make_ctx(ws)
    ctx.set_instance_tile(0, 0, 8)
    ctx.set_instance_tile(1, 1, 1)
    gas = [oracle_ga(w, inst=i) for i, w in enumerate(ws)]
    for g in (1, 3, 4, 8):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, 2, f"instance {i} generation {ctx.generation}")
            _check_best(ctx, ga, i, f"instance {i} generation {ctx.generation}")
    ctx.close()
