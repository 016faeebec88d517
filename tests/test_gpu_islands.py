"""GPU parity of the island-layout ablation configurations (one cellular
torus, one pseudo island, two islands of the same kind with migration, and
the benchmarked dual layout at other migration intervals) against the
oracle: same seed, same trajectory, bit-exact genes and makespans."""
import pytest

from gpu_util import assert_same_state, ensure_built, make_ctx, oracle_ga, say
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", inputs.ISLAND_VARIANTS)
def test_island_variant_trajectory(variant):
    """Each layout at 1/8 of the side (the single torus is 8x16), migration
    every 10 generations, 40 generations compared after every chunk."""
    ensure_built()
    w = inputs.island_variant(variant, seed=1, scale=8, interval=10)
    n_isl = len(w["islands"])
    say(f"[islands] {variant} scale=8")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    assert_same_state(ctx, ga, 0, n_isl, f"{variant} generation 0")
    for g in (10, 1, 14, 15):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, n_isl, f"{variant} generation {ctx.generation}")
    b1, b2 = ctx.best(0), ga.best()
    assert b1["makespan"] == b2["makespan"] and b1["generation"] == b2["generation"]
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


@pytest.mark.parametrize("interval", [10, 50])
def test_dual_layout_other_intervals(interval):
    """The dual layout at 1/4 of the side with migration every 10 or 50
    generations, 100 generations."""
    ensure_built()
    w = inputs.island_variant("dual", seed=2, scale=4, interval=interval)
    say(f"[islands] dual scale=4 interval={interval}")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for g in (50, 50):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"interval {interval} generation {ctx.generation}")
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


@pytest.mark.parametrize("variant", ["cellular", "pseudo"])
def test_single_island_full_size(variant):
    """The single 64x128 torus and the single pseudo island of 8192 at full
    size: generation 0 compared whole, then the GPU state after 5
    generations is loaded into the oracle and generations 6 and 7 compared."""
    ensure_built()
    w = inputs.island_variant(variant, seed=1)
    say(f"[islands] {variant} full size")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    assert_same_state(ctx, ga, 0, 1, f"{variant} generation 0")
    ctx.evolve(5)
    genes, mk = ctx.population(0, 0)
    ga.set_population(0, genes, mk)
    ga.set_generation(5)
    for g in (6, 7):
        ctx.evolve(1)
        ga.evolve(1)
        assert_same_state(ctx, ga, 0, 1, f"{variant} generation {g}")
    ctx.close()


@pytest.mark.parametrize("variant", inputs.ISLAND_VARIANTS)
def test_paper_setting_batched_seeds(variant):
    """Section 5's setting (300 jobs, 4 stages, 2 machines, p in [1, 5], 512
    individuals) with four GA seeds as four instances of one context, as the
    ablation experiment runs them; migration every 10; 30 generations."""
    ensure_built()
    ws = []
    for r in range(4):
        w = inputs.paper_setting(variant, interval=10)
        w["seed"] = 1000 + r
        ws.append(w)
    n_isl = len(ws[0]["islands"])
    say(f"[islands] paper setting {variant}, 4 seeds")
    ctx = make_ctx(ws)
    gas = [oracle_ga(w, inst=i) for i, w in enumerate(ws)]
    for g in (10, 20):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, n_isl, f"{variant} seed {1000 + i} generation {ctx.generation}")
    for i, ga in enumerate(gas):
        assert ctx.best(i)["makespan"] == ga.best()["makespan"]
        assert ctx.migration_counters(i) == ga.counters()
    ctx.close()


@pytest.mark.parametrize("sel", [1, 2])
@pytest.mark.parametrize("variant", ["dual", "cellular2"])
def test_selection_variants_trajectory(variant, sel):
    """Parent selection variants (1: self + best neighbour, 2: binary
    tournaments) on the medium instance's layouts at 1/8 of the side, and in
    Section 5's setting with two GA seeds as two instances; 25 generations."""
    ensure_built()
    w = inputs.island_variant(variant, seed=1, scale=8, interval=10)
    for x in w["islands"]:
        if x["kind"] == 0:
            x["sel"] = sel
    ws = [w]
    for r in range(2):
        v = inputs.paper_setting(variant, interval=10, sel=sel)
        v["seed"] = 2000 + r
        ws.append(v)
    n_isl = len(w["islands"])
    say(f"[islands] {variant} selection {sel}")
    ctx = make_ctx(ws)
    gas = [oracle_ga(v, inst=i) for i, v in enumerate(ws)]
    for g in (5, 20):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, n_isl, f"{variant} sel {sel} instance {i} generation {ctx.generation}")
    for i, ga in enumerate(gas):
        assert ctx.best(i)["makespan"] == ga.best()["makespan"]
    ctx.close()


@pytest.mark.parametrize("n_pairs", [1, 2, 8])
def test_ring_edge_topology(n_pairs):
    """Topology 2 (the penetration rule on every ring edge in turn) with 2, 4
    and 16 islands, against the oracle; with a topology-1 instance of the
    same shape in the same context, 40 generations and one forced epoch."""
    ensure_built()
    m, p = inputs.make_instance(60, 4, 1, 4, seed=9)
    isl = [inputs.cellular(4, 4, 0.9, 0.1) for _ in range(n_pairs)] + \
          [inputs.pseudo(16, 0.75, 0.05) for _ in range(n_pairs)]
    ws = [dict(m=m, p=p, islands=isl, interval=5, topology=2, seed=31),
          dict(m=m, p=p, islands=isl, interval=5, topology=1, seed=32)]
    n_isl = len(isl)
    say(f"[islands] ring-edge topology, {n_isl} islands")
    ctx = make_ctx(ws)
    gas = [oracle_ga(v, inst=i) for i, v in enumerate(ws)]
    for g in (5, 15, 20):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, n_isl, f"topology {ws[i]['topology']} generation {ctx.generation}")
    ctx.migrate(0)
    gas[0].migrate()
    for i, ga in enumerate(gas):
        assert_same_state(ctx, ga, i, n_isl, f"topology {ws[i]['topology']} after forced epoch")
        assert ctx.migration_counters(i) == ga.counters()
        assert ctx.best(i)["makespan"] == ga.best()["makespan"]
    ctx.close()
