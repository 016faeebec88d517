"""GPU parity of the lane mapping (one lane decodes one chromosome through
every stage; ffs_set_mapping(1)) against the oracle, and its agreement
with the per-stage mapping.

Decode: bit-exact makespans at every workload shape and at the edge cases
(one job, one stage, single-machine stages, processing times above 255,
rows shorter than a window, a flush that spans two windows), and rows
that are not permutations.  Generation loop: whole trajectories of the
tiny workload, the scaled medium and large ones and uneven batched
instances, every tile width, a mapping switched mid-run."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_state, ensure_built, make_ctx, oracle_ga, say
from paper_1903_10722_amd import inputs
from paper_1903_10722_amd.binding import FFSError

pytestmark = pytest.mark.gpu

SMALL_ISLANDS = [inputs.cellular(3, 3, 0.9, 0.1), inputs.pseudo(2, 0.75, 0.0)]


def _inst(n, S, m_lo, m_hi, seed, machines=None, p_hi=99):
    m, p = inputs.make_instance(n, S, m_lo, m_hi, p_hi=p_hi, seed=seed, machines=machines)
    return dict(m=m, p=p, islands=SMALL_ISLANDS, interval=0)


SHAPES = [
    # name, n, S, m_lo, m_hi, machines, p_hi, count, checked
    ("tiny", 20, 3, 2, 2, [2, 2, 2], 99, 3001, 3001),
    ("medium", 100, 5, 1, 5, None, 99, 4099, 1500),
    ("large", 500, 10, 3, 5, None, 99, 1031, 300),
    ("surrogate", 1000, 20, 2, 6, None, 99, 517, 60),
    ("batched_n20_S20", 20, 20, 1, 5, None, 99, 777, 777),
    ("batched_n500_S5", 500, 5, 1, 5, None, 99, 613, 200),
    ("batched_n200_S10", 200, 10, 1, 5, None, 99, 611, 200),
    ("one_job", 1, 4, 1, 3, None, 99, 70, 70),
    ("one_stage", 37, 1, 3, 3, [3], 99, 300, 300),
    ("single_machines", 40, 6, 1, 1, [1] * 6, 99, 300, 300),
    ("eight_machines", 50, 3, 1, 8, [8, 1, 7], 99, 300, 300),
    ("wide_p", 60, 4, 1, 4, None, 5000, 300, 300),
    # processing times of 1-3 (1-2): equal completions everywhere, so the order among them (dispatch
    # order, the keys' tie-break) decides most dispatches; both fit the three-field keys
    ("tie_heavy", 300, 6, 1, 4, None, 3, 2001, 600),
    ("tie_heavy_wide_lists", 64, 4, 5, 8, None, 2, 1500, 1500),
    ("short_rows", 5, 7, 1, 4, None, 99, 200, 200),
    ("flush_spans_windows", 17, 3, 5, 8, [8, 7, 6], 99, 300, 300),
    ("many_stages", 12, 40, 1, 3, None, 99, 150, 150),
    ("long_rows", 2000, 3, 1, 4, None, 20, 130, 20),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[s[0] for s in SHAPES])
def test_lane_decode_parity(shape):
    ensure_built()
    name, n, S, lo, hi, machines, p_hi, count, checked = shape
    w = _inst(n, S, lo, hi, seed=13 + n + S, machines=machines, p_hi=p_hi)
    assert int(w["m"].sum()) <= 160 and int(w["m"].max()) <= 8
    say(f"[lane] decode shape={name} n={n} S={S} m={w['m'].tolist()} count={count}")
    ctx = make_ctx([w], mapping=1)
    perms = inputs.random_perms(count, n, seed=7 + n)
    got = ctx.evaluate(0, perms).cpu().numpy()
    rng = np.random.default_rng(2)
    idx = np.arange(count) if checked >= count else np.sort(rng.choice(count, checked, replace=False))
    idx = np.union1d(idx, [0, count - 1])
    want = oracle.decode_many(w["m"], w["p"], perms[idx])
    assert np.array_equal(got[idx], want), f"first mismatch at row {idx[np.argmax(got[idx] != want)]}"
    ctx.close()


def test_lane_decode_key_overflow_falls_back():
    """The three-field key (completion, dispatch index, job) holds
    completions below 2^(32 - 2 jb): 16384 at n = 300.  Three job types,
    each with processing time 60 on its own stage and 1 elsewhere, one
    machine per stage: the lower bound is 6200, so the instance takes the
    three-field key, but permutations sorted by type take about 18000.  Rows
    of both kinds share waves; every makespan matches the oracle (the lanes
    past the limit are decoded again with the two-field key)."""
    ensure_built()
    n, S = 300, 3
    m = np.ones(S, dtype=np.int32)
    p = np.ones((n, S), dtype=np.int32)
    p[np.arange(n), np.arange(n) % S] = 60
    lb = max(int(p.sum(1).max()), int(p.sum(0).max()))
    jb = int(np.ceil(np.log2(n)))
    assert 3 * lb < 2 * (1 << (32 - 2 * jb))       # the three-field key is taken
    rng = np.random.default_rng(11)
    by_type = np.argsort(np.arange(n) % S, kind="stable")
    rows = []
    for r in range(256):
        if r % 5 == 0:
            q = by_type.copy()
            # a few swaps keep it far above the limit
            for _ in range(3):
                a, b = rng.integers(0, n, 2)
                q[a], q[b] = q[b], q[a]
            rows.append(q)
        else:
            rows.append(rng.permutation(n))
    perms = np.asarray(rows, dtype=np.int32)
    want = oracle.decode_many(m, p, perms)
    assert (want[::5] > 16384).all() and (want[1::5] < 16384).all()
    w = dict(m=m, p=p, islands=SMALL_ISLANDS, interval=0)
    say("[lane] key overflow fallback n=300")
    ctx = make_ctx([w], mapping=1)
    got = ctx.evaluate(0, perms).cpu().numpy()
    assert np.array_equal(got, want), f"first mismatch at row {np.argmax(got != want)}"
    ctx.close()


def test_lane_decode_rejects_non_permutations():
    """Out-of-range values and repeated values give -1 on their rows only."""
    ensure_built()
    w = _inst(30, 4, 1, 4, seed=5)
    ctx = make_ctx([w], mapping=1)
    perms = inputs.random_perms(200, 30, seed=3)
    perms[7, 4] = 30
    perms[50, 0] = -1
    perms[51, 3] = perms[51, 9]
    perms[199, 29] = perms[199, 0]
    from paper_1903_10722_amd.binding import FFS_EINVAL
    say("[lane] invalid rows")
    with pytest.raises(FFSError):
        ctx.evaluate(0, perms)
    out, rc = ctx.evaluate(0, perms, check=False)
    assert rc == FFS_EINVAL
    got = out.cpu().numpy()
    bad = [7, 50, 51, 199]
    assert (got[bad] == -1).all()
    ok = np.setdiff1d(np.arange(200), bad)
    assert np.array_equal(got[ok], oracle.decode_many(w["m"], w["p"], perms[ok]))
    # the flag is cleared: a clean call succeeds
    clean = inputs.random_perms(64, 30, seed=4)
    assert np.array_equal(ctx.evaluate(0, clean).cpu().numpy(), oracle.decode_many(w["m"], w["p"], clean))
    ctx.close()


@pytest.mark.parametrize("inst_seed", [1, 2])
def test_lane_tiny_trajectory(inst_seed):
    """Tiny workload (8x8 cellular + 64 pseudo, n=20, S=3) on the lane
    mapping: 100 generations, migration every 10, compared after every chunk
    with the best-ever record."""
    ensure_built()
    w = inputs.workload("tiny", seed=inst_seed)
    say(f"[lane] tiny inst_seed={inst_seed}")
    ctx = make_ctx([w], mapping=1)
    assert ctx.mapping() == 1
    ga = oracle_ga(w)
    assert_same_state(ctx, ga, 0, 2, "generation 0")
    done = 0
    for chunk in [1, 4, 5, 10, 20, 60]:
        ctx.evolve(chunk)
        ga.evolve(chunk)
        done += chunk
        assert_same_state(ctx, ga, 0, 2, f"generation {done}")
        b1, b2 = ctx.best(0), ga.best()
        assert (b1["makespan"], b1["generation"]) == (b2["makespan"], b2["generation"])
        assert b1["perm"].tolist() == b2["perm"].tolist()
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


@pytest.mark.parametrize("n", [20, 500, 520])
def test_lane_odd_counts(n):
    """Islands whose waves hold an odd number of chromosomes (a 7x9 torus,
    30 pairs) on the lane mapping, with rows of 32, 512 and 544 genes: 30
    generations with adaptive migration every 10, compared with the oracle
    after every chunk."""
    ensure_built()
    m, p = inputs.make_instance(n, 6, 1, 4, seed=7)
    isl = [inputs.cellular(7, 9, 0.9, 0.2), inputs.pseudo(30, 0.75, 0.05)]
    w = dict(m=m, p=p, islands=isl, interval=10, theta=1.0, topology=0)
    say(f"[lane] odd counts n={n}")
    ctx = make_ctx([w], mapping=1)
    assert ctx.mapping() == 1
    ga = oracle_ga(w)
    for g in (1, 9, 10, 10):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"n={n} generation {ctx.generation}")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


def test_lane_medium_scaled_trajectory():
    """Medium instance (n=100, S=5, m in [1,5]) on 32x32 + 1024 islands,
    60 generations with adaptive migration every 20, lane mapping."""
    ensure_built()
    w = inputs.workload("medium", seed=1, scale=2)
    say("[lane] medium scale=2")
    ctx = make_ctx([w], mapping=1)
    ga = oracle_ga(w)
    for g in (19, 1, 20, 20):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"generation {ctx.generation}")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


def test_lane_sixteen_islands_and_long_rows():
    """Large instance (n=500, S=10) on 16 islands of 64 with ring-then-
    adaptive migration, and the n=1000, S=20 instance on 8x8 + 64: 40
    generations each on the lane mapping, compared at every epoch."""
    ensure_built()
    for w, nis in ((inputs.workload("large", seed=1, scale=16), 16),
                   (inputs.workload("surrogate", seed=2, scale=8), 2)):
        say(f"[lane] n={w['p'].shape[0]} S={w['p'].shape[1]} islands={nis}")
        ctx = make_ctx([w], mapping=1)
        ga = oracle_ga(w)
        for g in (20, 20):
            ctx.evolve(g)
            ga.evolve(g)
            assert_same_state(ctx, ga, 0, nis, f"generation {ctx.generation}")
        assert ctx.best(0)["makespan"] == ga.best()["makespan"]
        ctx.close()


def test_lane_batched_uneven_instances():
    """Eight uneven batched instances (n up to 500, S up to 20, grids shrunk
    eightfold) in one lane-mapped context, 20 generations with migration
    every 10, each compared with its oracle run."""
    ensure_built()
    ws = inputs.batched_workloads(count=8, batch_seed=7, scale=8)
    say("[lane] batched 8 instances")
    ctx = make_ctx(ws, mapping=1)
    assert ctx.mapping() == 1
    ctx.evolve(20)
    for i, w in enumerate(ws):
        ga = oracle_ga(w, inst=i)
        ga.evolve(20)
        assert_same_state(ctx, ga, i, 2, f"instance {i} n={w['p'].shape}")
        assert ctx.best(i)["makespan"] == ga.best()["makespan"]
    ctx.close()


def test_lane_tiles_and_mapping_switch_agree():
    """Medium instance on 16x16 + 256: the per-stage mapping and the lane
    mapping at 1, 2, 4 and 8 waves per workgroup give the same trajectory,
    and so does a run that switches mapping after bind."""
    ensure_built()
    w = inputs.workload("medium", seed=3, scale=4)
    ref = None
    for mapping, wpb in ((0, 4), (1, 1), (1, 2), (1, 4), (1, 8)):
        say(f"[lane] mapping={mapping} waves_per_block={wpb}")
        ctx = make_ctx([w], mapping=mapping, waves_per_block=wpb)
        assert ctx.mapping() == mapping
        ctx.evolve(25)
        state = [ctx.population(0, i) for i in range(2)]
        best = ctx.best(0)
        ctx.close()
        if ref is None:
            ref = (state, best)
            continue
        for i in range(2):
            assert np.array_equal(state[i][0], ref[0][i][0]) and np.array_equal(state[i][1], ref[0][i][1])
        assert best["makespan"] == ref[1]["makespan"] and best["perm"].tolist() == ref[1]["perm"].tolist()
    ctx = make_ctx([w], mapping=0)
    ctx.evolve(9)
    ctx.set_mapping(1)
    assert ctx.mapping() == 1
    ctx.evolve(16)
    for i in range(2):
        g, m = ctx.population(0, i)
        assert np.array_equal(g, ref[0][i][0]) and np.array_equal(m, ref[0][i][1])
    ctx.close()


def test_automatic_mapping_choice():
    """Automatic mapping: per lane for the large workload's 262144
    individuals, per stage for the medium one's 8192 and whenever a stage
    has more than 8 machines."""
    ensure_built()
    big = inputs.workload("large", seed=1)
    ctx = make_ctx([big])
    assert ctx.mapping() == 1
    ctx.close()
    ctx = make_ctx([inputs.workload("medium", seed=1)])
    assert ctx.mapping() == 0
    ctx.close()
    w = _inst(50, 3, 1, 16, seed=3, machines=[16, 1, 7])
    ctx = make_ctx([w], mapping=1)
    assert ctx.mapping() == 0
    ctx.close()


def test_instance_tiles_and_concurrent_classes():
    """Eight uneven batched instances (grids shrunk eightfold) with a tile
    each (both mappings, 1 to 8 waves per workgroup): every instance follows
    its oracle trajectory over 20 generations with migration every 10, and
    running the launches one after another gives the same state."""
    ensure_built()
    ws = inputs.batched_workloads(count=8, batch_seed=7, scale=8)
    tiles = [(1, 4), (0, 2), (1, 1), (0, 8), (1, 8), (0, 1), (1, 2), (0, 4)]
    states = []
    for concurrent in (True, False):
        say(f"[lane] instance tiles, concurrent={concurrent}")
        from paper_1903_10722_amd import Context
        ctx = Context(device=0)
        for w in ws:
            ctx.add_instance(w["m"], w["p"], w["islands"], interval=w["interval"], seed=101)
        for i, (m, wv) in enumerate(tiles):
            ctx.set_instance_tile(i, m, wv)
        ctx.set_concurrent(concurrent)
        ctx.bind()
        assert ctx.mapping() == 2
        ctx.evolve(20)
        states.append([[ctx.population(i, x) for x in range(2)] for i in range(len(ws))])
        if concurrent:
            for i, w in enumerate(ws):
                ga = oracle_ga(w, inst=i)
                ga.evolve(20)
                assert_same_state(ctx, ga, i, 2, f"instance {i} tile {tiles[i]}")
                assert ctx.best(i)["makespan"] == ga.best()["makespan"]
        ctx.close()
    for a, b in zip(states[0], states[1]):
        for (g1, m1), (g2, m2) in zip(a, b):
            assert np.array_equal(g1, g2) and np.array_equal(m1, m2)


def test_instance_tile_change_after_bind():
    """Re-tiling one instance of a bound context mid-run keeps the trajectory."""
    ensure_built()
    ws = inputs.batched_workloads(count=3, batch_seed=11, scale=8)
    ctx = make_ctx(ws)
    ctx.evolve(7)
    ctx.set_instance_tile(1, 1, 2)
    ctx.set_instance_tile(2, 0, 1)
    ctx.evolve(8)
    for i, w in enumerate(ws):
        ga = oracle_ga(w, inst=i)
        ga.evolve(15)
        assert_same_state(ctx, ga, i, 2, f"instance {i}")
    ctx.close()


def test_per_shape_autotuner_keeps_trajectories():
    """The per-group tile autotuner picks a tile for each group of instances
    (timed on throwaway contexts holding the whole batch) and applies it; the
    tuned context follows the oracle."""
    ensure_built()
    from paper_1903_10722_amd import Context
    from paper_1903_10722_amd.autotune import autotune_instances
    ws = inputs.batched_workloads(count=4, batch_seed=7, scale=8)
    ctx = Context(device=0)
    for w in ws:
        ctx.add_instance(w["m"], w["p"], w["islands"], interval=w["interval"], seed=101)
    rep = autotune_instances(ctx, generations=2, use_cache=False)
    say(f"[lane] tuned tiles: {[(k, v['tile']) for k, v in rep['groups'].items()]}")
    assert sum(v["instances"] for v in rep["groups"].values()) == len(ws)
    assert rep["ms_per_generation"]["tuned"] <= rep["ms_per_generation"]["automatic"]
    ctx.bind()
    ctx.evolve(12)
    for i, w in enumerate(ws):
        ga = oracle_ga(w, inst=i)
        ga.evolve(12)
        assert_same_state(ctx, ga, i, 2, f"instance {i}")
    ctx.close()
