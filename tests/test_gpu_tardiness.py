"""GPU parity of the paper-faithful variant (include/ffs_tt.h) against its
oracle: decodes of caller-supplied assignments and whole GA trajectories,
bit-exact (int64 objectives in hundredths, machine indices)."""
import numpy as np
import pytest

from gpu_util import ensure_built, say
from oracle import tardiness as ot
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu


def _ctx(inst, islands, interval, runs=1, seed=101):
    from paper_1903_10722_amd.tardiness import TtContext
    return TtContext(inst, islands, interval=interval, theta=1.0, seed=seed, runs=runs)


def _random_genes(inst, count, seed):
    rng = np.random.default_rng(seed)
    M = np.asarray(inst["M"])
    S = len(M)
    J = inst["P"].shape[0]
    return (rng.random((count, J * S)) * np.tile(M, J)).astype(np.int32)


@pytest.mark.parametrize("shape", [(300, 4, [2, 2, 2, 2]), (37, 3, [1, 3, 4]), (1, 2, [2, 1]), (64, 2, [4, 2]),
                                   (65, 5, [2, 3, 1, 4, 2]), (1024, 2, [2, 2]), (130, 7, [3, 1, 2, 4, 1, 2, 3])])
def test_decode_matches_oracle(shape):
    ensure_built()
    J, S, M = shape
    inst = inputs.tardiness_instance(J, S, M, seed=J + S)
    say(f"[tt] decode J={J} S={S} M={M}")
    ctx = _ctx(inst, [inputs.pseudo(2, 0.75, 0.0)], interval=0)
    genes = _random_genes(inst, 96, seed=J)
    got = ctx.evaluate(genes).cpu().numpy()
    want = np.array([ot.decode(inst, g)[0] for g in genes], dtype=np.int64)
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:10]
    ctx.close()


def test_decode_rejects_out_of_range_genes():
    ensure_built()
    inst = inputs.tardiness_instance(20, 3, [2, 3, 1], seed=3)
    ctx = _ctx(inst, [inputs.pseudo(2, 0.75, 0.0)], interval=0)
    genes = _random_genes(inst, 4, seed=1)
    genes[1, 5] = 3          # stage 2 has 3 machines: 3 is out of range
    genes[3, 2] = 1          # stage 3 has 1 machine
    got = ctx.evaluate(genes).cpu().numpy()
    assert got[1] == -1 and got[3] == -1
    assert got[0] == ot.decode(inst, genes[0])[0] and got[2] == ot.decode(inst, genes[2])[0]
    ctx.close()


def _same(ctx, ga, run, n_isl, what):
    for i in range(n_isl):
        g1, o1 = ctx.population(run, i)
        g2, o2 = ga.population(i)
        if not np.array_equal(o1, o2):
            bad = np.nonzero(o1 != o2)[0]
            raise AssertionError(f"{what} island {i}: objectives differ at {bad[:8]} gpu={o1[bad[:4]]} oracle={o2[bad[:4]]}")
        assert np.array_equal(g1, g2), f"{what} island {i}: genes differ"


@pytest.mark.parametrize("runs", [1, 3])
def test_small_trajectory_with_migration(runs):
    ensure_built()
    inst = inputs.tardiness_instance(20, 3, [2, 3, 1], seed=5)
    isl = [inputs.cellular(6, 6, 1.0, 0.05), inputs.pseudo(36, 0.75, 0.1)]
    say(f"[tt] small trajectory runs={runs}")
    ctx = _ctx(inst, isl, interval=5, runs=runs, seed=11)
    gas = [ot.GA(inst, isl, interval=5, seed=11, inst_id=r) for r in range(runs)]
    for r, ga in enumerate(gas):
        _same(ctx, ga, r, 2, f"run {r} generation 0")
    done = 0
    for chunk in (1, 4, 5, 7, 13):
        ctx.evolve(chunk)
        done += chunk
        for r, ga in enumerate(gas):
            ga.evolve(chunk)
            _same(ctx, ga, r, 2, f"run {r} generation {done}")
            b1, b2 = ctx.best(r), ga.best()
            assert (b1["objective"], b1["generation"], b1["island"], b1["slot"]) == \
                   (b2["objective"], b2["generation"], b2["island"], b2["slot"])
            assert np.array_equal(b1["genes"], b2["genes"])
            assert ctx.counters(r) == ga.counters()
    ctx.close()


def test_section5_size_trajectory():
    """Section 5's sizes: 300 jobs, 4 stages, 2 unrelated machines each, a
    16x16 cellular island and a pseudo island of 256 (rates 1.00 / 0.05 and
    0.75), migration every 10 generations here so that epochs are covered."""
    ensure_built()
    w = inputs.tardiness_setting("dual", seed=1)
    say("[tt] section-5 size trajectory")
    ctx = _ctx(w["inst"], w["islands"], interval=10, seed=3)
    ga = ot.GA(w["inst"], w["islands"], interval=10, seed=3)
    _same(ctx, ga, 0, 2, "generation 0")
    for g in (9, 1, 10, 15):
        ctx.evolve(g)
        ga.evolve(g)
        _same(ctx, ga, 0, 2, f"generation {ga.generation}")
    assert ctx.best(0)["objective"] == ga.best()["objective"]
    assert ctx.counters(0) == ga.counters()
    ctx.close()


def test_forced_migration_and_restored_state():
    ensure_built()
    inst = inputs.tardiness_instance(30, 4, [2, 2, 3, 2], seed=9)
    isl = [inputs.cellular(4, 5, 1.0, 0.05), inputs.pseudo(20, 0.75, 0.0),
           inputs.cellular(3, 4, 0.9, 0.1), inputs.pseudo(12, 0.5, 0.05)]
    say("[tt] four islands, forced epoch, restored state")
    ctx = _ctx(inst, isl, interval=0, seed=5)
    ga = ot.GA(inst, isl, interval=0, seed=5)
    ctx.evolve(6)
    ga.evolve(6)
    _same(ctx, ga, 0, 4, "generation 6")
    ctx.migrate()
    ga.migrate()
    _same(ctx, ga, 0, 4, "forced epoch")
    assert ctx.counters(0) == ga.counters()
    # a state taken from the GPU, loaded into the oracle at another generation
    ctx.set_generation(11)
    ga.set_generation(11)
    ctx.evolve(3)
    ga.evolve(3)
    _same(ctx, ga, 0, 4, "after restore")
    ctx.close()


def test_theta_below_one_and_largest_islands():
    """theta = 0.3 (the threshold branch of equation (1) in exact 128-bit
    arithmetic) on islands of 4096 (the largest sort span), four machines at
    one stage."""
    ensure_built()
    inst = inputs.tardiness_instance(12, 3, [4, 2, 1], seed=12)
    isl = [inputs.cellular(64, 64, 1.0, 0.05), inputs.pseudo(4096, 0.75, 0.05)]
    say("[tt] theta 0.3, islands of 4096")
    from paper_1903_10722_amd.tardiness import TtContext
    ctx = TtContext(inst, isl, interval=4, theta=0.3, seed=21, runs=1)
    ga = ot.GA(inst, isl, interval=4, theta=0.3, seed=21)
    for g in (4, 4, 3):
        ctx.evolve(g)
        ga.evolve(g)
        _same(ctx, ga, 0, 2, f"generation {ga.generation}")
    assert ctx.counters(0) == ga.counters()
    ctx.close()


def test_state_loaded_from_the_oracle():
    """ffs_tt_set_population: a state the oracle reached, loaded into the GPU
    context, evolves identically on both sides."""
    ensure_built()
    inst = inputs.tardiness_instance(40, 4, [2, 3, 2, 1], seed=13)
    isl = [inputs.cellular(5, 6, 1.0, 0.1), inputs.pseudo(30, 0.75, 0.1)]
    say("[tt] state loaded from the oracle")
    ga = ot.GA(inst, isl, interval=6, seed=31)
    ga.evolve(9)
    ctx = _ctx(inst, isl, interval=6, seed=31)
    ctx.set_generation(9)
    for i in range(2):
        g, o = ga.population(i)
        ctx.set_population(0, i, g, o)
    _same(ctx, ga, 0, 2, "loaded")
    ctx.evolve(8)
    ga.evolve(8)
    _same(ctx, ga, 0, 2, "after 8 generations")
    ctx.close()


@pytest.mark.parametrize("runs", [1, 2])
def test_line_sweep_trajectory(runs):
    """The asynchronous line-sweep update (one launch per anti-diagonal) on a
    6x5 cellular island beside a pseudo island, with migration, then a switch
    back to the synchronous update; every chunk bit-exact."""
    ensure_built()
    inst = inputs.tardiness_instance(24, 3, [2, 3, 2], seed=17)
    isl = [inputs.cellular(6, 5, 1.0, 0.1), inputs.pseudo(30, 0.75, 0.05)]
    say(f"[tt] line sweep runs={runs}")
    from paper_1903_10722_amd.tardiness import TtContext
    ctx = TtContext(inst, isl, interval=4, theta=1.0, seed=23, runs=runs, sweep=True)
    gas = [ot.GA(inst, isl, interval=4, seed=23, inst_id=r, sweep=True) for r in range(runs)]
    for chunk in (1, 3, 4, 6):
        ctx.evolve(chunk)
        for r, ga in enumerate(gas):
            ga.evolve(chunk)
            _same(ctx, ga, r, 2, f"run {r} sweep generation {ga.generation}")
            assert ctx.best(r)["objective"] == ga.best()["objective"]
    ctx.lib.ffs_tt_set_update(ctx._h, 0)
    for ga in gas:
        ga._lib.or_tt_ga_set_update(ga._h, 0)
    ctx.evolve(3)
    for r, ga in enumerate(gas):
        ga.evolve(3)
        _same(ctx, ga, r, 2, f"run {r} synchronous again")
    ctx.close()


def test_line_sweep_section5_size():
    ensure_built()
    w = inputs.tardiness_setting("dual", seed=1)
    say("[tt] line sweep at section-5 size")
    from paper_1903_10722_amd.tardiness import TtContext
    ctx = TtContext(w["inst"], w["islands"], interval=10, seed=3, sweep=True)
    ga = ot.GA(w["inst"], w["islands"], interval=10, seed=3, sweep=True)
    for g in (5, 7):
        ctx.evolve(g)
        ga.evolve(g)
        _same(ctx, ga, 0, 2, f"generation {ga.generation}")
    ctx.close()


def test_argument_errors_are_reported():
    """Invalid instances, islands and call orders give the documented status
    and leave the context usable."""
    ensure_built()
    import ctypes
    from paper_1903_10722_amd import binding
    from paper_1903_10722_amd.tardiness import load
    lib = load()
    h = ctypes.c_void_p()
    assert lib.ffs_tt_create(None, ctypes.byref(h)) == binding.FFS_OK
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)

    def inst_rc(J, S, M, MX, P, R, D, WT=100):
        M, P, R = (np.ascontiguousarray(x, dtype=np.int32) for x in (M, P, R))
        D = np.ascontiguousarray(D, dtype=np.int64)
        return lib.ffs_tt_set_instance(h, J, S, M.ctypes.data_as(i32p), MX, P.ctypes.data_as(i32p),
                                       R.ctypes.data_as(i32p), D.ctypes.data_as(i64p), WT)

    good = inputs.tardiness_instance(5, 2, [2, 1], seed=1)
    P = good["P"].copy()
    P[0, 0, 1] = 0
    assert inst_rc(5, 2, good["M"], 2, P, good["R"], good["D"]) == binding.FFS_EINVAL           # p < 1
    assert inst_rc(5, 2, [2, 1], 3, np.ones((5, 2, 3)), good["R"], good["D"]) == binding.FFS_EINVAL   # MX != max M
    assert inst_rc(1100, 1, [1], 1, np.ones((1100, 1, 1)), np.zeros(1100), np.zeros(1100)) == binding.FFS_EUNSUPPORTED
    assert inst_rc(5, 2, good["M"], 2, good["P"], good["R"], good["D"]) == binding.FFS_OK
    odd = binding.IslandSpec(1, 0, 0, 7, 0.75, 0.0, 0)
    assert lib.ffs_tt_add_island(h, ctypes.byref(odd)) == binding.FFS_EINVAL                      # odd pseudo size
    sel = binding.IslandSpec(0, 4, 4, 16, 1.0, 0.05, 2)
    assert lib.ffs_tt_add_island(h, ctypes.byref(sel)) == binding.FFS_EINVAL                      # selection != 0
    assert lib.ffs_tt_evolve(h, 1) == binding.FFS_ESTATE                                          # before bind
    assert lib.ffs_tt_set_update(h, 2) == binding.FFS_EINVAL
    assert b"update mode" in lib.ffs_tt_last_error(h)
    assert lib.ffs_tt_destroy(h) == binding.FFS_OK


@pytest.mark.parametrize("machines", [[2, 3], [2, 2]])
def test_trajectory_above_512_jobs(machines):
    """More than 512 jobs: the decode's 16-positions-per-lane instantiations
    (up to 4 and up to 2 machines per stage) inside the generation kernel,
    with migration and the line sweep."""
    ensure_built()
    inst = inputs.tardiness_instance(600, 2, machines, seed=29)
    isl = [inputs.cellular(4, 4, 1.0, 0.1), inputs.pseudo(16, 0.75, 0.05)]
    say("[tt] J=600 trajectory")
    from paper_1903_10722_amd.tardiness import TtContext
    for sweep in (False, True):
        ctx = TtContext(inst, isl, interval=3, seed=41, sweep=sweep)
        ga = ot.GA(inst, isl, interval=3, seed=41, sweep=sweep)
        _same(ctx, ga, 0, 2, f"sweep={sweep} generation 0")
        ctx.evolve(4)
        ga.evolve(4)
        _same(ctx, ga, 0, 2, f"sweep={sweep} generation 4")
        ctx.close()
