"""GPU parity of the line-sweep update (an alternative reading of Section
4.2's update schedule: the cells of a cellular island in row-major order, in
place) against the oracle's in-place sweep.  The library runs it as one
launch per anti-diagonal r + c after each generation launch; every state is
compared whole, genes and makespans, at the generations named."""
import numpy as np
import pytest

from gpu_util import assert_same_state, ensure_built, make_ctx, oracle_ga, say
from paper_1903_10722_amd import inputs

pytestmark = pytest.mark.gpu


def _sweep_workload(n, S, rows, cols, pseudo, interval, seed=1, sel=0, mlo=1, mhi=5):
    m, p = inputs.make_instance(n, S, mlo, mhi, seed=seed)
    isl = [inputs.cellular(rows, cols, inputs.CELL_PC, inputs.CELL_PM, sel=sel, sweep=1),
           inputs.pseudo(pseudo, inputs.PAIR_PC, inputs.PAIR_PM)]
    return dict(m=m, p=p, islands=isl, interval=interval, theta=1.0, topology=0)


@pytest.mark.parametrize("mapping", [1, 0])
@pytest.mark.parametrize("sel", [0, 1, 2])
def test_line_sweep_small_trajectory(sel, mapping):
    """A non-square 7 x 11 torus (anti-diagonals of 1 to 7 cells, both wraps)
    beside a pseudo island, generation by generation through two migration
    epochs; the generation launches use the lane or the per-stage mapping."""
    ensure_built()
    w = _sweep_workload(30, 4, 7, 11, 64, interval=6, seed=3, sel=sel)
    say(f"[sweep] 7x11 selection {sel} mapping {mapping}")
    ctx = make_ctx([w], mapping=mapping)
    ctx.set_graphs(False)
    ga = oracle_ga(w)
    assert_same_state(ctx, ga, 0, 2, "generation 0")
    for g in range(1, 14):
        ctx.evolve(1)
        ga.evolve(1)
        assert_same_state(ctx, ga, 0, 2, f"sel {sel} mapping {mapping} generation {g}")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    ctx.close()


def test_line_sweep_medium_size_in_graphs():
    """The medium workload's layout (n = 100, 5 stages, 64 x 64 + 4096) with
    the cellular island swept: one eager generation, then whole migration
    epochs replayed from a captured graph (127 anti-diagonal launches per
    generation inside it), compared at every epoch end and once mid-epoch."""
    ensure_built()
    w = inputs.workload("medium", seed=1)
    w["islands"][0]["sweep"] = 1
    say("[sweep] medium size, graphs")
    ctx = make_ctx([w])
    ga = oracle_ga(w)
    for g in (1, 19, 20, 20, 7):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 2, f"medium sweep generation {ctx.generation}")
    assert ctx.best(0)["makespan"] == ga.best()["makespan"]
    ctx.close()


def test_line_sweep_beside_synchronous_instances():
    """Two instances in one context, one with a swept island (wide rows, 4 x
    40) and one synchronous: each follows its own oracle."""
    ensure_built()
    a = _sweep_workload(50, 6, 4, 40, 96, interval=5, seed=5)
    b = inputs.workload("medium", seed=2, scale=4)
    b["interval"] = 5
    say("[sweep] mixed context")
    ctx = make_ctx([a, b])
    gas = [oracle_ga(a, inst=0), oracle_ga(b, inst=1)]
    for g in (3, 7, 10):
        ctx.evolve(g)
        for i, ga in enumerate(gas):
            ga.evolve(g)
            assert_same_state(ctx, ga, i, 2, f"instance {i} generation {ctx.generation}")
    ctx.close()


def test_line_sweep_rejections():
    from paper_1903_10722_amd import Context
    from paper_1903_10722_amd.binding import FFSError
    ensure_built()
    m, p = inputs.make_instance(20, 3, 1, 3, seed=1)
    ctx = Context(device=0)
    bad_kind = dict(inputs.pseudo(16, 0.5, 0.0), sweep=1)
    with pytest.raises(FFSError):
        ctx.add_instance(m, p, [inputs.cellular(4, 4, 0.9, 0.1), bad_kind], interval=0)
    with pytest.raises(FFSError):
        ctx.add_instance(m, p, [inputs.cellular(4, 4, 0.9, 0.1, sweep=2), inputs.pseudo(16, 0.5, 0.0)], interval=0)
    with pytest.raises(FFSError):
        ctx.add_instance(m, p, [inputs.cellular(4, 4, 0.9, 0.1, sweep=1), inputs.pseudo(16, 0.5, 0.0)], interval=0,
                         surrogate_k=4)
    m9, p9 = inputs.make_instance(20, 3, 9, 9, seed=1)
    with pytest.raises(FFSError):
        ctx.add_instance(m9, p9, [inputs.cellular(4, 4, 0.9, 0.1, sweep=1), inputs.pseudo(16, 0.5, 0.0)], interval=0)
    ctx.close()


def test_line_sweep_sixteen_islands_with_ring():
    """The large workload's layout at 1/16 of the side (8 swept 8 x 8 grids and
    8 pseudo islands, ring-then-adaptive migration every 5 generations),
    generation by generation on the lane mapping (every anti-diagonal launch
    holds all eight swept islands) against the oracle."""
    ensure_built()
    w = inputs.workload("large", seed=3, scale=16)
    w["interval"] = 5
    for x in w["islands"]:
        if x["kind"] == 0:
            x["sweep"] = 1
    say("[sweep] sixteen islands, ring")
    ctx = make_ctx([w], mapping=1)
    ga = oracle_ga(w)
    for g in (1, 4, 1, 5, 5):
        ctx.evolve(g)
        ga.evolve(g)
        assert_same_state(ctx, ga, 0, 16, f"sixteen islands sweep generation {ctx.generation}")
    assert ctx.migration_counters(0) == ga.counters()
    ctx.close()


def test_line_sweep_checkpoint_restore():
    """A checkpoint taken mid-run and restored into a fresh context continues
    the line-sweep trajectory exactly as the uninterrupted run and the oracle
    do."""
    ensure_built()
    w = _sweep_workload(40, 5, 9, 6, 54, interval=4, seed=9, sel=2)
    say("[sweep] checkpoint and restore")
    a = make_ctx([w])
    a.evolve(7)
    image = a.checkpoint()
    a.evolve(9)
    b = make_ctx([w])
    b.restore(image)
    b.evolve(9)
    ga = oracle_ga(w)
    ga.evolve(16)
    assert_same_state(a, ga, 0, 2, "uninterrupted generation 16")
    assert_same_state(b, ga, 0, 2, "restored generation 16")
    assert a.checkpoint() == b.checkpoint()
    a.close()
    b.close()
