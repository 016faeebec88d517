"""Checkpoint and restore of a context (include/ffs.h ffs_checkpoint_*):
a run continued from a restored image follows exactly the trajectory of the
uninterrupted run and of the oracle, on another tile shape too; images of
other instances are refused."""
import numpy as np
import pytest

from gpu_util import assert_same_state, ensure_built, make_ctx, oracle_ga, say
from paper_1903_10722_amd import inputs
from paper_1903_10722_amd.binding import FFSError

pytestmark = pytest.mark.gpu


def _state(ctx, n_inst, n_isl):
    out = []
    for i in range(n_inst):
        pops = [ctx.population(i, x) for x in range(n_isl)]
        b = ctx.best(i)
        out.append((pops, b["makespan"], b["generation"], b["perm"].tolist(), ctx.migration_counters(i)))
    return out


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        for (g1, m1), (g2, m2) in zip(x[0], y[0]):
            assert np.array_equal(g1, g2) and np.array_equal(m1, m2)
        assert x[1:] == y[1:]


def test_restore_continues_the_same_trajectory():
    ensure_built()
    ws = [inputs.workload("medium", seed=2, scale=4), inputs.workload("tiny", seed=3)]
    say("[checkpoint] two instances, save at 23, continue 17")
    a = make_ctx(ws)
    a.evolve(23)
    image = a.checkpoint()
    a.evolve(17)
    want = _state(a, 2, 2)
    a.close()
    b = make_ctx(ws, waves_per_block=2)
    b.evolve(5)                       # a different state, replaced by the image
    b.restore(image)
    assert b.generation == 23
    b.evolve(17)
    _same(_state(b, 2, 2), want)
    # and the oracle agrees with both
    ga = oracle_ga(ws[0])
    ga.evolve(40)
    assert_same_state(b, ga, 0, 2, "oracle at 40")
    b.close()


def test_restore_rejects_other_instances_and_truncated_images():
    ensure_built()
    w1 = inputs.workload("tiny", seed=1)
    w2 = inputs.workload("tiny", seed=2)
    say("[checkpoint] refusals")
    a = make_ctx([w1])
    a.evolve(3)
    image = a.checkpoint()
    b = make_ctx([w2])
    with pytest.raises(FFSError):
        b.restore(image)
    c = make_ctx([w1], seed=102)      # same instance, another GA seed
    with pytest.raises(FFSError):
        c.restore(image)
    with pytest.raises(FFSError):
        a.restore(image[:-1])
    with pytest.raises(FFSError):
        a.restore(b"\0" * len(image))
    # the refused loads left the context as it was
    ga = oracle_ga(w1)
    ga.evolve(3)
    assert_same_state(a, ga, 0, 2, "after refusals")
    for x in (a, b, c):
        x.close()


def test_restore_with_prescreen_state():
    """A pre-screened instance: network parameters, Adam moments and step
    count, replay ring and choices travel in the image."""
    ensure_built()
    from paper_1903_10722_amd import Context
    m, p = inputs.make_instance(40, 5, 2, 6, seed=8)
    isl = [inputs.cellular(8, 8, 0.9, 0.1), inputs.pseudo(64, 0.75, 0.0)]
    say("[checkpoint] pre-screen, save at 6, continue 5")

    def ctx():
        c = Context(device=0)
        c.add_instance(m, p, isl, interval=4, seed=21, surrogate_k=4, surrogate_warmup=2)
        c.bind()
        return c

    a = ctx()
    a.evolve(6)
    image = a.checkpoint()
    a.evolve(5)
    want = (_state(a, 1, 2), a.surrogate_params(), a.surrogate_choices(), a.surrogate_ring(0, 640))
    a.close()
    b = ctx()
    b.restore(image)
    b.evolve(5)
    _same(_state(b, 1, 2), want[0])
    assert np.array_equal(b.surrogate_params(), want[1])
    assert np.array_equal(b.surrogate_choices(), want[2])
    X, t = b.surrogate_ring(0, 640)
    assert np.array_equal(X, want[3][0]) and np.array_equal(t, want[3][1])
    b.close()
