"""GPU parity of the decode entry point (ffs_evaluate) against the oracle.

Bit-exact int32 makespans on seeded random permutations at every workload
shape (several tiles and a ragged tail), plus the edge cases: one job, one
stage, single-machine stages, 16 machines, processing times above 255,
64 stages, and rows that are not permutations."""
import numpy as np
import pytest

import oracle
from gpu_util import ensure_built, make_ctx, say
from paper_1903_10722_amd import inputs

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
    ("sixteen_machines", 50, 3, 1, 16, [16, 1, 7], 99, 300, 300),
    ("wide_p", 60, 4, 1, 4, None, 5000, 300, 300),
    # processing times of 1-3 (1-2): equal completions everywhere, so the order among them (dispatch
    # order, the keys' tie-break) decides most dispatches; both fit the three-field keys
    ("tie_heavy", 300, 6, 1, 4, None, 3, 2001, 600),
    ("tie_heavy_wide_lists", 64, 4, 5, 8, None, 2, 1500, 1500),
    ("sixty_four_stages", 12, 64, 1, 3, None, 99, 150, 150),
    ("more_jobs_than_lds_groups", 2000, 3, 1, 4, None, 20, 50, 20),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[s[0] for s in SHAPES])
def test_decode_parity(shape):
    ensure_built()
    name, n, S, lo, hi, machines, p_hi, count, checked = shape
    w = _inst(n, S, lo, hi, seed=11 + n + S, machines=machines, p_hi=p_hi)
    say(f"[decode] shape={name} n={n} S={S} m={w['m'].tolist()} count={count}")
    ctx = make_ctx([w])
    perms = inputs.random_perms(count, n, seed=5 + n)
    got = ctx.evaluate(0, perms).cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.arange(count) if checked >= count else np.sort(rng.choice(count, checked, replace=False))
    idx = np.union1d(idx, [0, count - 1])
    want = oracle.decode_many(w["m"], w["p"], perms[idx])
    assert np.array_equal(got[idx], want), f"first mismatch at row {idx[np.argmax(got[idx] != want)]}"
    lb = oracle.lower_bound(w["m"], w["p"])
    assert (got >= lb).all() and (got <= int(w["p"].sum())).all()
    ctx.close()


def test_decode_tile_shapes_agree():
    """Every waves-per-block tile gives the same makespans."""
    ensure_built()
    w = _inst(100, 5, 1, 5, seed=3)
    perms = inputs.random_perms(1000, 100, seed=9)
    ref = None
    for wpb in (1, 2, 4, 8):
        say(f"[decode] tile waves_per_block={wpb}")
        ctx = make_ctx([w], waves_per_block=wpb)
        got = ctx.evaluate(0, perms).cpu().numpy()
        ctx.close()
        if ref is None:
            ref = got
            assert np.array_equal(ref, oracle.decode_many(w["m"], w["p"], perms))
        assert np.array_equal(got, ref)


def test_decode_rejects_non_permutations():
    ensure_built()
    from paper_1903_10722_amd.binding import FFS_EINVAL
    w = _inst(30, 4, 1, 3, seed=4)
    perms = inputs.random_perms(200, 30, seed=2)
    bad = perms.copy()
    bad[3, 5] = bad[3, 6]            # duplicate
    bad[50, 0] = 30                  # out of range
    bad[51, 7] = -1                  # negative
    bad[199, :] = 0                  # all equal
    say("[decode] invalid rows")
    ctx = make_ctx([w])
    out, rc = ctx.evaluate(0, bad, check=False)
    out = out.cpu().numpy()
    assert rc == FFS_EINVAL
    for r in (3, 50, 51, 199):
        assert out[r] == -1
    good = np.setdiff1d(np.arange(200), [3, 50, 51, 199])
    assert np.array_equal(out[good], oracle.decode_many(w["m"], w["p"], bad[good]))
    # the error does not stick: a clean call afterwards succeeds
    ok = ctx.evaluate(0, perms).cpu().numpy()
    assert np.array_equal(ok, oracle.decode_many(w["m"], w["p"], perms))
    # empty input is a no-op
    assert ctx.evaluate(0, perms[:0]).numel() == 0
    ctx.close()


def test_instances_outside_limits_are_refused():
    ensure_built()
    from paper_1903_10722_amd import Context
    from paper_1903_10722_amd.binding import FFSError
    ctx = Context(device=0)
    m, p = inputs.make_instance(10, 3, 1, 2, seed=1)
    with pytest.raises(FFSError):
        ctx.add_instance(m, p * 0, SMALL_ISLANDS, interval=0)              # p = 0
    with pytest.raises(FFSError):
        ctx.add_instance(np.array([1, 17, 1]), p, SMALL_ISLANDS, interval=0)  # 17 machines
    with pytest.raises(FFSError):
        ctx.add_instance(m, p, [inputs.cellular(2, 5, 0.9, 0.1), inputs.pseudo(2, 0.7, 0)], interval=0)
    with pytest.raises(FFSError):
        ctx.add_instance(m, p, [inputs.cellular(3, 3, 0.9, 0.1), inputs.pseudo(3, 0.7, 0)], interval=0)
    with pytest.raises(FFSError):
        ctx.evolve(1)                                                      # not bound
    ctx.close()


def test_host_pointer_decode_matches_device_decode():
    """ffs_evaluate_host on host rows, in several staging chunks (1500 rows
    of 1000 jobs exceed the 4 MiB staging region), equals the device-pointer
    entry point and the oracle; invalid rows give -1 and FFS_EINVAL."""
    ensure_built()
    from paper_1903_10722_amd.binding import FFS_EINVAL, FFS_OK
    w = _inst(1000, 20, 2, 6, seed=31)
    perms = inputs.random_perms(1500, 1000, seed=7)
    say("[decode] host pointers, 1500 rows of 1000 jobs")
    ctx = make_ctx([w])
    got, rc = ctx.evaluate_host(0, perms)
    assert rc == FFS_OK
    assert np.array_equal(got, ctx.evaluate(0, perms).cpu().numpy())
    idx = np.array([0, 1, 700, 1048, 1049, 1050, 1499])
    assert np.array_equal(got[idx], oracle.decode_many(w["m"], w["p"], perms[idx]))
    bad = perms[:10].copy()
    bad[4, 0] = bad[4, 1]
    out, rc = ctx.evaluate_host(0, bad)
    assert rc == FFS_EINVAL and out[4] == -1
    assert np.array_equal(np.delete(out, 4), np.delete(got[:10], 4))
    ctx.close()
