"""Pins of the faithful variant's oracle (machine-assignment genotype,
unrelated machines, release and due dates, WT * sum T + C_max): hand-worked
schedules, schedule invariants, a reduction to the permutation decoder,
closed forms, exhaustive search on a tiny instance, the migration rule and
GA invariants.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import tardiness as tt
from paper_1903_10722_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _inst(M, P, R, D, WT):
    M = np.asarray(M, dtype=np.int32)
    P = np.asarray(P, dtype=np.int32)
    return dict(M=M, P=P, R=np.asarray(R, dtype=np.int32), D=np.asarray(D, dtype=np.int64), WT=WT)


def test_worked_examples():
    ex = json.load(open(os.path.join(HERE, "golden", "tardiness_worked_examples.json")))["examples"]
    for e in ex:
        inst = _inst(e["M"], e["P"], e["R"], e["D"], e["WT"])
        obj, cmax, tard, C = tt.decode(inst, e["genes"])
        assert C.tolist() == e["C"], e["name"]
        assert (obj, cmax, tard) == (e["objective"], e["cmax"], e["tardiness"]), e["name"]


def _schedule_checks(inst, genes, C):
    """Invariants that fix the schedule: capacity, precedence, release, and
    per machine a non-delay first-in-first-out service in arrival order."""
    M, P, R = inst["M"], inst["P"], inst["R"]
    J, S, _ = P.shape
    g = np.asarray(genes).reshape(J, S)
    prev_key = {j: (int(R[j]), j) for j in range(J)}     # arrival key at stage 1
    for s in range(S):
        start = {j: int(C[j, s]) - int(P[j, s, g[j, s]]) for j in range(J)}
        arrive = {j: (int(R[j]) if s == 0 else int(C[j, s - 1])) for j in range(J)}
        for j in range(J):
            assert start[j] >= arrive[j]                      # release / precedence
        for m in range(int(M[s])):
            jobs = [j for j in range(J) if g[j, s] == m]
            # first in, first out: service order = arrival order (ties: previous order)
            by_arrival = sorted(jobs, key=lambda j: (arrive[j], prev_key[j]))
            by_start = sorted(jobs, key=lambda j: start[j])
            assert by_arrival == by_start
            t_free = 0
            for j in by_arrival:
                # non-delay: a job starts as soon as it has arrived and the machine is free
                assert start[j] == max(t_free, arrive[j])
                t_free = int(C[j, s])
        # order key for the next stage: (completion, position in this stage's order)
        order = sorted(range(J), key=lambda j: (arrive[j], prev_key[j]))
        prev_key = {j: (int(C[j, s]), order.index(j)) for j in range(J)}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_schedule_invariants_random(seed):
    inst = inputs.tardiness_instance(12, 3, [2, 3, 1], seed=seed)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        genes = np.array([rng.integers(0, inst["M"][i % 3]) for i in range(12 * 3)], dtype=np.int32)
        obj, cmax, tard, C = tt.decode(inst, genes)
        _schedule_checks(inst, genes, C)
        assert cmax == C[:, -1].max()
        assert tard == int(np.maximum(C[:, -1] - inst["D"], 0).sum())
        assert obj == inst["WT"] * tard + cmax


def test_single_machine_stages_equal_permutation_decoder():
    """With one machine per stage and no release dates, stage 1 runs the jobs
    by index and every stage keeps that order: the permutation oracle's
    makespan for the identity permutation."""
    J, S = 15, 4
    rng = np.random.default_rng(5)
    p = rng.integers(1, 99, size=(J, S)).astype(np.int32)
    inst = _inst([1] * S, p[:, :, None], [0] * J, [10 ** 9] * J, 100)
    obj, cmax, tard, C = tt.decode(inst, np.zeros(J * S, dtype=np.int32))
    want = oracle.decode(np.ones(S, dtype=np.int32), p, np.arange(J, dtype=np.int32))
    assert tard == 0 and obj == cmax == want


def test_closed_forms_single_machine():
    """One stage, one machine, all released at 0: C_max is the sum of p; with
    D = 0 the tardiness is the sum of the prefix sums (index order)."""
    p = np.array([3, 1, 4, 1, 5, 9, 2, 6], dtype=np.int32) * 100
    inst = _inst([1], p[:, None, None], [0] * 8, [0] * 8, 7)
    obj, cmax, tard, C = tt.decode(inst, np.zeros(8, dtype=np.int32))
    assert cmax == p.sum()
    assert tard == int(np.cumsum(p).sum())
    assert obj == 7 * tard + cmax


def test_exhaustive_tiny_and_emax_bound():
    inst = inputs.tardiness_instance(3, 2, [2, 2], seed=4)
    E = tt.emax(inst)
    objs = []
    for genes in itertools.product([0, 1], repeat=6):
        obj, cmax, tard, C = tt.decode(inst, genes)
        _schedule_checks(inst, genes, C)
        assert 0 < obj <= E
        objs.append(obj)
    assert min(objs) < max(objs)


def test_complement_and_two_point():
    inst = inputs.tardiness_instance(5, 3, [2, 3, 1], seed=2)
    x = tt.random_genes(inst, 9, 0, 0, 0)
    y = tt.complement(inst, x)
    assert np.array_equal(tt.complement(inst, y), x)
    M = np.tile(inst["M"], 5)
    assert ((x >= 0) & (x < M)).all() and ((y >= 0) & (y < M)).all()
    assert np.array_equal(y, M - 1 - x)
    # two machines: the complement is the bit complement
    inst2 = inputs.tardiness_instance(5, 3, [2, 2, 2], seed=2)
    x2 = tt.random_genes(inst2, 9, 0, 0, 0)
    assert np.array_equal(tt.complement(inst2, x2), 1 - x2)
    # complementary parents give complementary children
    y2 = tt.complement(inst2, x2)
    for a, b in [(0, 14), (3, 7), (5, 5)]:
        c1 = tt.two_point(x2, y2, a, b)
        c2 = tt.two_point(y2, x2, a, b)
        assert np.array_equal(c1, 1 - c2)
        assert np.array_equal(c1[a:b + 1], x2[a:b + 1])
    assert np.array_equal(tt.two_point(x2, x2, 2, 9), x2)


def test_migration_policy_exact():
    # beta = 600/900: 1 - beta = 1/3 < 1, alpha N = 3 of 9, A (fitter) sends
    assert tt.migration_policy(1000, 100, 400, 9, 9, 1.0) == (3, True)
    # beyond 2^32: fitness 9e11 and 5e11, alpha = 4/9 of 9 = 4, exact
    assert tt.migration_policy(10 ** 12, 10 ** 11, 5 * 10 ** 11, 9, 9, 1.0) == (4, True)
    # B fitter; ceil(alpha N): alpha = 1/10 of 25 = 2.5 -> 3
    assert tt.migration_policy(1000, 100, 10, 25, 25, 1.0) == (3, False)
    # theta below 1 - beta: no migration; equal bests: none
    assert tt.migration_policy(1000, 100, 400, 9, 9, 0.25)[0] == 0
    assert tt.migration_policy(1000, 400, 400, 9, 9, 1.0)[0] == 0


def test_ga_invariants():
    inst = inputs.tardiness_instance(20, 3, [2, 2, 2], seed=3)
    isl = [inputs.cellular(6, 6, 1.0, 0.05), inputs.pseudo(36, 0.75, 0.0)]
    ga = tt.GA(inst, isl, interval=0, seed=7)
    E = ga.emax()
    prev = ga.population(0)[1].copy()
    for _ in range(15):
        ga.evolve(1)
        g0, o0 = ga.population(0)
        assert (o0 <= prev).all()                      # cellular: replace only if better
        prev = o0.copy()
        g1, o1 = ga.population(1)
        for q in range(18):                            # pseudo pairs stay complementary
            assert np.array_equal(g1[2 * q], 1 - g1[2 * q + 1])
        for g, o in ((g0, o0), (g1, o1)):
            assert all(tt.decode(inst, g[i])[0] == o[i] for i in range(0, len(o), 5))
            assert (o <= E).all()
    b = ga.best()
    assert b["objective"] == tt.decode(inst, b["genes"])[0]
    assert b["objective"] <= min(int(ga.population(i)[1].min()) for i in range(2))


def test_ga_migration_moves_best_into_worst():
    inst = inputs.tardiness_instance(20, 3, [2, 2, 2], seed=3)
    isl = [inputs.cellular(4, 4, 1.0, 0.05), inputs.pseudo(16, 0.75, 0.0)]
    ga = tt.GA(inst, isl, interval=0, seed=8)
    ga.evolve(3)
    (ga_, oa), (gb, ob) = ga.population(0), ga.population(1)
    E = ga.emax()
    count, a_sends = tt.migration_policy(E, int(oa.min()), int(ob.min()), 16, 16, 1.0)
    ga.migrate()
    (ga2, oa2), (gb2, ob2) = ga.population(0), ga.population(1)
    src_o, dst_o, dst_o2 = (oa, ob, ob2) if a_sends else (ob, oa, oa2)
    best = sorted(range(16), key=lambda s: (src_o[s], s))[:count]
    worst = sorted(range(16), key=lambda s: (dst_o[s], s))[::-1][:count]
    for r in range(count):
        assert dst_o2[worst[r]] == src_o[best[r]]
    assert ga.counters() == ((1, count) if count else (0, 0))


def test_line_sweep_spreads_the_best_in_one_generation():
    """With no crossover and no mutation a child copies its better parent.
    A unique best cell at the start of the sweep then reaches every cell of
    the torus in one line-sweep generation (each cell already sees its
    updated north or west neighbour); the synchronous update reaches only the
    cell's von Neumann neighbours."""
    inst = inputs.tardiness_instance(6, 2, [2, 2], seed=1)
    rows, cols = 5, 4
    isl = [inputs.cellular(rows, cols, 0.0, 0.0)]
    rng = np.random.default_rng(4)
    while True:
        genes = rng.integers(0, 2, size=(rows * cols, 12)).astype(np.int32)
        obj = np.array([tt.decode(inst, x)[0] for x in genes], dtype=np.int64)
        best = int(np.argmin(obj))
        if (obj == obj[best]).sum() == 1:
            break
    # the unique best at the sweep's first cell
    genes[[0, best]] = genes[[best, 0]]
    obj[[0, best]] = obj[[best, 0]]
    vmin = int(obj[0])
    for sweep, want_best in ((True, set(range(rows * cols))), (False, {0, 1, cols - 1, cols, (rows - 1) * cols})):
        ga = tt.GA(inst, isl, interval=0, seed=3, sweep=sweep)
        ga.set_population(0, genes, obj)
        ga.evolve(1)
        g, o = ga.population(0)
        got = {s for s in range(rows * cols) if o[s] == vmin}
        assert got == want_best, (sweep, sorted(got))
        for s in got:
            assert np.array_equal(g[s], genes[0])


def test_mutation_worked_example():
    """Hand-computed gene moves of the variant's mutation (reading T4): the
    gene always goes to another machine of its stage, and a one-machine
    stage is left alone."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "tt_mutation_worked_example.json")) as f:
        g = json.load(f)
    inst = dict(M=np.array(g["M"], dtype=np.int32))
    for c in g["cases"]:
        got = tt.mutate(inst, g["x"], c["d_flag"], c["d_i"], c["d_r"], g["tm"])
        assert got.tolist() == c["child"], c["name"]
    s = g["single_machine"]
    got = tt.mutate(dict(M=np.array(s["M"], dtype=np.int32)), s["x"], s["d_flag"], s["d_i"], s["d_r"], 1 << 32)
    assert got.tolist() == s["child"]


def test_mutation_changes_one_gene_to_every_other_machine():
    """When the flag fires, exactly one gene changes, to a machine of its
    stage other than the old one, and over a fine grid of the machine draw
    every other machine is reached evenly."""
    M = np.array([2, 3, 4, 6], dtype=np.int32)
    inst = dict(M=M)
    rng = np.random.default_rng(2)
    J = 5
    x = np.concatenate([rng.integers(0, M) for _ in range(J)]).astype(np.int32)
    for i in range(J * len(M)):
        d_i = -(-(i << 32) // (J * len(M)))      # smallest draw that selects gene i
        ms = int(M[i % len(M)])
        hits = np.zeros(ms, dtype=np.int64)
        for d_r in range(0, 1 << 32, 1 << 22):
            y = tt.mutate(inst, x, 0, d_i, d_r, 1 << 32)
            diff = np.nonzero(y != x)[0]
            assert diff.tolist() == [i]
            assert 0 <= y[i] < ms and y[i] != x[i]
            hits[y[i]] += 1
        others = np.delete(hits, x[i])
        assert hits[x[i]] == 0 and others.max() - others.min() <= 1
