"""Seeded synthetic inputs: flow-shop instances, permutations, workload shapes.

This module holds none of the method's arithmetic.  It only draws the numbers
that define a workload (machine counts, processing times, batch shapes, test
permutations) from numpy's Philox generator, so that the HIP path, the oracle,
the tests and the benchmark all see the same inputs for the same seed.

The paper measures on generated instances (Section 5, Table 1: processing times
uniform over a small integer range, several machines per stage); the workloads
below keep that structure -- independent uniform integer processing times, a
uniform machine count per stage -- at the sizes of the benchmarked configurations.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), stream]))


def make_instance(n: int, S: int, m_lo: int, m_hi: int, p_lo: int = 1, p_hi: int = 99,
                  seed: int = 1, machines=None):
    """(m[S], p[n][S]) int32; m uniform in [m_lo, m_hi] unless `machines` is given,
    p uniform in [p_lo, p_hi], job-major."""
    g = _rng(seed, 1)
    if machines is None:
        m = g.integers(m_lo, m_hi + 1, size=S).astype(np.int32)
    else:
        m = np.asarray(machines, dtype=np.int32)
        assert m.shape == (S,)
    p = g.integers(p_lo, p_hi + 1, size=(n, S)).astype(np.int32)
    return m, p


def random_perms(count: int, n: int, seed: int = 0) -> np.ndarray:
    """count x n int32, each row a uniformly random permutation of 0..n-1."""
    g = _rng(seed, 2)
    keys = g.random((count, n))
    return np.argsort(keys, axis=1).astype(np.int32)


def cellular(rows: int, cols: int, pc: float, pm: float, sel: int = 0, sweep: int = 0) -> dict:
    """A rows x cols cellular island; `sel` is the parent selection variant
    (0 two best of the neighbourhood, 1 self + best neighbour, 2 binary
    tournaments), `sweep` the update schedule (0 synchronous, 1 line sweep)."""
    return dict(kind=0, rows=rows, cols=cols, size=rows * cols, pc=pc, pm=pm, sel=sel, sweep=sweep)


def pseudo(size: int, pc: float, pm: float) -> dict:
    return dict(kind=1, rows=0, cols=0, size=size, pc=pc, pm=pm)


# Rates: the cellular island uses crossover 0.9 / swap mutation 0.1; the pseudo
# island crossover 0.75 (Section 5's pseudo-GA rate) and no mutation.
CELL_PC, CELL_PM = 0.9, 0.1
PAIR_PC, PAIR_PM = 0.75, 0.0


def workload(name: str, seed: int = 1, scale: int = 1) -> dict:
    """Instance + island layout + schedule of a named workload.

    `scale` > 1 shrinks every island side (and pseudo size) by that factor,
    keeping n, S and the distributions -- used for oracle-sized parity runs."""
    if name == "tiny":
        m, p = make_instance(20, 3, 2, 2, seed=seed, machines=[2, 2, 2])
        side = max(3, 8 // scale)
        isl = [cellular(side, side, CELL_PC, CELL_PM), pseudo(2 * ((side * side) // 2), PAIR_PC, PAIR_PM)]
        return dict(name=name, m=m, p=p, islands=isl, generations=100, interval=10, theta=1.0, topology=0)
    if name == "medium":
        m, p = make_instance(100, 5, 1, 5, seed=seed)
        side = max(3, 64 // scale)
        isl = [cellular(side, side, CELL_PC, CELL_PM), pseudo(side * side - (side * side) % 2, PAIR_PC, PAIR_PM)]
        return dict(name=name, m=m, p=p, islands=isl, generations=500, interval=20, theta=1.0, topology=0)
    if name == "large":
        m, p = make_instance(500, 10, 3, 5, seed=seed)
        side = max(3, 128 // scale)
        ps = side * side - (side * side) % 2
        isl = [cellular(side, side, CELL_PC, CELL_PM) for _ in range(8)] + \
              [pseudo(ps, PAIR_PC, PAIR_PM) for _ in range(8)]
        return dict(name=name, m=m, p=p, islands=isl, generations=1000, interval=20, theta=1.0, topology=1)
    if name == "surrogate":
        m, p = make_instance(1000, 20, 2, 6, seed=seed)
        side = max(3, 64 // scale)
        isl = [cellular(side, side, CELL_PC, CELL_PM), pseudo(side * side - (side * side) % 2, PAIR_PC, PAIR_PM)]
        return dict(name=name, m=m, p=p, islands=isl, generations=500, interval=20, theta=1.0, topology=0)
    raise KeyError(name)


# Island layouts of the ablation (which kind of island, and how many), all
# with the same number of individuals per generation.
ISLAND_VARIANTS = ("dual", "cellular", "pseudo", "cellular2", "pseudo2")


def _layout(variant: str, side: int, cell_rates, pair_rates) -> list:
    half = side * side - (side * side) % 2
    c = lambda r, k: cellular(r, k, *cell_rates)
    if variant == "dual":
        return [c(side, side), pseudo(half, *pair_rates)]
    if variant == "cellular":
        return [c(side, 2 * side)]
    if variant == "pseudo":
        return [pseudo(2 * half, *pair_rates)]
    if variant == "cellular2":
        return [c(side, side), c(side, side)]
    if variant == "pseudo2":
        return [pseudo(half, *pair_rates), pseudo(half, *pair_rates)]
    if variant == "ring16":
        return [c(side, side) for _ in range(8)] + [pseudo(half, *pair_rates) for _ in range(8)]
    raise KeyError(variant)


def island_variant(variant: str, seed: int = 1, scale: int = 1, interval: int = 20) -> dict:
    """The medium instance (n=100, S=5) with its 8192 individuals arranged as
    dual (64x64 cellular + 4096 pseudo, the benchmarked layout), cellular (one
    64x128 torus), pseudo (one island of 8192), cellular2 (two 64x64 tori) or
    pseudo2 (two islands of 4096); two-island layouts migrate every
    `interval` generations with the adaptive rule.  `scale` divides island
    sides (and pseudo sizes by its square) for oracle-sized runs."""
    m, p = make_instance(100, 5, 1, 5, seed=seed)
    isl = _layout(variant, max(3, 64 // scale), (CELL_PC, CELL_PM), (PAIR_PC, PAIR_PM))
    return dict(name=f"islands:{variant}", m=m, p=p, islands=isl, generations=2000, interval=interval,
                theta=1.0, topology=0)


# Section 5's experimental setting: 300 jobs, 4 stages, 2 machines per stage,
# processing times uniform in [1, 5] (Table 1), 256 individuals per island
# (512 for a single-population GA), crossover 1.00 / mutation 0.05 on the
# cellular island and crossover 0.75 on the pseudo island, 2000 generations,
# theta 1.  Identical machines and the makespan objective replace Table 1's
# unrelated machines, release and due dates.
PAPER_CELL_RATES = (1.0, 0.05)
PAPER_PAIR_RATES = (0.75, 0.0)


def paper_setting(variant: str = "dual", seed: int = 1, interval: int = 500, sel: int = 0,
                  topology: int = 0) -> dict:
    """Section 5's problem and population sizes with the layouts of
    island_variant at 512 individuals (dual = 16x16 cellular + 256 pseudo),
    or ring16: eight such pairs (4096 individuals) migrating with `topology`
    (1 ring then pairs, 2 the rule on every ring edge); `sel` is the cellular
    islands' parent selection variant."""
    m, p = make_instance(300, 4, 2, 2, p_lo=1, p_hi=5, seed=seed, machines=[2, 2, 2, 2])
    isl = _layout(variant, 16, PAPER_CELL_RATES + (sel,), PAPER_PAIR_RATES)
    return dict(name=f"paper:{variant}", m=m, p=p, islands=isl, generations=2000, interval=interval,
                theta=1.0, topology=topology if variant == "ring16" else 0)


def batched_workloads(count: int = 256, batch_seed: int = 7, scale: int = 1, n_choices=None) -> list[dict]:
    """The uneven batch: per instance n in {20,50,100,200,500}, S in {5,10,20},
    machines per stage uniform [1,5], p uniform [1,99], a dual island with an
    L x L cellular grid (L uniform in 32..128) and a pseudo island of L*L."""
    g = _rng(batch_seed, 3)
    n_choices = n_choices or [20, 50, 100, 200, 500]
    out = []
    for i in range(count):
        n = int(g.choice(n_choices))
        S = int(g.choice([5, 10, 20]))
        L = int(g.integers(32, 129))
        Ls = max(3, L // scale)
        m, p = make_instance(n, S, 1, 5, seed=batch_seed * 100003 + i + 1)
        isl = [cellular(Ls, Ls, CELL_PC, CELL_PM), pseudo(Ls * Ls - (Ls * Ls) % 2, PAIR_PC, PAIR_PM)]
        out.append(dict(name=f"batched[{i}]", m=m, p=p, islands=isl, generations=50, interval=10,
                        theta=1.0, topology=0))
    return out


# ---- the paper-faithful variant (unrelated machines, release and due dates) --
WT_PAPER = 100


def tardiness_instance(J: int = 300, S: int = 4, machines=None, seed: int = 1, wt: int = WT_PAPER,
                       p_lo: int = 1, p_hi: int = 5, release_scale: float = 1.0) -> dict:
    """Table 1's generator, every time in hundredths of a time unit:
    P[j][s][m] uniform integer in [p_lo, p_hi] (times 100), R_j uniform in
    [0, Pbar) with Pbar = sum_j sum_s (sum_m P_jsm / M_s), and
    D_j = R_j + Pbar_j (1 + sigma_j) with Pbar_j = sum_s (sum_m P_jsm / M_s)
    and sigma_j uniform in [0, 2]; R and D are floored to whole hundredths.
    P is [J][S][MX] (MX = max M_s; unused machine slots hold 0).
    `release_scale` < 1 compresses the release range to [0, Pbar * scale): a
    more loaded shop (an alternative reading of Table 1's R_j)."""
    M = np.asarray(machines if machines is not None else [2] * S, dtype=np.int32)
    assert M.shape == (S,) and (M >= 1).all()
    MX = int(M.max())
    g = _rng(seed, 5)
    P = np.zeros((J, S, MX), dtype=np.int32)
    for s in range(S):
        P[:, s, :M[s]] = g.integers(p_lo, p_hi + 1, size=(J, int(M[s]))) * 100
    pbar_j = np.zeros(J)
    for s in range(S):
        pbar_j += P[:, s, :M[s]].sum(axis=1) / float(M[s])     # hundredths
    pbar = float(pbar_j.sum())
    R = np.floor(g.random(J) * pbar * release_scale).astype(np.int32)
    sigma = g.random(J) * 2.0
    D = (R + np.floor(pbar_j * (1.0 + sigma))).astype(np.int64)
    return dict(J=J, S=S, M=M, P=P, R=R, D=D, WT=int(wt))


def tardiness_setting(variant: str = "dual", seed: int = 1, interval: int = 500, J: int = 300,
                      S: int = 4, side: int = 16, release_scale: float = 1.0) -> dict:
    """Section 5's setting on the faithful variant: 300 jobs, 4 stages, 2
    unrelated machines per stage, a side x side cellular island (crossover
    1.00, mutation 0.05) and a pseudo island of side^2 (crossover 0.75)."""
    inst = tardiness_instance(J, S, [2] * S, seed=seed, release_scale=release_scale)
    isl = _layout(variant, side, PAPER_CELL_RATES + (0,), PAPER_PAIR_RATES)
    return dict(name=f"tardiness:{variant}", inst=inst, islands=isl, generations=2000,
                interval=interval, theta=1.0)
