"""CPU oracle for the dual heterogeneous island GA (arXiv 1903.10722).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never imports it.  It shares no code
with the HIP library.  The arithmetic lives in ``ffs_oracle.c`` (plain,
single-threaded C); this module only builds it with gcc and marshals arrays.

Functions and the passage of the paper each follows:
  decode           Section 3 (problem), decoding rule = project reading
  ox               Section 4.2 "recombines two individuals" (Davis order crossover)
  fisher_yates     Section 4.1 "random initialization"
  cell_parents     Section 4.2, neighbourhood of the cellular GA (Fig. 3 reading)
  swap_mutation    Section 4.2 "undertakes the mutation" (one swap, j != i)
  pseudo_children  Section 4.1 operator level (a parent mates with its complement)
  migration_policy Section 4.3, equations (1) and (2)
  GA               Sections 4.1-4.3 (one whole island-GA trajectory)
  philox           Salmon et al. SC'11 (the counter-based generator)
  tardiness        the paper-faithful variant (``ffs_tt_oracle.c``): Section 3's
                   objective with release and due dates on unrelated machines,
                   Section 4.1's machine-assignment genotype, Table 1's data
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffs_oracle.c")
_SRC_TT = os.path.join(_HERE, "ffs_tt_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f64p = ctypes.POINTER(ctypes.c_double)

_lib = None


def build() -> str:
    """Compile the C oracle with gcc (always recompiles)."""
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           _SRC, _SRC_TT, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.or_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.or_philox4x64_10.restype = None
    lib.or_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
    lib.or_draw.restype = ctypes.c_uint32
    lib.or_decode.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i32p, _i64p, _i32p]
    lib.or_decode.restype = ctypes.c_int64
    lib.or_ox.argtypes = [ctypes.c_int, _i32p, _i32p, ctypes.c_int, ctypes.c_int, _i32p]
    lib.or_ox.restype = None
    lib.or_fisher_yates.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_int, _i32p]
    lib.or_fisher_yates.restype = None
    lib.or_cell_parents.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _i32p, _i32p]
    lib.or_cell_parents.restype = None
    lib.or_cell_parents_sel.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_uint32, ctypes.c_uint32, _i32p, _i32p]
    lib.or_cell_parents_sel.restype = None
    lib.or_ga_set_selection.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.or_ga_set_selection.restype = None
    lib.or_ga_set_sweep.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.or_ga_set_sweep.restype = None
    lib.or_migration_policy.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_int)]
    lib.or_migration_policy.restype = ctypes.c_int64
    lib.or_ga_create.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                 _i32p, _i32p, _i32p, _i32p, _f64p, _f64p, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
    lib.or_ga_create.restype = ctypes.c_void_p
    lib.or_ga_destroy.argtypes = [ctypes.c_void_p]
    lib.or_ga_evolve.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_ga_migrate.argtypes = [ctypes.c_void_p]
    lib.or_ga_generation.argtypes = [ctypes.c_void_p]
    lib.or_ga_generation.restype = ctypes.c_int
    lib.or_ga_get.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p, _i32p]
    lib.or_ga_set.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p, _i32p]
    lib.or_ga_best.argtypes = [ctypes.c_void_p, _i64p, ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _i32p]
    lib.or_ga_counters.argtypes = [ctypes.c_void_p, _i64p, _i64p]
    lib.or_ga_set_generation.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_ga_step_island.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_ga_cell_candidate.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p, _i32p]
    lib.or_ga_set_cell_choices.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p]
    lib.or_swap_mutation.argtypes = [ctypes.c_int, _i32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint64]
    lib.or_swap_mutation.restype = None
    lib.or_pseudo_children.argtypes = [ctypes.c_int, _i32p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64,
                                       ctypes.c_uint64, _i32p, _i32p]
    lib.or_pseudo_children.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def philox(ctr, key) -> list[int]:
    """Philox4x64-10 block for a 4-word counter and a 2-word key."""
    lib = _load()
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.or_philox4x64_10(_ptr(c, _u64p), _ptr(k, _u64p), _ptr(out, _u64p))
    return [int(x) for x in out]


def draw(seed, inst, island, slot, sub, gen, purpose, d) -> int:
    return int(_load().or_draw(seed, inst, island, slot, sub, gen, purpose, d))


def decode(m, p, perm, schedule: bool = False):
    """Makespan of `perm` (job ids) on the instance (m[S], p[n][S] job-major).

    With schedule=True also returns (start[n][S], machine[n][S])."""
    lib = _load()
    m = _i32(m)
    p = _i32(p)
    n, S = p.shape
    perm = _i32(perm)
    assert perm.shape == (n,)
    if schedule:
        st = np.zeros((n, S), dtype=np.int64)
        mc = np.zeros((n, S), dtype=np.int32)
        c = lib.or_decode(n, S, _ptr(m, _i32p), _ptr(p, _i32p), _ptr(perm, _i32p),
                          _ptr(st, _i64p), _ptr(mc, _i32p))
        return int(c), st, mc
    return int(lib.or_decode(n, S, _ptr(m, _i32p), _ptr(p, _i32p), _ptr(perm, _i32p), None, None))


def decode_many(m, p, perms) -> np.ndarray:
    perms = _i32(perms)
    return np.array([decode(m, p, x) for x in perms], dtype=np.int64)


def ox(p1, p2, a: int, b: int) -> np.ndarray:
    lib = _load()
    p1 = _i32(p1)
    p2 = _i32(p2)
    n = p1.shape[0]
    out = np.zeros(n, dtype=np.int32)
    lib.or_ox(n, _ptr(p1, _i32p), _ptr(p2, _i32p), a, b, _ptr(out, _i32p))
    return out


def fisher_yates(n: int, seed: int, inst: int, island: int, slot: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int32)
    _load().or_fisher_yates(n, seed, inst, island, slot, _ptr(out, _i32p))
    return out


def rate_threshold(p: float) -> int:
    """floor(p * 2^32), with p = 1 meaning "always" (2^32)."""
    if p <= 0.0:
        return 0
    if p >= 1.0:
        return 1 << 32
    return int(p * 4294967296.0)


def swap_mutation(x, d_flag: int, d_i: int, d_j: int, tm: int) -> np.ndarray:
    """The swap mutation of one child (Section 4.2) for given draws and a
    mutation threshold tm (mutate iff d_flag < tm); returns the new row."""
    out = _i32(x).copy()
    _load().or_swap_mutation(out.shape[0], _ptr(out, _i32p), d_flag, d_i, d_j, tm)
    return out


def pseudo_children(X, draws, tc: int, tm: int) -> tuple[np.ndarray, np.ndarray]:
    """The two children of one complementary pair (Section 4.1) from its
    better member X and the pair's nine draws d0..d8."""
    X = _i32(X)
    d = np.ascontiguousarray(np.asarray(draws, dtype=np.uint32))
    assert d.shape == (9,)
    n = X.shape[0]
    c1 = np.zeros(n, dtype=np.int32)
    c2 = np.zeros(n, dtype=np.int32)
    _load().or_pseudo_children(n, _ptr(X, _i32p), d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), tc, tm,
                               _ptr(c1, _i32p), _ptr(c2, _i32p))
    return c1, c2


def cell_parents(rows: int, cols: int, mk, slot: int, sel: int = 0, d6: int = 0, d7: int = 0) -> tuple[int, int]:
    """Parent slots of cell `slot` (selection variant `sel`; d6, d7 are the
    cell's draws 6 and 7, used by the binary tournaments of sel 2)."""
    mk = _i32(mk)
    a = ctypes.c_int32()
    b = ctypes.c_int32()
    if sel == 0:
        _load().or_cell_parents(rows, cols, _ptr(mk, _i32p), slot, ctypes.byref(a), ctypes.byref(b))
    else:
        _load().or_cell_parents_sel(rows, cols, _ptr(mk, _i32p), slot, sel, d6, d7, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def migration_policy(E, best_a, best_b, n_a, n_b, theta) -> tuple[int, bool]:
    """(count, emigrant_is_a) of one island pair."""
    flag = ctypes.c_int()
    c = _load().or_migration_policy(E, best_a, best_b, n_a, n_b, theta, ctypes.byref(flag))
    return int(c), bool(flag.value)


class GA:
    """One island-GA trajectory on one instance (see ffs_oracle.c)."""

    def __init__(self, m, p, islands, interval: int, theta: float = 1.0, topology: int = 0,
                 seed: int = 1, inst: int = 0):
        self._lib = _load()
        self.m = _i32(m)
        self.p = _i32(p)
        self.n, self.S = self.p.shape
        self.islands = [dict(x) for x in islands]
        k = len(self.islands)
        kinds = _i32([x["kind"] for x in self.islands])
        rows = _i32([x.get("rows", 0) for x in self.islands])
        cols = _i32([x.get("cols", 0) for x in self.islands])
        sizes = _i32([x.get("size", 0) for x in self.islands])
        pc = np.array([x["pc"] for x in self.islands], dtype=np.float64)
        pm = np.array([x["pm"] for x in self.islands], dtype=np.float64)
        self.sizes = [int(r * c) if kd == 0 else int(s) for kd, r, c, s in zip(kinds, rows, cols, sizes)]
        self._h = self._lib.or_ga_create(self.n, self.S, _ptr(self.m, _i32p), _ptr(self.p, _i32p), k,
                                         _ptr(kinds, _i32p), _ptr(rows, _i32p), _ptr(cols, _i32p),
                                         _ptr(sizes, _i32p), _ptr(pc, _f64p), _ptr(pm, _f64p),
                                         interval, theta, topology, seed, inst)
        for i, x in enumerate(self.islands):
            if x["kind"] == 0 and int(x.get("sel", 0)):
                self._lib.or_ga_set_selection(self._h, i, int(x["sel"]))
            if x["kind"] == 0 and int(x.get("sweep", 0)):
                self._lib.or_ga_set_sweep(self._h, i, 1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_ga_destroy(h)
            self._h = None

    @property
    def generation(self) -> int:
        return int(self._lib.or_ga_generation(self._h))

    def evolve(self, G: int):
        self._lib.or_ga_evolve(self._h, G)

    def migrate(self):
        self._lib.or_ga_migrate(self._h)

    def population(self, island: int):
        N = self.sizes[island]
        genes = np.zeros((N, self.n), dtype=np.int32)
        mk = np.zeros(N, dtype=np.int32)
        self._lib.or_ga_get(self._h, island, _ptr(genes, _i32p), _ptr(mk, _i32p))
        return genes, mk

    def set_population(self, island: int, genes, mk):
        genes = _i32(genes)
        mk = _i32(mk)
        assert genes.shape == (self.sizes[island], self.n)
        self._lib.or_ga_set(self._h, island, _ptr(genes, _i32p), _ptr(mk, _i32p))

    def set_generation(self, gen: int):
        self._lib.or_ga_set_generation(self._h, gen)

    def step_island(self, island: int):
        """Next generation of one island only (no migration, counters kept)."""
        self._lib.or_ga_step_island(self._h, island)

    def cell_candidate(self, island: int, slot: int, sub: int):
        """(child, meta) of a cell at the next generation from candidate stream
        `sub`; meta = (p1, p2, crossover, a, b, mutation, i, j)."""
        child = np.zeros(self.n, dtype=np.int32)
        meta = np.zeros(8, dtype=np.int32)
        self._lib.or_ga_cell_candidate(self._h, island, slot, sub, _ptr(child, _i32p), _ptr(meta, _i32p))
        return child, meta

    def set_cell_choices(self, island: int, choices):
        """Candidate stream per cell for the next generation only."""
        if choices is None:
            self._lib.or_ga_set_cell_choices(self._h, island, None)
        else:
            c = _i32(choices)
            assert c.shape == (self.sizes[island],)
            self._lib.or_ga_set_cell_choices(self._h, island, _ptr(c, _i32p))

    def best(self):
        mk = ctypes.c_int64()
        gen = ctypes.c_int()
        isl = ctypes.c_int()
        slot = ctypes.c_int()
        perm = np.zeros(self.n, dtype=np.int32)
        self._lib.or_ga_best(self._h, ctypes.byref(mk), ctypes.byref(gen), ctypes.byref(isl),
                             ctypes.byref(slot), _ptr(perm, _i32p))
        return dict(makespan=int(mk.value), generation=gen.value, island=isl.value,
                    slot=slot.value, perm=perm)

    def counters(self):
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        self._lib.or_ga_counters(self._h, ctypes.byref(a), ctypes.byref(b))
        return int(a.value), int(b.value)


def lower_bound(m, p) -> int:
    """max(max_k ceil(sum_j p_jk / m_k), max_j sum_k p_jk)."""
    m = np.asarray(m, dtype=np.int64)
    p = np.asarray(p, dtype=np.int64)
    stage = max(int(-(-p[:, k].sum() // m[k])) for k in range(p.shape[1]))
    job = int(p.sum(axis=1).max())
    return max(stage, job)
