"""Oracle of the paper-faithful variant (TEST INFRASTRUCTURE ONLY).

Marshals arrays for ``ffs_tt_oracle.c``: Section 3's objective
WT * sum T_j + C_max with release and due dates on unrelated machines
(Table 1's data), Section 4.1's machine-assignment genotype with its
complement layer, and the island GA of Sections 4.1-4.3 on it.  Times are
integers in hundredths of a time unit.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _load, _ptr, _i32, _i32p, _i64p, _f64p

_ready = False


def _lib():
    global _ready
    lib = _load()
    if _ready:
        return lib
    lib.or_tt_decode.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _i32p, _i32p, _i64p,
                                 ctypes.c_int64, _i32p, _i64p, _i64p, _i64p]
    lib.or_tt_decode.restype = ctypes.c_int64
    lib.or_tt_emax.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _i32p, _i32p, _i64p,
                               ctypes.c_int64]
    lib.or_tt_emax.restype = ctypes.c_int64
    lib.or_tt_two_point.argtypes = [ctypes.c_int, _i32p, _i32p, ctypes.c_int, ctypes.c_int, _i32p]
    lib.or_tt_complement.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p, _i32p]
    lib.or_tt_mutate.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_uint64]
    lib.or_tt_mutate.restype = None
    lib.or_tt_random_genes.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_int, ctypes.c_int, _i32p]
    lib.or_tt_migration_policy.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    lib.or_tt_migration_policy.restype = ctypes.c_int64
    lib.or_tt_ga_create.argtypes = [ctypes.c_int, ctypes.c_int, _i32p, ctypes.c_int, _i32p, _i32p, _i64p,
                                    ctypes.c_int64, ctypes.c_int, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64]
    lib.or_tt_ga_create.restype = ctypes.c_void_p
    lib.or_tt_ga_destroy.argtypes = [ctypes.c_void_p]
    lib.or_tt_ga_evolve.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_tt_ga_migrate.argtypes = [ctypes.c_void_p]
    lib.or_tt_ga_generation.argtypes = [ctypes.c_void_p]
    lib.or_tt_ga_generation.restype = ctypes.c_int
    lib.or_tt_ga_set_generation.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_tt_ga_set_update.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.or_tt_ga_emax.argtypes = [ctypes.c_void_p]
    lib.or_tt_ga_emax.restype = ctypes.c_int64
    lib.or_tt_ga_get.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p, _i64p]
    lib.or_tt_ga_set.argtypes = [ctypes.c_void_p, ctypes.c_int, _i32p, _i64p]
    lib.or_tt_ga_best.argtypes = [ctypes.c_void_p, _i64p, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _i32p]
    lib.or_tt_ga_counters.argtypes = [ctypes.c_void_p, _i64p, _i64p]
    _ready = True
    return lib


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _inst_args(inst):
    M = _i32(inst["M"])
    P = _i32(inst["P"])
    J, S, MX = P.shape
    return J, S, M, MX, P, _i32(inst["R"]), _i64(inst["D"]), int(inst["WT"])


def decode(inst, genes):
    """(objective, C_max, sum T, completions C[j][s] as a J x S array)."""
    J, S, M, MX, P, R, D, WT = _inst_args(inst)
    x = _i32(genes).reshape(-1)
    assert x.shape == (J * S,)
    C = np.zeros((J, S), dtype=np.int64)
    cmax = ctypes.c_int64()
    tard = ctypes.c_int64()
    obj = _lib().or_tt_decode(J, S, _ptr(M, _i32p), MX, _ptr(P, _i32p), _ptr(R, _i32p), _ptr(D, _i64p), WT,
                              _ptr(x, _i32p), _ptr(C, _i64p), ctypes.byref(cmax), ctypes.byref(tard))
    return int(obj), int(cmax.value), int(tard.value), C


def decode_many(inst, genes) -> np.ndarray:
    return np.array([decode(inst, g)[0] for g in np.asarray(genes)], dtype=np.int64)


def emax(inst) -> int:
    J, S, M, MX, P, R, D, WT = _inst_args(inst)
    return int(_lib().or_tt_emax(J, S, _ptr(M, _i32p), MX, _ptr(P, _i32p), _ptr(R, _i32p), _ptr(D, _i64p), WT))


def two_point(p1, p2, a, b):
    x1, x2 = _i32(p1), _i32(p2)
    out = np.zeros_like(x1)
    _lib().or_tt_two_point(len(x1), _ptr(x1, _i32p), _ptr(x2, _i32p), a, b, _ptr(out, _i32p))
    return out


def complement(inst, x):
    M = _i32(inst["M"])
    S = len(M)
    xx = _i32(x)
    out = np.zeros_like(xx)
    _lib().or_tt_complement(len(xx) // S, S, _ptr(M, _i32p), _ptr(xx, _i32p), _ptr(out, _i32p))
    return out


def mutate(inst, x, d_flag: int, d_i: int, d_r: int, tm: int) -> np.ndarray:
    """The variant's mutation of one child for given draws (gene i moves to
    another machine of its stage); returns the new row."""
    M = _i32(inst["M"])
    out = _i32(x).copy()
    J = out.shape[0] // M.shape[0]
    _lib().or_tt_mutate(J, M.shape[0], _ptr(M, _i32p), _ptr(out, _i32p), d_flag, d_i, d_r, tm)
    return out


def random_genes(inst, seed, inst_id, island, slot):
    J, S, M, MX, P, R, D, WT = _inst_args(inst)
    out = np.zeros(J * S, dtype=np.int32)
    _lib().or_tt_random_genes(J, S, _ptr(M, _i32p), seed, inst_id, island, slot, _ptr(out, _i32p))
    return out


def migration_policy(E, best_a, best_b, n_a, n_b, theta):
    ea = ctypes.c_int()
    c = _lib().or_tt_migration_policy(E, best_a, best_b, n_a, n_b, theta, ctypes.byref(ea))
    return int(c), bool(ea.value)


class GA:
    """One trajectory of the variant's island GA (same seed, same trajectory)."""

    def __init__(self, inst, islands, interval=500, theta=1.0, seed=101, inst_id=0, sweep=False):
        lib = _lib()
        J, S, M, MX, P, R, D, WT = _inst_args(inst)
        self.J, self.S, self.L = J, S, J * S
        kinds = _i32([i["kind"] for i in islands])
        rows = _i32([i["rows"] for i in islands])
        cols = _i32([i["cols"] for i in islands])
        sizes = _i32([i["size"] for i in islands])
        pc = np.ascontiguousarray([float(i["pc"]) for i in islands], dtype=np.float64)
        pm = np.ascontiguousarray([float(i["pm"]) for i in islands], dtype=np.float64)
        self.sizes = [int(x) for x in sizes]
        self._lib = lib
        self._h = lib.or_tt_ga_create(J, S, _ptr(M, _i32p), MX, _ptr(P, _i32p), _ptr(R, _i32p), _ptr(D, _i64p), WT,
                                      len(islands), _ptr(kinds, _i32p), _ptr(rows, _i32p), _ptr(cols, _i32p),
                                      _ptr(sizes, _i32p), _ptr(pc, _f64p), _ptr(pm, _f64p), int(interval),
                                      float(theta), int(seed), int(inst_id))
        lib.or_tt_ga_set_update(self._h, 1 if sweep else 0)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.or_tt_ga_destroy(self._h)
            self._h = None

    def evolve(self, G: int):
        self._lib.or_tt_ga_evolve(self._h, G)

    def migrate(self):
        self._lib.or_tt_ga_migrate(self._h)

    @property
    def generation(self) -> int:
        return self._lib.or_tt_ga_generation(self._h)

    def set_generation(self, g: int):
        self._lib.or_tt_ga_set_generation(self._h, g)

    def emax(self) -> int:
        return int(self._lib.or_tt_ga_emax(self._h))

    def population(self, island: int):
        genes = np.zeros((self.sizes[island], self.L), dtype=np.int32)
        obj = np.zeros(self.sizes[island], dtype=np.int64)
        self._lib.or_tt_ga_get(self._h, island, _ptr(genes, _i32p), _ptr(obj, _i64p))
        return genes, obj

    def set_population(self, island: int, genes, obj):
        g = _i32(genes)
        o = _i64(obj)
        assert g.shape == (self.sizes[island], self.L)
        self._lib.or_tt_ga_set(self._h, island, _ptr(g, _i32p), _ptr(o, _i64p))

    def best(self):
        obj = ctypes.c_int64()
        gen, isl, slot = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        genes = np.zeros(self.L, dtype=np.int32)
        self._lib.or_tt_ga_best(self._h, ctypes.byref(obj), ctypes.byref(gen), ctypes.byref(isl),
                                ctypes.byref(slot), _ptr(genes, _i32p))
        return dict(objective=int(obj.value), generation=gen.value, island=isl.value, slot=slot.value,
                    genes=genes)

    def counters(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._lib.or_tt_ga_counters(self._h, ctypes.byref(a), ctypes.byref(b))
        return int(a.value), int(b.value)
