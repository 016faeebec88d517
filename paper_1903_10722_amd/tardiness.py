"""ctypes binding of include/ffs_tt.h (the paper-faithful variant):
argument marshalling only.  Every step runs in the HIP library; PyTorch
provides the device workspace and the stream.  Loading fails loudly if the
library was not built -- there is no fallback."""
from __future__ import annotations

import ctypes

import numpy as np

from .binding import FFS_OK, FFSError, IslandSpec, load_library

TT_EXPORTS = [
    "ffs_tt_create", "ffs_tt_destroy", "ffs_tt_last_error", "ffs_tt_set_instance", "ffs_tt_add_island",
    "ffs_tt_configure", "ffs_tt_workspace_size", "ffs_tt_bind_workspace", "ffs_tt_evolve", "ffs_tt_migrate",
    "ffs_tt_generation", "ffs_tt_get_population", "ffs_tt_set_population", "ffs_tt_set_generation",
    "ffs_tt_best", "ffs_tt_counters", "ffs_tt_evaluate", "ffs_tt_set_timing", "ffs_tt_kernel_time",
    "ffs_tt_set_update",
]

_ready = False


def load():
    global _ready
    lib = load_library()
    if _ready:
        return lib
    P = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    pi32, pi64 = ctypes.POINTER(i32), ctypes.POINTER(i64)
    lib.ffs_tt_create.argtypes = [P, ctypes.POINTER(P)]
    lib.ffs_tt_destroy.argtypes = [P]
    lib.ffs_tt_last_error.argtypes = [P]
    lib.ffs_tt_last_error.restype = ctypes.c_char_p
    lib.ffs_tt_set_instance.argtypes = [P, i32, i32, pi32, i32, pi32, pi32, pi64, i64]
    lib.ffs_tt_add_island.argtypes = [P, ctypes.POINTER(IslandSpec)]
    lib.ffs_tt_configure.argtypes = [P, i32, ctypes.c_double, u64, i32]
    lib.ffs_tt_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.ffs_tt_bind_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.ffs_tt_evolve.argtypes = [P, i32]
    lib.ffs_tt_migrate.argtypes = [P]
    lib.ffs_tt_generation.argtypes = [P, pi32]
    lib.ffs_tt_get_population.argtypes = [P, i32, i32, pi32, pi64]
    lib.ffs_tt_set_population.argtypes = [P, i32, i32, pi32, pi64]
    lib.ffs_tt_set_generation.argtypes = [P, i32]
    lib.ffs_tt_best.argtypes = [P, i32, pi64, pi32, pi32, pi32, pi32]
    lib.ffs_tt_counters.argtypes = [P, i32, pi64, pi64]
    lib.ffs_tt_evaluate.argtypes = [P, P, i32, P]
    lib.ffs_tt_set_timing.argtypes = [P, i32]
    lib.ffs_tt_set_update.argtypes = [P, i32]
    lib.ffs_tt_kernel_time.argtypes = [P, ctypes.POINTER(ctypes.c_double), pi64]
    _ready = True
    return lib


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class TtContext:
    """One context of the variant: set the instance and islands, bind, then
    evolve / evaluate / best / population.  `runs` independent runs of the GA
    (run r uses instance id r in its random streams)."""

    def __init__(self, inst: dict, islands, interval: int = 500, theta: float = 1.0, seed: int = 101,
                 runs: int = 1, device: int = 0, stream=None, sweep: bool = False):
        import torch
        self._torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        rc = self.lib.ffs_tt_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != FFS_OK:
            raise FFSError(rc, "context creation failed")
        self._h = h
        self.ws = None
        M, P = _i32(inst["M"]), _i32(inst["P"])
        J, S, MX = P.shape
        self.J, self.S, self.L = J, S, J * S
        self._check(self.lib.ffs_tt_set_instance(self._h, J, S, _p(M, ctypes.c_int32), MX, _p(P, ctypes.c_int32),
                                                 _p(_i32(inst["R"]), ctypes.c_int32),
                                                 _p(_i64(inst["D"]), ctypes.c_int64), int(inst["WT"])))
        self.sizes = []
        for isl in islands:
            spec = IslandSpec(int(isl["kind"]), int(isl.get("rows", 0)), int(isl.get("cols", 0)),
                              int(isl["size"]), float(isl["pc"]), float(isl["pm"]), 0)
            self._check(self.lib.ffs_tt_add_island(self._h, ctypes.byref(spec)))
            self.sizes.append(int(isl["size"]))
        self.runs = runs
        self._check(self.lib.ffs_tt_configure(self._h, int(interval), float(theta), int(seed), int(runs)))
        self._check(self.lib.ffs_tt_set_update(self._h, 1 if sweep else 0))
        b = ctypes.c_size_t()
        self._check(self.lib.ffs_tt_workspace_size(self._h, ctypes.byref(b)))
        nbytes = int(b.value)
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) & ~255
        self._check(self.lib.ffs_tt_bind_workspace(self._h, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)))

    def _check(self, rc: int):
        if rc != FFS_OK:
            raise FFSError(rc, self.lib.ffs_tt_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ffs_tt_destroy(self._h)
            self._h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def evolve(self, generations: int):
        self._check(self.lib.ffs_tt_evolve(self._h, int(generations)))

    def migrate(self):
        self._check(self.lib.ffs_tt_migrate(self._h))

    @property
    def generation(self) -> int:
        g = ctypes.c_int32()
        self._check(self.lib.ffs_tt_generation(self._h, ctypes.byref(g)))
        return g.value

    def set_generation(self, gen: int):
        self._check(self.lib.ffs_tt_set_generation(self._h, int(gen)))

    def population(self, run: int, island: int):
        n = self.sizes[island]
        genes = np.zeros((n, self.L), dtype=np.int32)
        obj = np.zeros(n, dtype=np.int64)
        self._check(self.lib.ffs_tt_get_population(self._h, run, island, _p(genes, ctypes.c_int32),
                                                   _p(obj, ctypes.c_int64)))
        return genes, obj

    def set_population(self, run: int, island: int, genes, obj):
        g, o = _i32(genes), _i64(obj)
        assert g.shape == (self.sizes[island], self.L)
        self._check(self.lib.ffs_tt_set_population(self._h, run, island, _p(g, ctypes.c_int32),
                                                   _p(o, ctypes.c_int64)))

    def best(self, run: int = 0) -> dict:
        o = ctypes.c_int64()
        gen, isl, slot = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        genes = np.zeros(self.L, dtype=np.int32)
        self._check(self.lib.ffs_tt_best(self._h, run, ctypes.byref(o), ctypes.byref(gen), ctypes.byref(isl),
                                         ctypes.byref(slot), _p(genes, ctypes.c_int32)))
        return dict(objective=o.value, generation=gen.value, island=isl.value, slot=slot.value, genes=genes)

    def counters(self, run: int = 0):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.ffs_tt_counters(self._h, run, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def evaluate(self, genes):
        """Objectives (torch int64, device) of the rows of `genes` (count x J*S)."""
        torch = self._torch
        t = genes if isinstance(genes, torch.Tensor) else torch.from_numpy(np.asarray(genes, dtype=np.uint8))
        t = t.to(device=self.device, dtype=torch.uint8).contiguous()
        assert t.shape[1] == self.L
        out = torch.empty(t.shape[0], dtype=torch.int64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.lib.ffs_tt_evaluate(self._h, ctypes.c_void_p(t.data_ptr()), int(t.shape[0]),
                                             ctypes.c_void_p(out.data_ptr())))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def set_timing(self, enable: bool):
        self._check(self.lib.ffs_tt_set_timing(self._h, 1 if enable else 0))

    def kernel_time(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.ffs_tt_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
