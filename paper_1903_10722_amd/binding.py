"""ctypes binding of include/ffs.h: argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts
numpy / torch arguments into the C structs and pointers the ABI expects and
raises FFSError on a negative status.  PyTorch provides the device workspace
and the stream.  The library must be built (see build.py); loading fails
loudly otherwise -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "libffs.so")

FFS_OK, FFS_EINVAL, FFS_ENOMEM, FFS_EDEVICE, FFS_ESTATE, FFS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5

EXPORTS = [
    "ffs_ctx_create", "ffs_ctx_destroy", "ffs_last_error", "ffs_create_instance",
    "ffs_set_waves_per_block", "ffs_workspace_size", "ffs_bind_workspace", "ffs_evaluate",
    "ffs_evolve", "ffs_migrate", "ffs_best", "ffs_get_population", "ffs_generation",
    "ffs_migration_counters", "ffs_set_graphs", "ffs_set_timing", "ffs_kernel_time",
    "ffs_surrogate_params", "ffs_surrogate_set_params", "ffs_mlp_forward", "ffs_mlp_gradients",
    "ffs_mlp_train_step", "ffs_surrogate_candidates", "ffs_surrogate_choices", "ffs_surrogate_ring",
    "ffs_evaluate_host", "ffs_checkpoint_size", "ffs_checkpoint_save", "ffs_checkpoint_load",
    "ffs_set_mapping", "ffs_get_mapping", "ffs_evaluate_noalloc", "ffs_set_instance_tile",
    "ffs_set_concurrent", "ffs_set_chains", "ffs_get_chains",
]

N_PARAMS = 394753
PARAM_SLICES = {"W1": (0, (512, 256)), "b1": (131072, (512,)), "W2": (131584, (512, 512)),
                "b2": (393728, (512,)), "w3": (394240, (512,)), "b3": (394752, (1,))}


class FFSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ffs error {code}: {msg}")
        self.code = code


class IslandSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("size", ctypes.c_int32), ("p_c", ctypes.c_double), ("p_m", ctypes.c_double),
                ("selection", ctypes.c_int32), ("sweep", ctypes.c_int32)]


class GAConfig(ctypes.Structure):
    _fields_ = [("migration_interval", ctypes.c_int32), ("topology", ctypes.c_int32),
                ("theta", ctypes.c_double), ("surrogate_k", ctypes.c_int32),
                ("surrogate_warmup", ctypes.c_int32)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load the built HIP library (raises if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"HIP library missing: {_LIB_PATH} (build it with __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    pi32 = ctypes.POINTER(i32)
    lib.ffs_ctx_create.argtypes = [P, ctypes.POINTER(P)]
    lib.ffs_ctx_destroy.argtypes = [P]
    lib.ffs_ctx_destroy.restype = None
    lib.ffs_last_error.argtypes = [P]
    lib.ffs_last_error.restype = ctypes.c_char_p
    lib.ffs_create_instance.argtypes = [P, i32, i32, pi32, pi32, ctypes.POINTER(IslandSpec), i32,
                                        ctypes.POINTER(GAConfig), u64, pi32]
    lib.ffs_set_waves_per_block.argtypes = [P, i32]
    lib.ffs_set_mapping.argtypes = [P, i32]
    lib.ffs_set_instance_tile.argtypes = [P, i32, i32, i32]
    lib.ffs_set_concurrent.argtypes = [P, i32]
    lib.ffs_evaluate_noalloc.argtypes = [P, i32, i32, pi32, pi32, P, i32, P]
    lib.ffs_get_mapping.argtypes = [P, pi32]
    lib.ffs_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.ffs_bind_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.ffs_evaluate.argtypes = [P, i32, P, i32, P]
    lib.ffs_evaluate_host.argtypes = [P, i32, pi32, i32, pi32]
    lib.ffs_checkpoint_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.ffs_checkpoint_save.argtypes = [P, P, ctypes.c_size_t]
    lib.ffs_checkpoint_load.argtypes = [P, P, ctypes.c_size_t]
    lib.ffs_evolve.argtypes = [P, i32]
    lib.ffs_migrate.argtypes = [P, i32]
    lib.ffs_best.argtypes = [P, i32, pi32, pi32, pi32]
    lib.ffs_get_population.argtypes = [P, i32, i32, pi32, pi32]
    lib.ffs_generation.argtypes = [P, pi32]
    lib.ffs_migration_counters.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.ffs_set_graphs.argtypes = [P, i32]
    lib.ffs_set_timing.argtypes = [P, i32]
    lib.ffs_kernel_time.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    pf32 = ctypes.POINTER(ctypes.c_float)
    pu16 = ctypes.POINTER(ctypes.c_uint16)
    lib.ffs_surrogate_params.argtypes = [P, i32, pf32]
    lib.ffs_surrogate_set_params.argtypes = [P, i32, pf32]
    lib.ffs_mlp_forward.argtypes = [P, i32, P, i32, P, P, P]
    lib.ffs_mlp_gradients.argtypes = [P, i32, P, P, i32, P, P, P]
    lib.ffs_mlp_train_step.argtypes = [P, i32, P, P, i32]
    lib.ffs_surrogate_candidates.argtypes = [P, i32, i32, pu16, pf32, pf32, pi32]
    lib.ffs_surrogate_choices.argtypes = [P, i32, pi32]
    lib.ffs_surrogate_ring.argtypes = [P, i32, i32, i32, pu16, pf32]
    for name in EXPORTS:
        if name not in ("ffs_ctx_destroy", "ffs_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Context:
    """One library context on a torch CUDA (HIP) stream.

    Usage: add_instance(...) for every instance, then bind(), then evolve /
    evaluate / best / population."""

    def __init__(self, device: int = 0, stream=None, waves_per_block: int | None = None,
                 mapping: int | None = None):
        import torch
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        # a dedicated stream (default priority) so that epochs can be captured as graphs
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        self._check(self.lib.ffs_ctx_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), None)
        self._h = h
        self.ws = None
        self.instances = []
        if waves_per_block is not None:
            self._check(self.lib.ffs_set_waves_per_block(self._h, waves_per_block))
        if mapping is not None:
            self._check(self.lib.ffs_set_mapping(self._h, mapping))

    def _check(self, rc: int, h="self"):
        if rc != FFS_OK:
            msg = self.lib.ffs_last_error(self._h).decode() if h == "self" else "context creation failed"
            raise FFSError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ffs_ctx_destroy(self._h)
            self._h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_instance(self, m, p, islands, interval: int, theta: float = 1.0, topology: int = 0,
                     seed: int = 1, surrogate_k: int = 0, surrogate_warmup: int = 5) -> int:
        m = _i32(m)
        p = _i32(p)
        n, S = p.shape
        specs = (IslandSpec * len(islands))()
        for i, x in enumerate(islands):
            specs[i] = IslandSpec(int(x["kind"]), int(x.get("rows", 0)), int(x.get("cols", 0)),
                                  int(x.get("size", 0)), float(x["pc"]), float(x["pm"]), int(x.get("sel", 0)),
                                  int(x.get("sweep", 0)))
        cfg = GAConfig(int(interval), int(topology), float(theta), int(surrogate_k), int(surrogate_warmup))
        out = ctypes.c_int32()
        self._check(self.lib.ffs_create_instance(self._h, n, S, _p32(m), _p32(p), specs, len(islands),
                                                 ctypes.byref(cfg), ctypes.c_uint64(seed), ctypes.byref(out)))
        sizes = [int(x["rows"]) * int(x["cols"]) if int(x["kind"]) == 0 else int(x["size"]) for x in islands]
        self.instances.append(dict(n=n, S=S, sizes=sizes, args=dict(m=m, p=p, islands=[dict(x) for x in islands],
                                                                     interval=interval, theta=theta,
                                                                     topology=topology, seed=seed,
                                                                     surrogate_k=surrogate_k,
                                                                     surrogate_warmup=surrogate_warmup)))
        return out.value

    def workspace_size(self) -> int:
        b = ctypes.c_size_t()
        self._check(self.lib.ffs_workspace_size(self._h, ctypes.byref(b)))
        return int(b.value)

    def bind(self):
        torch = self._torch
        nbytes = self.workspace_size()
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.ws.data_ptr()
        ptr = (ptr + 255) & ~255
        self._check(self.lib.ffs_bind_workspace(self._h, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes)))

    def evaluate(self, inst: int, perms, check: bool = True):
        """Makespans (torch int32, device) of the rows of `perms`."""
        torch = self._torch
        t = perms if isinstance(perms, torch.Tensor) else torch.from_numpy(_i32(perms))
        t = t.to(device=self.device, dtype=torch.int32).contiguous()
        count = t.shape[0]
        out = torch.empty(count, dtype=torch.int32, device=self.device)
        # the input was produced on the caller's stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        rc = self.lib.ffs_evaluate(self._h, inst, ctypes.c_void_p(t.data_ptr()), count,
                                   ctypes.c_void_p(out.data_ptr()))
        if check:
            self._check(rc)
        return out if check else (out, rc)

    def evaluate_host(self, inst: int, perms) -> tuple[np.ndarray, int]:
        """Makespans (numpy int32) of host rows through the host-pointer entry
        point; returns (makespans, status)."""
        a = _i32(perms)
        out = np.zeros(a.shape[0], dtype=np.int32)
        rc = self.lib.ffs_evaluate_host(self._h, inst, _p32(a), a.shape[0], _p32(out))
        return out, rc

    def checkpoint(self) -> bytes:
        """Byte image of the whole context at its current generation."""
        n = ctypes.c_size_t()
        self._check(self.lib.ffs_checkpoint_size(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.ffs_checkpoint_save(self._h, buf, n))
        return buf.raw

    def restore(self, image: bytes):
        """Load a checkpoint taken from a context with the same instances."""
        buf = ctypes.create_string_buffer(bytes(image), len(image))
        self._check(self.lib.ffs_checkpoint_load(self._h, buf, ctypes.c_size_t(len(image))))

    def evolve(self, generations: int):
        self._check(self.lib.ffs_evolve(self._h, int(generations)))

    def migrate(self, inst: int):
        self._check(self.lib.ffs_migrate(self._h, inst))

    def best(self, inst: int) -> dict:
        n = self.instances[inst]["n"]
        mk = ctypes.c_int32()
        gen = ctypes.c_int32()
        perm = np.zeros(n, dtype=np.int32)
        self._check(self.lib.ffs_best(self._h, inst, ctypes.byref(mk), ctypes.byref(gen), _p32(perm)))
        return dict(makespan=mk.value, generation=gen.value, perm=perm)

    def population(self, inst: int, island: int):
        info = self.instances[inst]
        N = info["sizes"][island]
        genes = np.zeros((N, info["n"]), dtype=np.int32)
        mk = np.zeros(N, dtype=np.int32)
        self._check(self.lib.ffs_get_population(self._h, inst, island, _p32(genes), _p32(mk)))
        return genes, mk

    @property
    def generation(self) -> int:
        g = ctypes.c_int32()
        self._check(self.lib.ffs_generation(self._h, ctypes.byref(g)))
        return g.value

    def migration_counters(self, inst: int):
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        self._check(self.lib.ffs_migration_counters(self._h, inst, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_waves_per_block(self, waves: int):
        self._check(self.lib.ffs_set_waves_per_block(self._h, int(waves)))

    def set_mapping(self, mapping: int):
        """-1 automatic, 0 one lane per stage, 1 one lane per chromosome (ffs_set_mapping)."""
        self._check(self.lib.ffs_set_mapping(self._h, int(mapping)))

    def set_instance_tile(self, inst: int, mapping: int = -1, waves: int = 0):
        """Tile of one instance (ffs_set_instance_tile): mapping -1/0/1, waves 0/1/2/4/8."""
        self._check(self.lib.ffs_set_instance_tile(self._h, int(inst), int(mapping), int(waves)))

    def set_concurrent(self, enable: bool):
        """Run a generation's launches side by side (True, the default) or in turn."""
        self._check(self.lib.ffs_set_concurrent(self._h, 1 if enable else 0))

    def set_chains(self, chains: int):
        """Launch chains of island groups: 1, 2 or -1 (automatic)."""
        self._check(self.lib.ffs_set_chains(self._h, int(chains)))

    def chains(self) -> int:
        used = ctypes.c_int32()
        self._check(self.lib.ffs_get_chains(self._h, ctypes.byref(used)))
        return int(used.value)

    def mapping(self) -> int:
        """Mapping the generation launches use: 0 per stage, 1 per lane, 2 mixed."""
        v = ctypes.c_int32()
        self._check(self.lib.ffs_get_mapping(self._h, ctypes.byref(v)))
        return v.value

    def set_graphs(self, enable: bool):
        self._check(self.lib.ffs_set_graphs(self._h, 1 if enable else 0))

    def set_timing(self, enable: bool):
        self._check(self.lib.ffs_set_timing(self._h, 1 if enable else 0))

    def kernel_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.lib.ffs_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ---- learned pre-screen -------------------------------------------------
    def _ptr(self, t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    def surrogate_params(self, inst: int = 0) -> np.ndarray:
        out = np.zeros(N_PARAMS, dtype=np.float32)
        self._check(self.lib.ffs_surrogate_params(self._h, inst, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_surrogate_params(self, params, inst: int = 0):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        assert a.shape == (N_PARAMS,)
        self._check(self.lib.ffs_surrogate_set_params(self._h, inst, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def mlp_forward(self, X, inst: int = 0):
        """X: torch uint16-as-int16 BF16 bits [rows][256] on the device -> (y, H1, H2)."""
        torch = self._torch
        rows = X.shape[0]
        y = torch.empty(rows, dtype=torch.float32, device=self.device)
        H1 = torch.empty((rows, 512), dtype=torch.int16, device=self.device)
        H2 = torch.empty((rows, 512), dtype=torch.int16, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.lib.ffs_mlp_forward(self._h, inst, self._ptr(X), rows, self._ptr(y), self._ptr(H1), self._ptr(H2)))
        return y, H1, H2

    def mlp_gradients(self, X, t, inst: int = 0):
        torch = self._torch
        rows = X.shape[0]
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        dZ2 = torch.empty((rows, 512), dtype=torch.int16, device=self.device)
        dZ1 = torch.empty((rows, 512), dtype=torch.int16, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.lib.ffs_mlp_gradients(self._h, inst, self._ptr(X), self._ptr(t), rows, self._ptr(g),
                                               self._ptr(dZ2), self._ptr(dZ1)))
        return g, dZ2, dZ1

    def mlp_train_step(self, X, t, inst: int = 0):
        torch = self._torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self.lib.ffs_mlp_train_step(self._h, inst, self._ptr(X), self._ptr(t), X.shape[0]))

    def surrogate_candidates(self, inst: int = 0, exact: bool = False, features: bool = False):
        info = self.instances[inst]
        k = int(info["args"]["surrogate_k"])
        cells = sum(s for s, x in zip(info["sizes"], info["args"]["islands"]) if int(x["kind"]) == 0)
        pred = np.zeros(cells * k, dtype=np.float32)
        ex = np.zeros(cells * k, dtype=np.float32) if exact else None
        X = np.zeros((cells * k, 256), dtype=np.uint16) if features else None
        ch = np.zeros(cells, dtype=np.int32)
        pf = ctypes.POINTER(ctypes.c_float)
        self._check(self.lib.ffs_surrogate_candidates(
            self._h, inst, 1 if exact else 0,
            X.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)) if X is not None else None,
            pred.ctypes.data_as(pf), ex.ctypes.data_as(pf) if ex is not None else None, _p32(ch)))
        return dict(pred=pred.reshape(cells, k), exact=None if ex is None else ex.reshape(cells, k),
                    features=None if X is None else X.reshape(cells, k, 256), choice=ch)

    def surrogate_choices(self, inst: int = 0) -> np.ndarray:
        info = self.instances[inst]
        cells = sum(s for s, x in zip(info["sizes"], info["args"]["islands"]) if int(x["kind"]) == 0)
        ch = np.zeros(cells, dtype=np.int32)
        self._check(self.lib.ffs_surrogate_choices(self._h, inst, _p32(ch)))
        return ch

    def surrogate_ring(self, first: int, count: int, inst: int = 0):
        X = np.zeros((count, 256), dtype=np.uint16)
        t = np.zeros(count, dtype=np.float32)
        self._check(self.lib.ffs_surrogate_ring(self._h, inst, first, count,
                                                X.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                                                t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return X, t


def evaluate_noalloc(m, p, perms, out, stream=None) -> int:
    """ffs_evaluate_noalloc: makespans of the rows of `perms` (torch int32
    [count, n] on the current device) into `out` (torch int32 [count], same
    device) for the instance (m, p) given here, without a context or
    workspace.  Returns the status code (FFS_OK, or FFS_EINVAL when some rows
    are not permutations); other failures raise FFSError."""
    import torch
    lib = load_library()
    m = _i32(m)
    p = _i32(p)
    n, S = p.shape
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.ffs_evaluate_noalloc(ctypes.c_void_p(st.cuda_stream), int(n), int(S), _p32(m), _p32(p.reshape(-1)),
                                  ctypes.c_void_p(perms.data_ptr()), int(perms.shape[0]),
                                  ctypes.c_void_p(out.data_ptr()))
    if rc not in (FFS_OK, FFS_EINVAL):
        raise FFSError(rc, "ffs_evaluate_noalloc failed")
    return rc
