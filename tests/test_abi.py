"""The C-ABI library builds, loads and exports every entry point that
include/ffs.h and include/ffs_tt.h declare (no device calls: runs without a
GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1903_10722_amd import binding
from paper_1903_10722_amd.build import build_library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("ffs.h", "ffs_tt.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(ffs_[a-z_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(binding.library_path()):
        build_library()
    return binding.library_path()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["ffs_create_instance", "ffs_evaluate", "ffs_evolve", "ffs_migrate", "ffs_best"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ffs_[a-z_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    from paper_1903_10722_amd import tardiness
    assert sorted(binding.EXPORTS + tardiness.TT_EXPORTS) == sorted(_declared())


def test_library_loads_and_reports_errors_without_device(lib_path):
    lib = binding.load_library()
    for n in _declared():
        assert hasattr(lib, n)
    # argument checks that need no device
    assert lib.ffs_ctx_create(None, None) == binding.FFS_EINVAL
    assert lib.ffs_last_error(None) == b"null context"
    from paper_1903_10722_amd import tardiness
    tl = tardiness.load()
    assert tl.ffs_tt_create(None, None) == binding.FFS_EINVAL
    assert tl.ffs_tt_last_error(None) == b"null context"
    assert tl.ffs_tt_evolve(None, 1) == binding.FFS_EINVAL
    assert tl.ffs_tt_set_update(None, 1) == binding.FFS_EINVAL


def test_oracle_and_library_share_no_code():
    """The oracle is plain C built by gcc; the HIP sources never include it and
    the oracle never includes the HIP headers."""
    csrc = os.path.join(ROOT, "paper_1903_10722_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower()
    otxt = open(os.path.join(ROOT, "oracle", "ffs_oracle.c")).read()
    assert "#include \"" not in otxt
    for f in os.listdir(os.path.join(ROOT, "paper_1903_10722_amd")):
        if f.endswith(".py"):
            assert "import oracle" not in open(os.path.join(ROOT, "paper_1903_10722_amd", f)).read()


def test_island_variants_hold_8192_individuals():
    """Host-side check of the ablation layouts: every layout holds the same
    8192 individuals per generation on the same instance."""
    from paper_1903_10722_amd import inputs
    base = inputs.island_variant("dual")
    for v in inputs.ISLAND_VARIANTS:
        w = inputs.island_variant(v)
        assert sum(x["size"] for x in w["islands"]) == 8192
        assert (w["p"] == base["p"]).all() and (w["m"] == base["m"]).all()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with a message."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
