"""Host logic of bench.py that needs no GPU: the device-code digest that
gates the recorded HBM traffic, the lookup of that figure in the committed
rocprofv3 summaries, and the guard that keeps non-finite numbers out of the
JSON line."""
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _profile_fields(path):
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    return vals


def test_digest_depends_on_every_source_byte():
    csrc = os.path.join(ROOT, "paper_1903_10722_amd", "csrc")

    def read(f, extra=b""):
        with open(os.path.join(csrc, f), "rb") as fh:
            return fh.read() + extra

    for sources in (bench.KERNEL_SOURCES, bench.TT_KERNEL_SOURCES):
        base = bench.source_digest(sources=sources)
        assert base == bench.source_digest(read=read, sources=sources)
        last = sources[-1]
        changed = bench.source_digest(read=lambda f: read(f, b" " if f == last else b""), sources=sources)
        assert changed != base


@pytest.mark.parametrize("kernel,workload,sources", [("k_generation", "medium", "main"),
                                                     ("k_generation", "large", "main"),
                                                     ("k_tt_generation", "section5", "tt")])
def test_recorded_traffic_follows_the_digest(kernel, workload, sources):
    srcs = bench.KERNEL_SOURCES if sources == "main" else bench.TT_KERNEL_SOURCES
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    assert os.path.exists(path), path
    vals = _profile_fields(path)
    got = bench.recorded_traffic(kernel, workload, srcs)
    if vals.get("source_sha256") == bench.source_digest(sources=srcs):
        assert got == float(vals["hbm_bytes_per_launch"])
    else:
        assert got is None


def test_recorded_traffic_missing_profile_is_none():
    assert bench.recorded_traffic("no_such_kernel", "no_such_workload") is None


def test_non_finite_numbers_become_null():
    assert bench._finite_or_none(float("nan")) is None
    assert bench._finite_or_none(float("inf")) is None
    assert bench._finite_or_none(-float("inf")) is None
    assert bench._finite_or_none(0.25) == 0.25
    assert not math.isnan(bench._finite_or_none(0.0))


def test_host_cpu_is_text():
    assert isinstance(bench.host_cpu(), str)


def test_cpu_baseline_runs_the_oracle_on_one_core():
    """The CPU baseline times the oracle in a child process pinned to one
    core, on the named workload (tiny here, briefly)."""
    import oracle
    oracle.build()
    r = bench.cpu_baseline("tiny", 1, 0.5)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "decodes/s"
    assert r["value"] > 0 and len(r["affinity"]) == 1
    assert "tiny workload" in r["sample"]
