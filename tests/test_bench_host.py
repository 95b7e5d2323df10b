"""Host-side logic of bench.py, no GPU: the algorithmic bytes per fluid
node (every population read and written once, 2 Q S, plus the PR relaxation
time read and written: FP64 in FP64 runs, FP32 otherwise), the refusal of
more than one GPU, and that a traffic figure taken on other kernel sources
is not reported."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("lattice,q", [("D2Q9", 9), ("D3Q19", 19), ("D3Q27", 27)])
def test_algorithmic_bytes_per_node(lattice, q):
    f = bench.algorithmic_bytes_per_node
    for prec, s in (("FP64", 8), ("FP32", 4), ("FP16", 2)):
        assert f(lattice, "IR", prec) == 2 * q * s
        assert f(lattice, "PRI", prec) == 2 * q * s  # implicit tau: no field
        assert f(lattice, "IRHB", prec) == 2 * q * s
        assert f(lattice, "PR", prec) == 2 * q * s + 2 * (8 if prec == "FP64" else 4)


def test_headline_bytes():
    # D3Q27 FP64: 432 B (IR), 448 B (PR); FP16-shifted with an FP32 tau: 108 / 116 B
    assert bench.algorithmic_bytes_per_node("D3Q27", "IR", "FP64") == 432
    assert bench.algorithmic_bytes_per_node("D3Q27", "PR", "FP64") == 448
    assert bench.algorithmic_bytes_per_node("D3Q27", "IR", "FP16") == 108
    assert bench.algorithmic_bytes_per_node("D3Q27", "PR", "FP16") == 116


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       timeout=120, env=dict(os.environ, **env))
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_traffic_only_for_matching_kernel_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.kernel_source_hash() == h  # deterministic
    assert bench.traffic_from_profile("0" * 16, 1) is None
