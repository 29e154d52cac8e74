"""Host-side checks of the benchmark's contract (no GPU): one GPU only, the
command line, and the rule that ties a committed traffic measurement to the
kernel source it was taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_flags():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--no-cpu", "--no-transport", "--no-slab", "--no-pulse",
                 "--only", "--no-autotune", "--copy-probe"):
        assert flag in r.stdout, flag


@pytest.fixture()
def bench_module():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_unknown_leg_is_refused():
    r = _run("--only", "long_chain,nonsense")
    assert r.returncode == 2 and "nonsense" in r.stderr


def test_traffic_is_reported_only_for_the_measured_source(bench_module):
    """The committed traffic figure belongs to the kernel source whose hash it
    records; any other source reads as unmeasured (None)."""
    path = os.path.join(ROOT, "profiles", "k_draw_hash_2p26_traffic.txt")
    vals = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    sha = vals["kernel_source_sha256"].strip()
    assert bench_module.traffic_from_profiles(sha) == float(vals["hbm_bytes_per_launch"])
    assert bench_module.traffic_from_profiles("0" * 64) is None
    # fetch and write add up to the reported total, above the algorithmic 12 bytes per stream
    total = float(vals["hbm_fetch_bytes_per_launch"]) + float(vals["hbm_write_bytes_per_launch"])
    assert abs(total - float(vals["hbm_bytes_per_launch"])) <= 1.0
    assert float(vals["hbm_bytes_per_launch"]) >= int(vals["algorithmic_bytes_per_launch"]) == 12 * (1 << 26)
