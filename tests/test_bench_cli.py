"""The benchmark's command line on the CPU: the contract's flags exist, and a request for
more than one GPU exits with a message instead of running (one GPU is driven)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_contract_flags_are_accepted():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--mixed-ir", "--block", "--serving", "--ir-reference"):
        assert flag in r.stdout, flag


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _no_device():
    import torch
    return torch.cuda.device_count() == 0


def test_bench_and_smoke_fail_loudly_without_a_gpu():
    import pytest
    if not _no_device():
        pytest.skip("a device is present")
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode != 0 and '"metric"' not in r.stdout        # no number from any other route
    s = subprocess.run([sys.executable, "-c", "import __graft_entry__ as g; g.smoke()"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert s.returncode != 0 and "smoke ok" not in s.stdout
