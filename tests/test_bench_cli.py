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


def test_cpu_solve_extrapolation_is_consistent_on_a_small_array():
    """The extrapolated per-solve CPU figures add up as stated: iterations x (product +
    preconditioner) + projections, with the product at the given rate and the projections
    growing as iterations (iterations + 1) / 2 basis vectors."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    a = bench.cpu_solve_extrapolation(W.tiny(), iterations=10, product_bytes=2e9, cpu_gbs=4.0, seconds=0.5)
    b = bench.cpu_solve_extrapolation(W.tiny(), iterations=20, product_bytes=2e9, cpu_gbs=4.0, seconds=0.5)
    for r, it in ((a, 10), (b, 20)):
        s = r["solve_extrapolated"]
        assert s["iterations"] == it and abs(s["compressed_product_s"] - 0.5) < 1e-12
        assert s["preconditioner_s"] > 0 and s["arnoldi_s"] > 0
        total = it * (s["compressed_product_s"] + s["preconditioner_s"]) + s["arnoldi_s"]
        assert abs(s["solve_s"] - total) <= 1e-3 * total
        assert r["matrix_free_dense_product"]["particle_rows_timed"] >= 1
        assert r["matrix_free_dense_product"]["s_extrapolated"] > 0
    # 20 steps project onto 210 basis vectors in all, 10 steps onto 55 (per-vector times are
    # timed separately in the two calls, so only the order of the ratio is fixed)
    ratio = b["solve_extrapolated"]["arnoldi_s"] / a["solve_extrapolated"]["arnoldi_s"]
    assert 210 / 55 / 3 < ratio < 210 / 55 * 3
