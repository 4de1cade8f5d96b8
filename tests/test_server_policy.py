"""The solve server's admission policy (host code, no GPU): built with g++ from the library's
own header and run; plus option validation through the C ABI."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "policy_test"
    src = os.path.join(ROOT, "tests", "server_policy_test.cpp")
    inc = os.path.join(ROOT, "paper_2603_10586_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"


def test_server_rejects_invalid_options():
    from paper_2603_10586_amd import _lib as L
    lib = L.load()
    h = C.c_void_p()
    for bad in (dict(slots=0), dict(slots=17), dict(hbm_budget=0), dict(eps=0.0), dict(mode=1),
                dict(block_width=65), dict(op_cache=-1), dict(restart=0), dict(tune_tiles=2), dict(max_bypass=-1)):
        o = dict(slots=2, hbm_budget=1 << 30, eps=1e-6, restart=100, max_iter=100, mode=L.SOLVE_BLOCK,
                 block_width=0, op_cache=1, seed=0)
        o.update(bad)
        assert lib.qrvie_server_create(0, C.byref(L.ServerOptsC(**o)), C.byref(h)) == L.ERR_INVALID_ARG, bad
