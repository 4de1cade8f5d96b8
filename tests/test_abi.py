"""The C-ABI library loads on the CPU and exports every symbol the header declares (no GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qrvie.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(qrvie_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_problem_statement_calls():
    names = declared_functions()
    for required in ("qrvie_geom_create", "qrvie_op_create", "qrvie_apply", "qrvie_precondition",
                     "qrvie_solve", "qrvie_rhs_plane_waves"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2603_10586_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libqrvie.so is not built (run __graft_entry__.build())")
    import ctypes
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's calls
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_status_strings_without_a_device():
    from paper_2603_10586_amd import _lib
    lib = _lib.load()
    assert lib.qrvie_status_string(0) == b"ok"
    assert lib.qrvie_status_string(5) == b"not converged"


def test_context_creation_fails_cleanly_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes
    from paper_2603_10586_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.qrvie_ctx_create(0, None, 0, ctypes.byref(h))
    assert st == _lib.ERR_DEVICE and not h.value


def test_entry_points_reject_null_handles_without_a_device():
    """Argument checks run before any device work: null handles give QRVIE_ERR_INVALID_ARG."""
    import ctypes
    from paper_2603_10586_amd import _lib
    lib = _lib.load()
    out = ctypes.c_double()
    assert lib.qrvie_probe_read(None, None, 16, 1, ctypes.byref(out)) == _lib.ERR_INVALID_ARG
    assert lib.qrvie_probe_mfma(None, 1, ctypes.byref(out)) == _lib.ERR_INVALID_ARG
    t = _lib.BlockTune()
    assert lib.qrvie_op_tune_block(None, None, 0, 16, 1, ctypes.byref(t)) == _lib.ERR_INVALID_ARG
    ms = (ctypes.c_double * 4)()
    fl = (ctypes.c_int64 * 4)()
    assert lib.qrvie_op_profile_block(None, None, 16, 1, ms, fl) == _lib.ERR_INVALID_ARG
    assert lib.qrvie_solve(None, None, 1, None, 1, None, 1, None, None) == _lib.ERR_INVALID_ARG


def test_binding_refuses_host_tensors_before_any_library_call():
    import torch
    from paper_2603_10586_amd import api
    n = 144
    with pytest.raises(TypeError):
        api._cols([0j] * n, n, 0, "apply")
    with pytest.raises(ValueError):
        api._cols(torch.zeros(2, n, dtype=torch.complex128), n, 0, "apply")        # host memory
    with pytest.raises(ValueError):
        api._device_tensor(torch.zeros(16, dtype=torch.float64), 0, "probe read")


def test_array_descriptor_refuses_mismatched_lengths():
    import numpy as np
    import workloads as W
    from paper_2603_10586_amd import api
    a = W.random_lattice(3, seed=1)
    d, keep = api.array_desc(a)
    assert d.n == 9 and d.n_eps in (1, 9)
    for field, bad in (("radius", a.radius[:-1]), ("height", a.height[:4]), ("lattice_ij", a.lattice_ij[:, :1]),
                       ("eps_r", a.eps_r[:2]), ("centers", a.centers[:, :2])):
        b = W.random_lattice(3, seed=1)
        setattr(b, field, bad)
        with pytest.raises(ValueError):
            api.array_desc(b)
    one_eps = W.random_lattice(3, seed=1)
    one_eps.eps_r = np.asarray([12 + 0.1j])
    assert api.array_desc(one_eps)[0].n_eps == 1


C_CLIENT = r"""
#include <stdio.h>
#include <string.h>
#include "qrvie.h"
int main(void) {
    if (strcmp(qrvie_status_string(QRVIE_OK), "ok") != 0) return 1;
    if (qrvie_geom_ndof(NULL) != 0) return 2;
    if (qrvie_solve(NULL, NULL, 1, NULL, 0, NULL, 0, NULL, NULL) != QRVIE_ERR_INVALID_ARG) return 3;
    if (qrvie_apply(NULL, NULL, 1, NULL, 0, NULL, 0) != QRVIE_ERR_INVALID_ARG) return 4;
    printf("ok\n");
    return 0;
}
"""


def test_header_is_plain_c_and_a_c_program_links_the_library(tmp_path):
    import shutil
    import subprocess
    from paper_2603_10586_amd import _lib
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "client.c"
    src.write_text(C_CLIENT)
    exe = tmp_path / "client"
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-L", libdir, "-lqrvie", f"-Wl,-rpath,{libdir}", "-Wl,-rpath-link,/opt/rocm/lib",
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stderr)
