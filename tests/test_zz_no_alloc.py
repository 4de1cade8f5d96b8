"""The no-allocation product entry point against the allocating one, through the C ABI.

qrvie_apply_noalloc runs the same kernels as qrvie_apply with its workspaces in the
library's fixed per-device scratch array, so its result must equal qrvie_apply's bit for
bit.  Two calls in a row, the second on a smaller operator, check that the array's leftover
contents from the first call do not leak into the second; the library's allocation
counters must not move during the calls; an operator whose product needs more than the
fixed scratch is refused with an error.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _setup(arr, c, cap=0, shared=False):
    import paper_2603_10586_amd as q
    geom = q.Geometry(c, arr)
    op = q.Operator(c, geom, eps=1e-6, max_block_rows=cap, share_transpose=shared)
    return geom, op


def _noalloc(c, op, x, y):
    st = c.lib.qrvie_apply_noalloc(c.h, op.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    return st


def test_noalloc_product_equals_the_allocating_product_twice_in_a_row():
    import torch
    import paper_2603_10586_amd as q
    c = q.Context(0)
    cases = []
    # the mid-size workload (32 x 32), then smaller arrays, one with transpose-shared factors
    for arr, seed, sh in ((W.mid(0), 0, False), (W.random_lattice(8, 8, seed=2), 1, True),
                          (W.random_lattice(5, 3, seed=11), 2, False)):
        geom, op = _setup(arr, c, shared=sh)
        rng = np.random.default_rng(seed)
        xh = rng.standard_normal(geom.ndof) + 1j * rng.standard_normal(geom.ndof)
        cases.append((geom, op, torch.from_numpy(xh).to("cuda")))
    for geom, op, x in cases:
        print(f"[noalloc] n={geom.ndof}", flush=True)
        ref = op.apply(x).cpu().numpy()
        y = torch.full_like(x, complex(np.nan, np.nan))
        used, peak = c.bytes_in_use(), c.peak_bytes(reset=True)
        c.order()
        assert _noalloc(c, op, x, y) == 0, c.lib.qrvie_last_error(c.h)
        c.stream.synchronize()
        assert c.bytes_in_use() == used and c.peak_bytes() == used      # no library allocation
        got = y.cpu().numpy()
        assert np.array_equal(got, ref)
    c.close()


def test_noalloc_refuses_an_operator_beyond_the_fixed_scratch():
    import torch
    import paper_2603_10586_amd as q
    c = q.Context(0)
    geom, op = _setup(W.random_lattice(48, 48, seed=3), c, cap=9216)
    x = torch.zeros(geom.ndof, dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    assert _noalloc(c, op, x, y) == 1                                   # QRVIE_ERR_INVALID_ARG
    assert b"scratch" in c.lib.qrvie_last_error(c.h)
    with pytest.raises(q.QrvieError):
        op.apply_noalloc(x, y)
    op.close()
    geom.close()
    c.close()
