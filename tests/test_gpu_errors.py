"""Failure handling through the C ABI: every error is a status, never a crash (GPU)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

from gpu_cases import ctx, to_dev

pytestmark = pytest.mark.gpu


def _status(fn):
    import paper_2603_10586_amd as q
    with pytest.raises(q.QrvieError) as e:
        fn()
    return e.value.status


def test_invalid_geometry_inputs():
    import paper_2603_10586_amd as q
    c = ctx()
    a = W.lattice(3, 2)
    a.centers[1, 0] = np.nan
    assert _status(lambda: q.Geometry(c, a)) == 1                      # non-finite centre
    b = W.lattice(3, 2)
    b.radius[2] = -0.1
    assert _status(lambda: q.Geometry(c, b)) == 1                      # negative radius
    d = W.lattice(3, 2)
    d.lattice_ij[4] = d.lattice_ij[1]
    assert _status(lambda: q.Geometry(c, d)) == 2                      # two particles on one site
    e = W.lattice(2, 2)
    e.cells_per_particle = 40
    assert _status(lambda: q.Geometry(c, e)) == 1
    empty = W.lattice(2, 2)                                            # no particles at all
    for f, shape in (("centers", (0, 3)), ("lattice_ij", (0, 2)), ("radius", (0,)), ("height", (0,)),
                     ("eps_r", (0,))):
        setattr(empty, f, np.zeros(shape, dtype=getattr(empty, f).dtype))
    assert _status(lambda: q.Geometry(c, empty)) == 1


def test_invalid_operator_and_solve_options():
    import paper_2603_10586_amd as q
    c = ctx()
    g = q.Geometry(c, W.random_lattice(3, 3, seed=1))
    assert _status(lambda: q.Operator(c, g, eps=0.0)) == 1
    assert _status(lambda: q.Operator(c, g, eps=-1e-6)) == 1
    op = q.Operator(c, g, eps=1e-6)
    v = q.rhs_plane_waves(c, g, [0.0], [0.0], [1])
    assert _status(lambda: op.solve(v, restart=0)) == 1
    assert _status(lambda: op.solve(v, tol=0.0)) == 1
    assert _status(lambda: q.rhs_plane_waves(c, g, [0.0], [0.0], [2])) == 1   # bad polarisation
    # NaN right-hand side
    bad = v.clone()
    bad[0, 3] = complex("nan")
    assert _status(lambda: op.solve(bad)) == 1
    # zero right-hand side: x = 0, converged
    x, info, st = op.solve(v * 0)
    assert st == 0 and info[0]["converged"] and float(x.abs().max()) == 0.0


def test_binding_refuses_tensors_the_kernels_cannot_take():
    import torch
    import paper_2603_10586_amd as q
    c = ctx()
    g = q.Geometry(c, W.random_lattice(3, 3, seed=1))
    op = q.Operator(c, g, eps=1e-6)
    v = q.rhs_plane_waves(c, g, [0.0, 10.0], [0.0, 0.0], [1, 0])
    n = g.ndof
    with pytest.raises(TypeError):
        op.apply(v.to(torch.complex64))                                    # wrong dtype
    with pytest.raises(ValueError):
        op.apply(v[:, : n - 1])                                            # wrong length
    with pytest.raises(ValueError):
        op.precondition(torch.zeros(n, 2, dtype=torch.complex128, device=v.device).t())   # strided
    with pytest.raises(ValueError):
        op.solve(v, x0=torch.zeros(1, n, dtype=torch.complex128, device=v.device))    # x0 too small
    with pytest.raises(ValueError):
        op.apply(v.cpu())                                                  # host memory
    with pytest.raises(ValueError):
        c.probe_read(torch.ones(1024, dtype=torch.float64))                # host memory
    # no right-hand sides: refused by the library, not launched
    assert _status(lambda: op.apply(torch.zeros(0, n, dtype=torch.complex128, device=v.device))) == 1
    assert _status(lambda: op.solve(torch.zeros(0, n, dtype=torch.complex128, device=v.device))) == 1
    # the valid call still works after the refusals
    x, info, st = op.solve(v, x0=torch.zeros_like(v), tol=1e-8, restart=200, max_iter=400)
    assert st == 0 and all(i["converged"] for i in info)


def test_hbm_budget_refuses_an_operator_that_does_not_fit():
    import paper_2603_10586_amd as q
    tight = q.Context(0, hbm_budget=4 << 20)
    g = q.Geometry(tight, W.random_lattice(6, 6, seed=3))
    used = tight.bytes_in_use()
    assert 0 < used < 4 << 20                                          # only the geometry is held
    assert _status(lambda: q.Operator(tight, g, eps=1e-6)) == 3
    assert tight.bytes_in_use() == used                                # nothing leaked by the refusal
    g.close()
    assert tight.bytes_in_use() == 0
    tight.close()


def test_footprint_estimate_bounds_the_operator():
    import paper_2603_10586_amd as q
    c = ctx()
    g = q.Geometry(c, W.random_lattice(6, 5, seed=4))
    est = q.Operator.footprint_estimate(g, eps=1e-6)
    op = q.Operator(c, g, eps=1e-6)
    assert op.stats()["device_bytes"] <= est


def test_happy_breakdown_single_particle():
    """One particle: the preconditioner is exact, GMRES stops after one step (§4)."""
    import paper_2603_10586_amd as q
    c = ctx()
    g = q.Geometry(c, W.lattice(1, radius=0.2))
    op = q.Operator(c, g, eps=1e-6)
    v = q.rhs_plane_waves(c, g, [0.0], [0.0], [1])
    x, info, st = op.solve(v, restart=10, tol=1e-12)
    assert st == 0 and info[0]["iterations"] <= 1
