"""The seeded input recipes (no GPU): sizes, ranges and structure of every workload, and
that the same seed gives the same inputs on every run."""
import math

import numpy as np

import workloads as W


def _check_lattice(a, nx, ny, pitch=0.5):
    n = nx * ny
    assert a.n_particles == n and a.centers.shape == (n, 3) and a.lattice_ij.shape == (n, 2)
    assert len({tuple(ij) for ij in a.lattice_ij}) == n                     # one particle per site
    i, j = a.lattice_ij[:, 0], a.lattice_ij[:, 1]
    assert i.min() == 0 and i.max() == nx - 1 and j.min() == 0 and j.max() == ny - 1
    assert np.allclose(a.centers[:, 0], (i - (nx - 1) / 2) * pitch)       # centred on the origin
    assert np.allclose(a.centers[:, 1], (j - (ny - 1) / 2) * pitch)
    assert np.all(a.centers[:, 2] == 0)
    assert np.all(2 * a.radius <= pitch + 1e-15)                           # disks never overlap
    assert np.all(a.height == 0.1) and np.all(a.eps_r == 12 + 0.1j)


def test_fixed_workloads_have_their_stated_shapes():
    t = W.tiny()
    _check_lattice(t, 4, 4)
    assert np.all(t.radius == 0.2)
    m = W.mid()
    _check_lattice(m, 32, 32)
    assert m.ndof == 1024 * 144 and 0.15 <= m.radius.min() and m.radius.max() <= 0.25
    assert abs(m.radius.mean() - 0.2) < 0.005                              # uniform on [0.15, 0.25]
    p = W.precision()
    _check_lattice(p, 96, 96)
    assert 0.15 <= p.radius.min() and p.radius.max() <= 0.25


def test_graded_metalens_profile_at_hand_computed_sites():
    b = W.batching()
    _check_lattice(b, 64, 64)
    assert 0.15 <= b.radius.min() and b.radius.max() < 0.25
    focal = 64 * 0.5
    for i, j in ((31, 31), (0, 0), (63, 10), (40, 5)):
        x, y = (i - 31.5) * 0.5, (j - 31.5) * 0.5
        turns = (x * x + y * y) / (2 * focal)                              # phi / 2pi, phi = pi rho^2 / F
        want = 0.15 + 0.1 * (turns - math.floor(turns))
        p = int(np.flatnonzero((b.lattice_ij[:, 0] == i) & (b.lattice_ij[:, 1] == j))[0])
        assert abs(b.radius[p] - want) < 1e-12
    assert len(np.unique(np.round(b.radius, 12))) > 100                    # a graded profile, not a constant


def test_serving_stream_follows_its_recipe():
    reqs = W.serving_requests(256, seed=0, rate_per_s=0.2)
    assert len(reqs) == 256
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 5.0) < 1.0                           # Poisson, mean gap 1 / rate
    sides = np.array([r.array.nx for r in reqs])
    assert sides.min() >= 8 and sides.max() <= 48 and len(np.unique(sides)) > 20
    for r in reqs:
        _check_lattice(r.array, r.array.nx, r.array.nx)
        assert 1 <= r.incidence.nrhs <= 16
        assert np.all(np.abs(r.incidence.theta_deg) <= 30) and set(r.incidence.pol) <= {0, 1}
        assert r.tol == 1e-6


def test_same_seed_same_inputs_and_other_seeds_differ():
    assert np.array_equal(W.mid(0).radius, W.mid(0).radius)
    assert not np.array_equal(W.mid(0).radius, W.mid(1).radius)
    a, b = W.serving_requests(8, seed=3), W.serving_requests(8, seed=3)
    for ra, rb in zip(a, b):
        assert ra.arrival_s == rb.arrival_s and np.array_equal(ra.array.radius, rb.array.radius)
        assert np.array_equal(ra.incidence.theta_deg, rb.incidence.theta_deg)
