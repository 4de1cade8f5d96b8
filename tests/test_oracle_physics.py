"""Pins of the oracle's discretisation and kernel against closed forms and
textbook limits (no GPU)."""
import math

import numpy as np
import pytest
import scipy.integrate

import workloads as W
from oracle import discretise, greens


def test_square_rule_has_24_cells_and_is_symmetric():
    sq = discretise.square_offsets()
    assert sq.shape == (24, 2)
    # closed under x -> -x, y -> -y and x <-> y
    s = {tuple(r) for r in sq}
    for x, y in s:
        assert (-x, y) in s and (x, -y) in s and (y, x) in s
    # the radius^2 classes 0.5, 2.5, 4.5, 6.5 with multiplicities 4, 8, 4, 8
    r2, counts = np.unique(np.sum(sq ** 2, axis=1), return_counts=True)
    assert np.allclose(r2, [0.5, 2.5, 4.5, 6.5])
    assert list(counts) == [4, 8, 4, 8]
    # the next class (1.5, 2.5) -> 8.5 lies outside 24/pi
    assert 6.5 < 24 / math.pi < 8.5


@pytest.mark.parametrize("r,t", [(0.2, 0.1), (0.15, 0.1), (0.25, 0.07)])
def test_cells_are_volume_exact(r, t):
    cells, vol = discretise.particle_cells(r, t)
    assert cells.shape == (48, 3)
    assert math.isclose(48 * vol, math.pi * r * r * t, rel_tol=1e-14)
    # canonical order: lower layer first, b then a ascending within a layer
    assert np.all(cells[:24, 2] < 0) and np.all(cells[24:, 2] > 0)
    lay = cells[:24, :2]
    keys = [(y, x) for x, y in lay]
    assert keys == sorted(keys)
    assert np.allclose(cells.mean(axis=0), 0.0, atol=1e-16)


def test_dyadic_matches_finite_difference_of_scalar_green():
    """G = (I + grad grad / k^2) g, checked with central differences."""
    k = 2 * math.pi
    d0 = np.array([0.31, -0.17, 0.05])
    h = 1e-4
    g = lambda x: greens.scalar_g(np.linalg.norm(x), k)
    hess = np.zeros((3, 3), dtype=complex)
    e = np.eye(3) * h
    for i in range(3):
        for j in range(3):
            hess[i, j] = (g(d0 + e[i] + e[j]) - g(d0 + e[i] - e[j])
                          - g(d0 - e[i] + e[j]) + g(d0 - e[i] - e[j])) / (4 * h * h)
    fd = g(d0) * np.eye(3) + hess / k ** 2
    G = greens.dyadic(d0, k)
    assert np.max(np.abs(G - fd)) / np.max(np.abs(G)) < 1e-6


def test_dyadic_far_field_limit():
    k = 2 * math.pi
    dh = np.array([1.0, 2.0, -0.5]) / np.linalg.norm([1.0, 2.0, -0.5])
    for R in (50.0, 500.0):
        G = greens.dyadic(dh * R, k)
        far = greens.scalar_g(R, k) * (np.eye(3) - np.outer(dh, dh))
        rel = np.max(np.abs(G - far)) / np.max(np.abs(far))
        assert rel < 3.0 / (k * R)


def test_self_term_is_the_pv_integral_plus_depolarisation():
    """k^2 PV-integral of the trace/3 of G over the sphere, by quadrature, minus 1/3."""
    k = 2 * math.pi
    for a in (0.01, 0.04, 0.1):
        # tr G = 2 g; the 1/R^3 parts integrate to zero over directions
        f = lambda R, part: (2.0 / 3.0) * k * k * (R * np.exp(-1j * k * R)).__getattribute__(part)
        re = scipy.integrate.quad(f, 0, a, args=("real",), epsabs=1e-15, epsrel=1e-13)[0]
        im = scipy.integrate.quad(f, 0, a, args=("imag",), epsabs=1e-15, epsrel=1e-13)[0]
        ref = re + 1j * im - 1.0 / 3.0
        assert abs(greens.self_term(a, k) - ref) < 1e-12


def test_self_term_small_ka_series():
    k = 2 * math.pi
    for a in (1e-3, 5e-3, 2e-2):
        ka = k * a
        series = -1 / 3 + ka ** 2 / 3 - 1j * (2 / 9) * ka ** 3
        assert abs(greens.self_term(a, k) - series) < 2 * ka ** 4


def test_single_cell_polarisability_clausius_mossotti_and_radiation_reaction():
    """alpha = V / (1/chi - s(a)) -> 4 pi a^3 (eps-1)/(eps+2), plus j k^3/(6 pi) in 1/alpha."""
    eps = 12 + 0.1j
    chi = eps - 1
    k = 2 * math.pi
    a = 1e-3
    V = 4 * math.pi * a ** 3 / 3
    alpha = V / (1 / chi - greens.self_term(a, k))
    alpha0 = 4 * math.pi * a ** 3 * (eps - 1) / (eps + 2)
    assert abs(alpha / alpha0 - 1) < 1e-4
    corr = 1 / alpha - 1 / alpha0
    # leading terms: -(ka)^2/3 / V (real, dynamic depolarisation) + j k^3 / (6 pi)
    assert abs(corr.imag - k ** 3 / (6 * math.pi)) / (k ** 3 / (6 * math.pi)) < 1e-3


def test_cell_sphere_radius_and_diagonal_entry_closed_form():
    """48 cells of volume pi r^2 t / 48: the equal-volume sphere has radius (r^2 t / 64)^(1/3),
    and each diagonal entry is V (1/chi - s(a)) with that radius (no other term)."""
    r, t, eps = 0.23, 0.1, 12.0 + 0.1j
    arr = W.lattice(1, radius=r, height=t, eps_r=eps)
    d = discretise.Discretisation(arr)
    a = (r * r * t / 64.0) ** (1.0 / 3.0)
    assert abs(d.a_eq[0] - a) <= 1e-15 * a
    Z = greens.assemble_dense(d)
    V = math.pi * r * r * t / 48.0
    want = V * (1.0 / (eps - 1.0) - greens.self_term(a, d.k))
    diag = np.diag(Z)
    assert np.allclose(diag, want, rtol=1e-13, atol=0)
    # the 3 x 3 block of one cell is diagonal
    assert np.all(Z[0:3, 0:3][~np.eye(3, dtype=bool)] == 0)


def test_off_diagonal_imaginary_part_is_the_radiated_power_of_the_cell_dipoles():
    """For any p, Im(p^H Z_off p) + k^3/(6 pi) sum V_m^2 |p_m|^2 is the power radiated by the
    dipoles V_n p_n: k^3/(16 pi^2) times the integral over directions of
    |(I - r^ r^) sum_n V_n p_n exp(-j k r^.r_n)|^2 (exp(+j omega t) convention).  The far
    field is summed here with its own Gauss-Legendre x trapezoid quadrature."""
    arr = W.random_lattice(2, 2, seed=3)
    d = discretise.Discretisation(arr)
    Z = greens.assemble_dense(d)
    pos, vol, _, _ = d.cell_arrays()
    nc, k = pos.shape[0], d.k
    Zoff = Z.copy()
    for m in range(nc):
        Zoff[3 * m:3 * m + 3, 3 * m:3 * m + 3] = 0
    rng = np.random.default_rng(7)
    p = rng.standard_normal(3 * nc) + 1j * rng.standard_normal(3 * nc)
    lhs = np.vdot(p, Zoff @ p).imag + k ** 3 / (6 * math.pi) * np.sum(vol ** 2 * np.sum(np.abs(p.reshape(-1, 3)) ** 2, 1))
    mu, wmu = np.polynomial.legendre.leggauss(48)
    nphi = 96
    phi = np.arange(nphi) * 2 * math.pi / nphi
    st = np.sqrt(1 - mu ** 2)
    rh = np.stack([np.outer(st, np.cos(phi)).ravel(), np.outer(st, np.sin(phi)).ravel(), np.repeat(mu, nphi)], 1)
    w = np.repeat(wmu, nphi) * (2 * math.pi / nphi)
    F = np.exp(-1j * k * rh @ pos.T) @ (vol[:, None] * p.reshape(-1, 3))
    Ft = F - rh * np.sum(rh * F, 1)[:, None]
    rhs = k ** 3 / (16 * math.pi ** 2) * np.sum(w * np.sum(np.abs(Ft) ** 2, 1))
    assert rhs > 0 and abs(lhs - rhs) <= 1e-12 * rhs


def test_matrix_is_complex_symmetric(tiny_oracle):
    Z = tiny_oracle["Z"]
    assert np.max(np.abs(Z - Z.T)) <= 1e-15 * np.max(np.abs(Z))


def test_blocks_are_reciprocal_on_a_random_array():
    arr = W.random_lattice(3, 2, seed=3)
    d = discretise.Discretisation(arr)
    A = greens.assemble_block(d, [0, 4], [1, 5, 2])
    B = greens.assemble_block(d, [1, 5, 2], [0, 4])
    assert np.max(np.abs(A - B.T)) <= 1e-15 * np.max(np.abs(A))


def test_identical_particles_have_identical_self_blocks(tiny_oracle):
    sb = tiny_oracle["self_blocks"]
    for p in range(1, sb.shape[0]):
        assert np.array_equal(sb[0], sb[p])


def test_plane_wave_normal_x_polarised(tiny_oracle):
    d = tiny_oracle["disc"]
    v = tiny_oracle["v"].reshape(-1, 3)
    pos, vol, _, _ = d.cell_arrays()
    # theta = 0: e = x^, phase exp(-j k z)
    assert np.allclose(v[:, 1], 0) and np.allclose(v[:, 2], 0)
    assert np.allclose(v[:, 0], vol * np.exp(-1j * d.k * pos[:, 2]), rtol=1e-15, atol=0)


@pytest.mark.parametrize("theta,phi", [(25.0, 0.0), (-30.0, 40.0), (60.0, 200.0)])
def test_plane_wave_oblique_is_a_transverse_right_handed_wave(tiny_oracle, theta, phi):
    # Reference triad from rotations of the z-directed wave: k^ = Rz(phi) Ry(theta) z^,
    # TM = Rz(phi) Ry(theta) x^ (in the plane of incidence), TE = Rz(phi) y^ (horizontal).
    t, f = math.radians(theta), math.radians(phi)
    Ry = np.array([[math.cos(t), 0, math.sin(t)], [0, 1, 0], [-math.sin(t), 0, math.cos(t)]])
    Rz = np.array([[math.cos(f), -math.sin(f), 0], [math.sin(f), math.cos(f), 0], [0, 0, 1]])
    k_ref, tm_ref, te_ref = Rz @ Ry @ [0, 0, 1], Rz @ Ry @ [1, 0, 0], Rz @ [0, 1, 0]
    assert np.allclose(np.cross(tm_ref, te_ref), k_ref, atol=1e-15)
    d = tiny_oracle["disc"]
    pos, vol, _, _ = d.cell_arrays()
    v = greens.plane_wave_rhs(d, [theta, theta], [phi, phi], [0, 1])
    for col, e_ref in ((0, te_ref), (1, tm_ref)):
        e = v[:, col].reshape(-1, 3) / vol[:, None]
        # every cell carries the same polarisation up to its phase exp(-j k k^.r)
        ph = np.exp(-1j * d.k * (pos @ k_ref))
        assert np.allclose(e, ph[:, None] * e_ref[None, :], rtol=0, atol=1e-14)
        # transverse, unit amplitude
        assert np.allclose(e @ k_ref, 0, atol=1e-14)
        assert np.allclose(np.linalg.norm(e, axis=1), 1.0, rtol=1e-14)


def test_matrix_free_product_equals_dense(tiny_oracle):
    d, Z = tiny_oracle["disc"], tiny_oracle["Z"]
    x = np.random.default_rng(1).standard_normal(Z.shape[0]) + 0j
    assert np.allclose(greens.matvec_free(d, x, chunk=5), Z @ x, rtol=1e-13, atol=0)
    rows = np.array([3, 7])
    y = greens.matvec_free(d, x, rows=rows)
    ref = (Z @ x).reshape(16, 144)[rows].reshape(-1)
    assert np.allclose(y, ref, rtol=1e-13, atol=0)
