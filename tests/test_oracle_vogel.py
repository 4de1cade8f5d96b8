"""Pins of the paper's own test geometry (no GPU): the Vogel spiral of §6.1, the voxelised
sphere that stands in for its meshed meta-atom, and the grouping on the paper's grid
(§5.3: level 1 is 3 x 3 blocks, halving per level; §5.4: a particle belongs to the block
of its centre and the finest level holds at most one particle per block)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import discretise, grouping


@pytest.mark.parametrize("n,radius_um", [(100, 1.73), (500, 3.87), (1000, 5.48), (2000, 7.75)])
def test_vogel_array_radii_match_the_paper(n, radius_um):
    """§6.1 prints the array radii 1.73, 3.87, 5.48 and 7.75 um for R = 100 nm spheres and
    r_i = R sqrt(3) sqrt(i); lengths here are in 600 nm wavelengths."""
    c = W.vogel(n).centers
    assert abs(np.max(np.hypot(c[:, 0], c[:, 1])) * 0.6 - radius_um) < 0.005


def test_vogel_angles_step_by_the_golden_angle():
    """Successive centres turn by 2 pi / phi^2 (about 137.5 degrees) and r_i^2 grows by c^2."""
    c = W.vogel(50).centers
    ang = np.unwrap(np.arctan2(c[:, 1], c[:, 0]))
    step = np.diff(ang) % (2 * math.pi)
    assert np.allclose(step, math.radians(137.50776405003785), atol=1e-12)
    r2 = c[:, 0] ** 2 + c[:, 1] ** 2
    assert np.allclose(np.diff(r2), 3.0 * W.VOGEL_SPHERE_RADIUS ** 2, rtol=1e-12)


def test_spheres_do_not_overlap():
    c = W.vogel(500).centers[:, :2]
    d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)) + np.eye(len(c)) * 1e9
    assert d.min() > 2 * W.VOGEL_SPHERE_RADIUS


def test_sphere_cells_fill_the_sphere_volume_without_overlap():
    R = 0.3
    cells, vol = discretise.sphere_cells(R)
    h = vol ** (1.0 / 3.0)
    assert cells.shape == (48, 3)
    assert abs(48 * vol - 4.0 / 3.0 * math.pi * R ** 3) <= 1e-15
    # distinct cubes on one h-grid: centres differ by at least h in some coordinate
    g = cells / h + 1.5
    assert np.allclose(g, np.round(g), atol=1e-12)
    assert len({tuple(np.round(x).astype(int)) for x in g}) == 48
    # four layers of 12, mirror symmetric in x, y and z, centroid at the centre
    assert sorted(np.unique(np.round(g[:, 2]).astype(int), return_counts=True)[1]) == [12] * 4
    key = {tuple(np.round(x, 9)) for x in cells}
    for axis in range(3):
        m = cells.copy()
        m[:, axis] *= -1
        assert {tuple(np.round(x, 9)) for x in m} == key
    assert np.allclose(cells.mean(axis=0), 0.0, atol=1e-15)
    # the corners of each layer are the cubes left out: no centre at |x| = |y| = 3h/2
    assert not np.any((np.abs(np.abs(g[:, 0] - 1.5) - 1.5) < 1e-9) & (np.abs(np.abs(g[:, 1] - 1.5) - 1.5) < 1e-9))


def test_discretisation_uses_sphere_cells_for_sphere_arrays():
    arr = W.vogel(7)
    d = discretise.Discretisation(arr)
    ref, vol = discretise.sphere_cells(W.VOGEL_SPHERE_RADIUS)
    assert np.allclose(d.pos[3] - arr.centers[3][None, :], ref, atol=1e-15)
    assert np.all(d.vol == vol)


def test_paper_grid_by_hand():
    """Three centres on a line x = 0, 1, 2: the root square of side 2 (1 + 2^-20) centred on
    (1, 0) puts them in level-1 blocks (0, 1), (1, 1), (2, 1): one level, and every ordered
    pair compressed there (finest level)."""
    c = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    L, ij, origin, side = grouping.paper_grid(c)
    assert L == 1 and ij.tolist() == [[0, 1], [1, 1], [2, 1]]
    assert side == 2.0 * (1 + 2.0 ** -20)
    blocks, L2 = grouping.build_blocks_paper(c)
    assert L2 == 1 and len(blocks) == 6 and all(b.level == 1 for b in blocks)


def test_paper_grid_two_levels_by_hand():
    """Centres (0, 0), (0.2, 0) and (3, 3): the root square has side 3 (1 + 2^-20).  The
    first two centres share a block at levels 1, 2 and 3 (block sides about 1, 0.5, 0.25 >
    0.2) and separate at level 4 (side 0.125: blocks (0, 0) and (1, 0)); the third lies in
    block (23, 23).  The pair {0, 1} x {2} is far already at level 1 (blocks (0, 0) and
    (2, 2)); the pair 0-1 is compressed at the finest level."""
    c = np.array([[0.0, 0, 0], [0.2, 0, 0], [3.0, 3.0, 0]])
    L, ij, origin, side = grouping.paper_grid(c)
    assert L == 4
    assert ij[0].tolist() == [0, 0] and ij[1].tolist() == [1, 0] and ij[2].tolist() == [23, 23]
    blocks, _ = grouping.build_blocks_paper(c)
    # the far pair of particles 0/1 and 2 is compressed on level 1 (blocks (0, 0) and (2, 2)),
    # the pair 0-1 at the finest level
    lv = {(b.rows, b.cols): b.level for b in blocks}
    assert lv[((0, 1), (2,))] == 1 and lv[((2,), (0, 1))] == 1
    assert lv[((0,), (1,))] == 4 and lv[((1,), (0,))] == 4
    assert len(blocks) == 4


@pytest.mark.parametrize("n", [100, 500])
def test_paper_grid_places_each_centre_in_its_block_at_the_minimal_level(n):
    c = W.vogel(n).centers
    L, ij, origin, side = grouping.paper_grid(c)
    nb = 3 * 2 ** (L - 1)
    h = side / nb
    assert ij.min() >= 0 and ij.max() < nb
    for p in range(n):
        for a in range(2):
            lo = origin[a] + ij[p, a] * h
            assert lo - 1e-12 <= c[p, a] < lo + h + 1e-12
    assert np.all(ij >> (L - 1) < 3)                                   # level 1 is 3 x 3
    # one level coarser, some block holds two particles
    coarse = {(int(i) >> 1, int(j) >> 1) for i, j in ij}
    assert len(coarse) < n


@pytest.mark.parametrize("n", [100, 500])
def test_paper_grid_covers_every_distinct_pair_once_with_far_blocks(n):
    c = W.vogel(n).centers
    blocks, L = grouping.build_blocks_paper(c)
    cover = grouping.coverage_matrix(blocks, n)
    assert np.array_equal(cover, 1 - np.eye(n, dtype=np.int64))
    for b in blocks:
        cheb = grouping.chebyshev(b.row_node, b.col_node)
        assert cheb >= 2 or (b.level == L and cheb >= 1)
        if b.level > 1:
            pa = (b.row_node[0] >> 1, b.row_node[1] >> 1)
            pb = (b.col_node[0] >> 1, b.col_node[1] >> 1)
            assert grouping.chebyshev(pa, pb) <= 1
    # level 1 does compress far pairs of the 3 x 3 grid
    assert any(b.level == 1 for b in blocks)
