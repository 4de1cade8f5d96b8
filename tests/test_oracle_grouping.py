"""Pins of the recursive near/far grouping (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import grouping


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (2, 2), (3, 3), (4, 4), (5, 7), (8, 8), (6, 3), (9, 9)])
def test_every_distinct_pair_is_covered_exactly_once(nx, ny):
    arr = W.lattice(nx, ny)
    blocks = grouping.build_blocks(arr.lattice_ij, nx, ny)
    cover = grouping.coverage_matrix(blocks, arr.n_particles)
    expect = np.ones((arr.n_particles,) * 2, dtype=np.int64) - np.eye(arr.n_particles, dtype=np.int64)
    assert np.array_equal(cover, expect)


@pytest.mark.parametrize("nx,ny", [(5, 7), (8, 8), (16, 16)])
def test_compressed_pairs_are_far_or_finest_level(nx, ny):
    arr = W.lattice(nx, ny)
    L = grouping.n_levels(nx, ny)
    for b in grouping.build_blocks(arr.lattice_ij, nx, ny):
        cheb = grouping.chebyshev(b.row_node, b.col_node)
        assert cheb >= 2 or (b.level == L and cheb == 1)
        pa = (b.row_node[0] >> 1, b.row_node[1] >> 1)
        pb = (b.col_node[0] >> 1, b.col_node[1] >> 1)
        assert grouping.chebyshev(pa, pb) <= 1


def test_tiny_array_has_240_single_particle_blocks():
    arr = W.tiny()
    blocks = grouping.build_blocks(arr.lattice_ij, 4, 4)
    assert len(blocks) == 16 * 15
    assert all(len(b.rows) == 1 and len(b.cols) == 1 and b.level == 2 for b in blocks)


def test_first_compressing_level_count_by_hand():
    """Level 2 of a 4x4-block grid: all 16*15 ordered pairs minus the 84 near ones."""
    arr = W.lattice(32)
    blocks = grouping.build_blocks(arr.lattice_ij, 32, 32)
    counts = grouping.level_counts(blocks)
    near = 4 * 3 + 8 * 5 + 4 * 8   # corners, edges, interior neighbours in a 4x4 grid
    assert counts[2] == 16 * 15 - near == 156
    assert sum(counts.values()) == 39732
    assert counts == {2: 156, 3: 1116, 4: 5628, 5: 32832}
