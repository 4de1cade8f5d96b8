"""Recursive near/far grouping of a lattice array (oracle, pure Python).

Follows §5.1 (definition: two grid blocks are near when they share at least
one grid node, i.e. their integer cell coordinates differ by at most one in
each direction), §5.3 (eq. 5.4: a multilevel grid that halves the blocks in x
and y at each level; each level compresses the far interactions not yet
accounted for and passes the near ones to the next level) and §5.4 (each
particle belongs, whole, to the block containing its centre; at the finest
level a block holds at most one particle and every interaction between
distinct particles is compressed, so the near part left is the particle
block diagonal Z_D).

Grid reading for lattice arrays: a quadtree aligned to the lattice, padded to
2^L sites per side with L = ceil(log2(max(nx, ny))); level l has 2^l x 2^l
blocks, each covering 2^(L-l) lattice sites per side.  The pairs compressed at
level l are the ordered pairs (I, J) of occupied level-l blocks whose parents
are near and which are far (Chebyshev distance >= 2), plus, at the finest level
l = L, the near pairs I != J.

Grid reading for arrays without a lattice (the paper's Vogel spirals, §6.1),
``paper_grid`` / ``build_blocks_paper``: the paper's own grid, whose first level is
3 x 3 blocks and which halves the blocks at every further level, laid over the
bounding square of the particle centres (centred on the bounding box, side
(1 + 2^-20) times the larger extent so the outermost centres fall inside).  Level l
has 3 * 2^(l-1) blocks per side; a particle belongs to the block containing its
centre (§5.4); the finest level L is the first at which no block holds two particles
(§5.4: at most one meta-atom per block).  Level-1 blocks all share the root as parent,
so every far pair of level-1 blocks is compressed at level 1.

Pins (tests): every ordered pair of distinct particles is covered by exactly
one block (brute force); compressed pairs are far (or finest-level distinct);
the 4 x 4 array gives 16 * 15 = 240 single-particle blocks; on the paper grid each
particle's centre lies inside its block, level 1 is 3 x 3 and L is minimal.
"""
from __future__ import annotations

import math
from collections import defaultdict
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Block:
    level: int
    row_node: tuple[int, int]
    col_node: tuple[int, int]
    rows: tuple[int, ...]     # caller particle indices (ascending)
    cols: tuple[int, ...]


def n_levels(nx: int, ny: int) -> int:
    m = max(nx, ny)
    return 0 if m <= 1 else int(math.ceil(math.log2(m)))


def chebyshev(a, b) -> int:
    return max(abs(a[0] - b[0]), abs(a[1] - b[1]))


def node_members(lattice_ij: np.ndarray, L: int, level: int) -> dict:
    """Occupied level-`level` blocks -> sorted particle list."""
    shift = L - level
    members = defaultdict(list)
    for p, (i, j) in enumerate(np.asarray(lattice_ij)):
        members[(int(i) >> shift, int(j) >> shift)].append(p)
    return {k: tuple(v) for k, v in members.items()}


def build_blocks(lattice_ij: np.ndarray, nx: int, ny: int) -> list[Block]:
    L = n_levels(nx, ny)
    blocks = []
    for level in range(1, L + 1):
        nodes = node_members(lattice_ij, L, level)
        keys = sorted(nodes)
        for I in keys:
            pI = (I[0] >> 1, I[1] >> 1)
            for J in keys:
                if I == J:
                    continue
                pJ = (J[0] >> 1, J[1] >> 1)
                if chebyshev(pI, pJ) > 1:
                    continue              # accounted for at a coarser level
                if chebyshev(I, J) >= 2 or level == L:
                    blocks.append(Block(level, I, J, nodes[I], nodes[J]))
    return blocks


def level_counts(blocks: list[Block]) -> dict:
    out = defaultdict(int)
    for b in blocks:
        out[b.level] += 1
    return dict(out)


def coverage_matrix(blocks: list[Block], n: int) -> np.ndarray:
    """cover[p, q] = number of blocks containing the particle pair (p, q)."""
    cover = np.zeros((n, n), dtype=np.int64)
    for b in blocks:
        for p in b.rows:
            for q in b.cols:
                cover[p, q] += 1
    return cover


def paper_grid(centers: np.ndarray, max_level: int = 20):
    """(L, ij, origin, side): the finest level, each particle's block there (N, 2), and the
    root square (lower-left corner, side) of the paper's grid over the centres."""
    xy = np.asarray(centers, dtype=np.float64)[:, :2]
    lo, hi = xy.min(axis=0), xy.max(axis=0)
    side = float(max(hi[0] - lo[0], hi[1] - lo[1]))
    if not side > 0.0:
        side = 1.0
    side *= 1.0 + 2.0 ** -20
    origin = (0.5 * (lo[0] + hi[0]) - 0.5 * side, 0.5 * (lo[1] + hi[1]) - 0.5 * side)
    for L in range(1, max_level + 1):
        nb = 3 * 2 ** (L - 1)
        h = side / nb
        ij = np.empty((len(xy), 2), dtype=np.int64)
        for p, (x, y) in enumerate(xy):
            ij[p, 0] = min(nb - 1, int(math.floor((x - origin[0]) / h)))
            ij[p, 1] = min(nb - 1, int(math.floor((y - origin[1]) / h)))
        if len({(int(a), int(b)) for a, b in ij}) == len(xy):
            return L, ij, origin, side
    raise ValueError("two centres share a block at the deepest level")


def build_blocks_paper(centers: np.ndarray) -> tuple[list[Block], int]:
    """Blocks of the paper-grid grouping, and its number of levels."""
    L, ij, _, _ = paper_grid(centers)
    blocks = []
    for level in range(1, L + 1):
        nodes = node_members(ij, L, level)
        keys = sorted(nodes)
        for I in keys:
            for J in keys:
                if I == J:
                    continue
                if level > 1 and chebyshev((I[0] >> 1, I[1] >> 1), (J[0] >> 1, J[1] >> 1)) > 1:
                    continue              # parents far: compressed at a coarser level
                if chebyshev(I, J) >= 2 or level == L:
                    blocks.append(Block(level, I, J, nodes[I], nodes[J]))
    return blocks, L
