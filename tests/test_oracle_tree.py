"""Pins of the oracle's tree rule and zone geometry (Sec. 1 and Fig. 1)."""
import numpy as np
import pytest

from oracle.tree import OutOfBox, Tree, cell_index, morton_key
from synth import plummer_sphere


def test_morton_key_bit_order():
    assert morton_key(1, 0, 0, 3) == 1
    assert morton_key(0, 1, 0, 3) == 2
    assert morton_key(0, 0, 1, 3) == 4
    assert morton_key(2, 0, 0, 3) == 8
    # brute-force interleave
    for (x, y, z) in [(3, 5, 6), (7, 0, 1), (5, 5, 5)]:
        want = 0
        for b in range(3):
            want |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
        assert morton_key(x, y, z, 3) == want


def test_cell_index_half_open_and_clamped():
    pos = np.array([[0.0, 0.5, 1.0], [0.2499999, 0.25, 0.75]])
    ijk = cell_index(pos, (0, 0, 0), 1.0, 2)
    assert ijk.tolist() == [[0, 2, 3], [0, 1, 3]]
    with pytest.raises(OutOfBox):
        cell_index(np.array([[0.5, -1e-12, 0.5]]), (0, 0, 0), 1.0, 2)
    with pytest.raises(OutOfBox):
        cell_index(np.array([[0.5, np.nan, 0.5]]), (0, 0, 0), 1.0, 2)


def test_tiny_adaptive_tree_by_hand():
    # 5 particles, capacity 2, depth 3. Level 1: octant 0 holds 3 particles (split), octant 7
    # holds 2 (leaf). Level 2 inside octant 0: cube (0,0,0) holds 2 (leaf), cube (1,1,1) holds 1.
    pos = np.array([[0.10, 0.10, 0.10],   # level-2 cube (0,0,0)
                    [0.90, 0.90, 0.90],   # octant 7
                    [0.30, 0.30, 0.30],   # level-2 cube (1,1,1)
                    [0.20, 0.05, 0.15],   # level-2 cube (0,0,0)
                    [0.60, 0.70, 0.80]])  # octant 7
    t = Tree(pos, leaf_capacity=2, max_depth=3)
    assert t.perm.tolist() == [0, 3, 2, 4, 1]
    assert [len(l) for l in t.levels] == [1, 2, 2]
    l1, l2 = t.levels[1], t.levels[2]
    assert l1.coords.tolist() == [[0, 0, 0], [1, 1, 1]]
    assert list(zip(l1.pb, l1.pe)) == [(0, 3), (3, 5)]
    assert l1.split.tolist() == [True, False]
    assert l2.coords.tolist() == [[0, 0, 0], [1, 1, 1]]
    assert list(zip(l2.pb, l2.pe)) == [(0, 2), (2, 3)]
    assert l2.split.tolist() == [False, False]
    assert t.levels[0].children[0].tolist() == [0, -1, -1, -1, -1, -1, -1, 1]
    assert l2.parent.tolist() == [0, 0]


def test_uniform_tree_counts():
    rng = np.random.default_rng(0)
    t = Tree(rng.random((4096, 3)), uniform_depth=3)
    assert [len(l) for l in t.levels] == [1, 8, 64, len(t.levels[3])]
    assert not t.levels[3].split.any() and t.levels[2].split.all()


def test_zone_sizes_match_the_paper():
    # Sec. 1: 26 neighbours plus the cell itself; 6^3 - 3^3 = 189 interaction-zone cells.
    assert len(Tree.near_positions((5, 5, 5), 4)) == 27
    assert len(Tree.interaction_positions((5, 5, 5), 4)) == 189
    assert len(Tree.interaction_positions((4, 5, 6), 4)) == 189
    # clipped at the box: a corner cell at level 2 sees 4^3 - 2^3 = 56 cubes
    assert len(Tree.interaction_positions((0, 0, 0), 2)) == 64 - 8


@pytest.mark.parametrize("cap", [4, 16])
def test_zones_partition_every_particle_exactly_once(cap):
    # Cube-complete reading: near zone of the leaf plus the interaction zones of the leaf and
    # all its ancestors down to level 2 cover every particle once.
    p = plummer_sphere(1500, 5, a=0.1)
    t = Tree(p.positions(), leaf_capacity=cap, max_depth=6)
    rng = np.random.default_rng(1)
    leaves = list(t.leaves())
    for li in rng.choice(len(leaves), size=12, replace=False):
        l, i = leaves[li]
        count = np.zeros(t.n, dtype=np.int64)
        coord = t.levels[l].coords[i]
        for q in t.near_positions(coord, l):
            b, e = t.cube_range(l, q)
            count[b:e] += 1
        c, lev = coord.copy(), l
        while lev >= 2:
            for q in t.interaction_positions(c, lev):
                b, e = t.cube_range(lev, q)
                count[b:e] += 1
            c, lev = c >> 1, lev - 1
        assert np.all(count == 1), (l, i)
