"""Pins of the multi-block oracle (the 7-block atlas and its DSS, Sec. 4.3)."""
import numpy as np
import pytest

from oracle.multiblock import MultiBlockMesh
from synthetic_inputs import integer_valued


@pytest.mark.parametrize("k,n", [(1, 1), (1, 2), (2, 2), (3, 2)])
def test_node_count_and_valences(k, n):
    """The glued blocks form the cube-in-cube lattice: (m+1)^3 + m (6 m^2 + 2) nodes
    (m = kn).  Every block face is either glued to exactly one other block face or
    is part of the outer boundary; the blocks meeting at a node number 1 (inside
    a block), 2 (faces, and the outer edges between two caps), 3 (the 12 edges of
    the centre cube, the 8 diagonal lines from its corners outward, and the 8
    outer corners) or 4 (the corners of the centre cube): 8 of those and
    20 (m - 1) + 8 of valence 3, counted from the geometry."""
    M = MultiBlockMesh(k, n)
    m = k * n
    assert M.n_nodes == M.expected_node_count()
    assert set(np.unique(M.node_blocks)) <= {1, 2, 3, 4}
    assert np.sum(M.node_blocks == 4) == 8
    assert np.sum(M.node_blocks == 3) == 20 * (m - 1) + 8
    # copies per node: the blocks' own cell copies add up
    assert M.valence.sum() == M.len
    # inner-cube corner: 1 cell in the centre block + 1 in each of 3 caps
    corner = np.flatnonzero(np.all(np.abs(M.keys) == m * m, axis=1))
    assert len(corner) == 8 and np.all(M.valence[corner] == 4)


@pytest.mark.parametrize("k,n", [(2, 2), (3, 1)])
def test_dss_definitions(k, n):
    M = MultiBlockMesh(k, n)
    v = integer_valued(M.len, seed=5)
    s = M.dss(v)
    # every copy holds the sum of all copies of its node
    for j in np.random.default_rng(0).choice(M.n_nodes, 50, replace=False):
        c = np.flatnonzero(M.copy_node == j)
        assert np.all(s[c] == v[c].sum())
    # the averaging DSS is a projection onto the continuous vectors
    a = M.dss_average(v)
    assert np.allclose(M.dss_average(a), a, rtol=0, atol=1e-12)
    x = M.G @ np.arange(M.n_nodes, dtype=float)
    assert np.array_equal(M.dss_average(x), x)
