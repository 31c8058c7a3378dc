"""Pins for the oracle's interpolation points and Lagrange weights
(Section 2.1: Chebyshev/Mock-Chebyshev grids, eqs. (eqn:gdA)/(eqn:gdB);
Lagrange polynomials M_t)."""

import numpy as np
import pytest

from oracle.butterfly import (mock_chebyshev, mock_chebyshev_as_printed,
                              lagrange_1d, Trees)


def test_printed_grid_formula_collapses():
    # Taken literally, eq. (eqn:gdA) pairs +t with a descending node: for a
    # box of 16 and r = 8 only four distinct indices survive.  This is why
    # the ascending-node reading is used.
    assert list(mock_chebyshev_as_printed(16, 8)) == [7, 8, 9, 10]


def test_hand_computed_examples():
    # x_t = Round(t + (N_A - r) s_t), s_t = (1 - cos((t-1) pi/(r-1)))/2.
    # (16, 8): s = 0, .0495, .1883, .3887, .6113, .8117, .9505, 1
    #   -> 1, 2.40, 4.51, 7.11, 9.89, 12.49, 14.60, 16 -> rounded:
    assert list(mock_chebyshev(16, 8) + 1) == [1, 2, 5, 7, 10, 12, 15, 16]
    # (1024, 8): t = 2 gives 2 + 1016 * 0.049516 = 52.31 -> 52, etc.
    assert list(mock_chebyshev(1024, 8) + 1) == [1, 52, 194, 399, 626, 831,
                                                 973, 1024]
    # exact ties (s = 1/4, 1/2, 3/4 times an even-odd length) round up:
    # (16, 10), t = 4: 4 + 6 * 1/4 = 5.5 -> 6
    assert (mock_chebyshev(16, 10) + 1)[3] == 6
    # (32, 10), t = 7: 7 + 22 * 3/4 = 23.5 -> 24
    assert (mock_chebyshev(32, 10) + 1)[6] == 24
    # odd r: the middle node s = 1/2 exactly; (8, 7), t = 4: 4 + 1/2 -> 5
    assert list(mock_chebyshev(8, 7) + 1) == [1, 2, 3, 5, 6, 7, 8]


@pytest.mark.parametrize("r", range(2, 17))
def test_points_distinct_and_span_box(r):
    for L in range(0, 21):
        size = 1 << L
        p = mock_chebyshev(size, r)
        assert p.size == min(size, r)
        assert p[0] == 0 and p[-1] == size - 1
        assert np.all(np.diff(p) >= 1)


@pytest.mark.parametrize("r", range(2, 17))
def test_points_follow_chebyshev_density(r):
    # the points differ from (size-1) s_t by less than r (the +t offset);
    # so for large boxes they cluster at the ends like Chebyshev nodes.
    size = 1 << 16
    p = mock_chebyshev(size, r).astype(float)
    t = np.arange(r)
    s = (1 - np.cos(t * np.pi / (r - 1))) / 2
    assert np.max(np.abs(p - (size - 1) * s)) <= r


@pytest.mark.parametrize("nodes", [[0, 1], [0, 3, 7], [0, 2, 5, 9, 15],
                                   list(mock_chebyshev(64, 10)),
                                   list(mock_chebyshev(16, 8))])
def test_lagrange_identity_partition_and_polynomials(nodes):
    nodes = np.asarray(nodes, float)
    r = nodes.size
    # identity at the nodes
    assert np.allclose(lagrange_1d(nodes, nodes), np.eye(r), atol=1e-13)
    y = np.linspace(nodes[0], nodes[-1], 37)
    M = lagrange_1d(nodes, y)
    # partition of unity
    assert np.allclose(M.sum(axis=1), 1.0, atol=1e-11)
    # exact on polynomials of degree < r (scaled to the box to stay O(1))
    u = (nodes - nodes[0]) / max(1.0, nodes[-1] - nodes[0])
    uy = (y - nodes[0]) / max(1.0, nodes[-1] - nodes[0])
    for deg in range(r):
        assert np.allclose(M @ (u ** deg), uy ** deg, atol=1e-10)


def test_lagrange_single_point_is_one():
    assert lagrange_1d([5.0], [5.0, 9.0]).tolist() == [[1.0], [1.0]]


def test_tree_geometry_2d():
    T = Trees(2, 16, 3)
    # level-2 boxes have side 4; 3 points per dimension -> 9 tensor points
    pts = T.points(2)
    assert pts.shape == (16, 9, 2)
    # box (1, 2) starts at (4, 8); its points are offsets {0, 2, 3}^2 (side 4,
    # r = 3: 1 + 1*0, 2 + 1*0.5 -> 3 (tie up), 3 + 1 -> 4; 1-based)
    b = T.flat(2, np.array([1, 2]))
    off = mock_chebyshev(4, 3)
    assert list(off) == [0, 2, 3]
    expect = np.array([[4 + i, 8 + j] for i in off for j in off])
    assert np.array_equal(pts[b], expect)
    # centers: lower middle
    assert list(T.centers(2)[b]) == [4 + 1, 8 + 1]
    # tensor Lagrange = product of 1D weights
    rel = np.array([[1, 3], [2, 0]])
    M = T.lagrange(2, rel)
    L1 = lagrange_1d(off, [1, 2])  # first coords
    L2 = lagrange_1d(off, [3, 0])
    for t, (i, j) in enumerate([(i, j) for i in range(3) for j in range(3)]):
        assert np.isclose(M[t, 0], L1[0, i] * L2[0, j])
        assert np.isclose(M[t, 1], L1[1, i] * L2[1, j])
