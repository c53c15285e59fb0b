"""Oracle stencils (Sec. 2.1: each node's N_L nearest nodes, minimum image in
the unit periodic cell) pinned to an independent k-d tree, to hand-derived
tie orders on a lattice, and to the host fixture's stencils."""
import itertools

import numpy as np
import pytest
from scipy.spatial import cKDTree

import nodecloud as nc
import oracle as O


def test_knn_matches_periodic_kdtree():
    """Random points (no ties): scipy's periodic k-d tree gives the same
    neighbours in the same order, including across the cell faces."""
    rng = np.random.default_rng(1)
    pts = rng.random((3000, 3))
    q = np.r_[rng.random((400, 3)), [[0.001, 0.999, 0.0005], [0.5, 0.0, 1.0 - 1e-9]]]
    got = O.knn(pts, 30, q)
    d, ref = cKDTree(pts, boxsize=1.0).query(q % 1.0, k=30)
    assert np.array_equal(got, ref)
    assert np.array_equal(O.knn(pts, 30)[:, 0], np.arange(3000))  # each point is its own nearest


def test_knn_tie_order_on_a_lattice():
    """On an n^3 lattice with spacing 1/8 (exact in binary, so equal distances
    are equal to the last bit) every node has 6 neighbours at 1/8, 12 at
    sqrt(2)/8 and 8 at sqrt(3)/8.  With node (a, b, c) at index
    (a n + b) n + c the expected columns are those shells, each in ascending
    index order, after the node itself."""
    n = 8
    lat = np.array(list(itertools.product(range(n), repeat=3)))
    pts = lat / n
    S = O.knn(pts, 27)
    for i in (0, 7, 100, 300, n ** 3 - 1):
        a = lat[i]
        shells = {1: [], 2: [], 3: []}
        for off in itertools.product((-1, 0, 1), repeat=3):
            s = sum(abs(o) for o in off)
            if s:
                b = (a + np.array(off)) % n
                shells[s].append(int((b[0] * n + b[1]) * n + b[2]))
        expect = [i] + sorted(shells[1]) + sorted(shells[2]) + sorted(shells[3])
        assert S[i].tolist() == expect


def test_solver_stencils_match_host_fixture(small_cloud):
    """Interior rows: the nl nearest nodes; surface rows: the node, then its
    nl - 1 nearest interior nodes.  The host fixture takes its candidates from
    scipy's k-d tree and orders exact ties by index too, so the two agree
    element for element; this cloud has 16 rows with exactly tied neighbours
    (the advancing front places many pairs at exactly h), where the tree's own
    order differs."""
    c = small_cloud
    got = O.solver_stencils(c.pos, c.n_int, 30)
    assert np.array_equal(got, nc.solver_stencils(c, 30))
    _, raw = cKDTree(c.pos, boxsize=1.0).query(c.pos[:c.n_int], k=30)
    differs = (raw != got[:c.n_int]).any(1)
    assert differs.sum() > 0
    assert all(set(raw[i]) == set(got[i]) for i in np.where(differs)[0])


def test_knn_argument_errors():
    with pytest.raises(ValueError):
        O.knn(np.zeros((4, 3)), 5)
    with pytest.raises(ValueError):
        O.knn(np.zeros((4, 3)), 0)


@pytest.mark.parametrize("k", [7, 10, 19, 27])
def test_host_fixture_tie_order_on_a_lattice(k):
    """The host fixture asks the tree for a few extra candidates and widens
    where a tie reaches past them (k = 10 cuts the 12 face diagonals)."""
    n = 8
    pts = np.array(list(itertools.product(range(n), repeat=3))) / n
    assert np.array_equal(nc.stencils(pts, k), O.knn(pts, k))


def test_tile_plan_definition_by_brute_force():
    """The oracle's tile plan against a pure-Python construction (set, sort,
    list.index) on a small cloud with a ragged last tile: every halo is the
    sorted set of its tile's stencil entries and every entry maps back."""
    c = nc.sphere_cloud(0.3, 0.05, 0.3, 0.1, seed=1)
    S = nc.solver_stencils(c, 20)[:300]  # 4 full tiles and a ragged one of 44
    halos, lidx = O.tile_plan(S, 64)
    assert len(halos) == 5
    for t, h in enumerate(halos):
        rows = S[64 * t:64 * t + 64]
        ref = sorted(set(int(x) for x in rows.ravel()))
        assert list(h) == ref
        for i in range(len(rows)):
            for j in range(S.shape[1]):
                assert ref.index(int(rows[i, j])) == lidx[64 * t + i, j]
