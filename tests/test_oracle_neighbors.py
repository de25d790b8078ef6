"""Pins of the oracle's neighbour search and cell binning (Sec. 4.1, Alg. 1).

The definition is the all-pairs set {j : |x_i - x_j| < 2h}; it is checked
against scipy's k-d tree (a different algorithm), and the cell-list search is
checked against the brute force. Hash/sort/cellStart are checked against
geometric properties of the grid.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2507_05643_amd import scenes


def _positions(sc):
    parts = [sc.pos.astype(np.float64)]
    for b in sc.bodies:
        q = np.asarray(b.quat)
        assert np.allclose(q, [1, 0, 0, 0])
        parts.append(np.asarray(b.pos, dtype=np.float64) + b.markers.astype(np.float64))
    return np.concatenate(parts)


def test_bruteforce_equals_kdtree(orc):
    sc = scenes.column(seed=3, n=8)
    x = _positions(sc)
    xf = x.astype(np.float32).astype(np.float64)
    off, nbr = orc.neighbors(sc.params, x, mode="brute")
    R = 2 * sc.params["h"]
    tree = cKDTree(xf)
    ref = tree.query_ball_point(xf, R)
    for i in range(x.shape[0]):
        mine = set(nbr[off[i]:off[i + 1]].tolist())
        theirs = set(ref[i])
        diff = mine ^ theirs
        for j in diff:  # only pairs at the boundary (|d| == 2h up to rounding) may differ
            d = np.linalg.norm(xf[i] - xf[j])
            assert abs(d - R) < 1e-12
        assert i in mine  # the self pair is in the list


def test_cells_equal_bruteforce(orc):
    for seed in (0, 1):
        sc = scenes.plate_patch(seed=seed, nx=10, ny=9, nz=6)
        x = _positions(sc)
        o1, n1 = orc.neighbors(sc.params, x, mode="brute")
        o2, n2 = orc.neighbors(sc.params, x, mode="cells")
        assert np.array_equal(o1, o2)
        assert np.array_equal(n1, n2)


def test_cells_equal_bruteforce_subset(orc):
    sc = scenes.column(seed=5, n=9)
    x = _positions(sc)
    ids = np.sort(np.random.default_rng(0).choice(x.shape[0], 900, replace=False)).astype(np.int32)
    o1, n1 = orc.neighbors(sc.params, x, ids=ids, mode="brute")
    o2, n2 = orc.neighbors(sc.params, x, ids=ids, mode="cells")
    assert np.array_equal(o1, o2) and np.array_equal(n1, n2)
    assert set(n1.tolist()) <= set(ids.tolist())


def test_interior_lattice_has_57_neighbours(orc):
    sc = scenes.column(seed=0, n=9, jitter=0.0, walls=False)
    x = _positions(sc)
    off, nbr = orc.neighbors(sc.params, x, mode="cells")
    cnt = np.diff(off)
    c = np.array([4, 4, 4])
    i = int(c[0] + 9 * c[1] + 81 * c[2])
    assert cnt[i] == 57


def test_hash_sort_cellstart_properties(orc):
    sc = scenes.plate_patch(seed=2, nx=12, ny=10, nz=7)
    p = sc.params
    x = _positions(sc)
    xf = x.astype(np.float32).astype(np.float64)
    sid, skey, cs, ce = orc.sort_cells(p, x)
    dims, inv = orc.grid_dims(p)
    n = x.shape[0]
    # a permutation, ordered by (cell, id)
    assert np.array_equal(np.sort(sid), np.arange(n))
    assert np.all(np.diff(skey) >= 0)
    same = np.diff(skey) == 0
    assert np.all(np.diff(sid)[same] > 0)
    # each particle's cell box contains it: c = z*(Y*X) + y*X + x, cell size 2h
    cz = skey // (dims[0] * dims[1])
    cy = (skey // dims[0]) % dims[1]
    cx = skey % dims[0]
    lo = np.asarray(p["domain_lo"])
    size = 2 * p["h"]
    for ax, cc in enumerate((cx, cy, cz)):
        v = xf[sid, ax]
        assert np.all(v >= lo[ax] + cc * size - 1e-12)
        assert np.all(v < lo[ax] + (cc + 1) * size + 1e-12)
    # cellStart / cellEnd cover exactly the particles of each cell
    M = int(np.prod(dims))
    assert cs.size == M
    assert np.all(ce >= cs)
    assert int(np.sum(ce - cs)) == n
    for c in np.unique(skey):
        assert np.all(skey[cs[c]:ce[c]] == c)
    empty = ce == cs
    assert np.all(cs[1:][empty[1:]] >= ce[:-1][empty[1:]])


def test_persistent_list_schedule(orc):
    """Lists are rebuilt only when step mod ps_freq == 0, from start-of-step
    positions, and reused otherwise (Alg. 2)."""
    from oracle.oracle import Oracle
    for ps in (1, 10):
        sc = scenes.cluster(seed=4, n=5, vel_scale=2.0, sigma_scale=0.0)
        sc.params["ps_freq"] = ps
        o = Oracle(sc, nbr_mode="cells")
        x0 = o.state()["pos"].copy()
        o.step(4)
        x4 = o.state()["pos"].copy()
        o.step(1)
        proc, off, nbr = o.lists()
        ref_off, ref_nbr = orc.neighbors(sc.params, x4 if ps == 1 else x0, mode="brute")
        assert np.array_equal(off, ref_off) and np.array_equal(nbr, ref_nbr)
