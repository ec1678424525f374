"""Pins of the oracle's Hilbert keys and of the tree built on them.

Hilbert order only changes the order in which the boxes of Sec. 3's
octasection are visited: the boxes, and every per-particle interaction list,
stay those of the Morton tree.  The pins take the curve's defining
properties on small grids (a bijection onto 0 .. 8^b - 1 that starts at the
origin, consecutive indices face-adjacent, every box at every level one
contiguous run of indices), and for the tree: the same set of boxes as the
Morton tree, the same per-particle (G = 1) interaction counts and forces, and
the direct sum at theta = 0.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_0709_3331_amd import inputs

H, M = oracle.CURVE_HILBERT, oracle.CURVE_MORTON


def grid_keys(bits, b=10):
    """Keys of every cell centre of a 2^bits grid, at key depth b: the grid
    cells are the level-`bits` boxes of the unit cube."""
    side = 1 << bits
    ijk = np.array(list(itertools.product(range(side), repeat=3)), dtype=np.int64)
    x = (ijk + 0.5) / side
    lo, e = np.zeros(3), 0                   # the cube [0, 1)^3
    k = oracle.keys(x, lo, e, b, curve=H) >> np.uint64(3 * (b - bits))
    return ijk, k.astype(np.int64)


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_bijection_from_the_origin(bits):
    ijk, k = grid_keys(bits)
    assert sorted(k.tolist()) == list(range(8 ** bits))
    assert k[np.all(ijk == 0, axis=1)][0] == 0


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_consecutive_cells_are_face_adjacent(bits):
    ijk, k = grid_keys(bits)
    path = ijk[np.argsort(k)]
    step = np.abs(np.diff(path, axis=0))
    assert np.all(step.sum(axis=1) == 1), "every step moves one cell along one axis"


@pytest.mark.parametrize("bits", [2, 3, 4])
def test_every_box_is_one_run_of_indices(bits):
    ijk, k = grid_keys(bits)
    for lvl in range(1, bits):
        shift = bits - lvl
        box = ijk >> shift
        pref = k >> (3 * shift)
        # one prefix per box and one box per prefix
        pairs = {(tuple(bx), int(p)) for bx, p in zip(box, pref)}
        assert len(pairs) == 8 ** lvl


def test_full_depth_keys_of_the_metric_cloud_are_a_permutation_of_cells():
    # at b = 21 the same property, sampled: particles in one level-6 box share
    # the top 18 bits of their key, and different boxes have different prefixes
    cl, _ = inputs.metric(0)
    lo, e = oracle.cube(cl.x)
    kh = oracle.keys(cl.x, lo, e, 21, curve=H)
    km = oracle.keys(cl.x, lo, e, 21, curve=M)
    # the level-6 box of each particle, from its Morton key
    box_m = km >> np.uint64(3 * 15)
    box_h = kh >> np.uint64(3 * 15)
    pairs = np.unique(np.stack([box_m, box_h], axis=1), axis=0)
    assert len(pairs) == len(np.unique(box_m)) == len(np.unique(box_h))


def _box_set(t):
    lev, first, count, skip = t.nodes()
    cen = t.centres()
    return sorted(zip(lev.tolist(), map(tuple, np.round(cen, 15).tolist()), count.tolist(),
                      (skip == np.arange(len(lev)) + 1).tolist()))


@pytest.mark.parametrize("cap", [1, 8, 24])
def test_same_boxes_as_the_morton_tree(cap):
    cl = inputs.gaussian_cloud(3000, 1.0, 1e-3, 1e-5, 71)
    th = oracle.Tree(cl.x, cl.q, 0.5, 0.01, leaf_cap=cap, curve=H)
    tm = oracle.Tree(cl.x, cl.q, 0.5, 0.01, leaf_cap=cap, curve=M)
    assert th.nnodes == tm.nnodes
    assert _box_set(th) == _box_set(tm)
    # preorder: a node's particles are the contiguous run its first/count name
    lev, first, count, skip = th.nodes()
    kh = th.sorted_keys()
    assert np.all(np.diff(kh.astype(object)) >= 0)
    for k in range(0, len(lev), 37):
        run = kh[first[k]:first[k] + count[k]] >> np.uint64(3 * (21 - lev[k]))
        assert np.all(run == run[0])


def test_per_particle_lists_do_not_depend_on_the_curve():
    cl = inputs.gaussian_cloud(1500, 1.0, 1e-3, 1e-5, 72)
    rh = oracle.Tree(cl.x, cl.q, 0.6, 0.01, leaf_cap=8, G=1, curve=H).eval(want_phi=True)
    rm = oracle.Tree(cl.x, cl.q, 0.6, 0.01, leaf_cap=8, G=1, curve=M).eval(want_phi=True)
    assert (rh["m2p"], rh["p2p"]) == (rm["m2p"], rm["p2p"])
    assert np.linalg.norm(rh["f"] - rm["f"]) / np.linalg.norm(rm["f"]) < 1e-13
    assert np.linalg.norm(rh["phi"] - rm["phi"]) / np.linalg.norm(rm["phi"]) < 1e-13


def test_hilbert_tree_at_theta0_is_the_direct_sum():
    cl = inputs.gaussian_cloud(700, 1.0, 1e-3, 1e-5, 73)
    r = oracle.Tree(cl.x, cl.q, 0.0, 0.01, leaf_cap=8, G=32, curve=H).eval(want_phi=True)
    fd, pd = oracle.direct(cl.x, cl.q, 0.01)
    assert r["m2p"] == 0
    assert np.linalg.norm(r["f"] - fd) / np.linalg.norm(fd) < 1e-13


def test_chunk_groups_in_hilbert_order_are_more_compact():
    # the point of the curve: a run of G consecutive particles spans fewer
    # far-apart boxes, so the shared lists are shorter
    cl = inputs.gaussian_cloud(20000, 1.0, 1e-3, 1e-5, 74)
    rh = oracle.Tree(cl.x, cl.q, 0.5, 0.01, curve=H).eval(want_phi=False)
    rm = oracle.Tree(cl.x, cl.q, 0.5, 0.01, curve=M).eval(want_phi=False)
    assert rh["m2p"] + rh["p2p"] < rm["m2p"] + rm["p2p"]


def test_an_invalid_curve_is_refused():
    cl = inputs.gaussian_cloud(10, 1.0, 1e-3, 1e-5, 75)
    with pytest.raises(ValueError):
        oracle.Tree(cl.x, cl.q, 0.5, 0.01, curve=2)
