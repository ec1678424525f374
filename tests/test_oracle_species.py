"""Pins of the oracle's paper-literal pseudo-particles (Sec. 3, Eq. (5)).

With EXP_SPECIES a box carries, per sign of charge, the summed charge placed
at that species' centre of charge, and it is accepted for a target iff
s/theta + delta < d for every species it holds (delta: pseudo-particle to box
centre, d: target to pseudo-particle).  The pins: theta = 0 is the direct sum;
a box whose species are single particles is represented exactly; the
accepted and opened counts equal an independent numpy walk written from the
definition; the force error falls as theta does.
"""
import numpy as np
import pytest

import oracle
from paper_0709_3331_amd import inputs

S = oracle.EXP_SPECIES


def relrms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_theta0_is_the_direct_sum():
    cl = inputs.gaussian_cloud(500, 1.0, 1e-3, 1e-5, 21)
    r = oracle.Tree(cl.x, cl.q, 0.0, 0.01, leaf_cap=4, G=16, expansion=S).eval(want_phi=True)
    fd, pd = oracle.direct(cl.x, cl.q, 0.01)
    assert r["m2p"] == 0
    assert relrms(r["f"], fd) < 1e-13 and relrms(r["phi"], pd) < 1e-13


def test_single_particle_species_are_exact():
    # an ion and an electron share one box far from the target: their two
    # pseudo-particles are the particles themselves
    x = np.array([[0.10, 0.10, 0.10], [0.12, 0.11, 0.10], [0.90, 0.90, 0.90]])
    q = np.array([1.0, -1.0, 1.0])
    t = oracle.Tree(x, q, 0.9, 0.001, leaf_cap=2, G=1, expansion=S)
    r = t.eval(want_phi=True, group_counts=True)
    fd, pd = oracle.direct(x, q, 0.001)
    assert r["m2p"] >= 1                      # the pair's box was accepted
    np.testing.assert_allclose(r["f"][2], fd[2], rtol=1e-13)
    assert r["phi"][2] == pytest.approx(pd[2], rel=1e-13)


def _numpy_counts(x, q, theta, leaf_cap):
    """Accepted-box and opened-source counts of the per-particle walk, from
    the definition of Eq. (5) with per-species pseudo-particles."""
    t = oracle.Tree(x, q, theta, 0.01, leaf_cap=leaf_cap, G=1)
    lev, first, count, skip = t.nodes()
    cen = t.centres()
    perm = t.perm()
    xs, qs = x[perm], q[perm]
    lo, e = t.cube()
    M = len(lev)
    pseudo = []
    for k in range(M):
        sl = slice(first[k], first[k] + count[k])
        ent = []
        for sign in (1, -1):
            m = np.sign(qs[sl]) == sign
            if not m.any():
                continue
            Q = qs[sl][m].sum()
            c = (qs[sl][m][:, None] * xs[sl][m]).sum(axis=0) / Q
            ent.append((c, np.linalg.norm(c - cen[k])))
        pseudo.append(ent)
    m2p = p2p = 0
    for i in range(len(x)):
        stack = [0]
        while stack:
            k = stack.pop()
            s = 2.0 ** (e - lev[k])
            ok = all(s / theta + dlt < np.linalg.norm(xs[i] - c) for c, dlt in pseudo[k])
            if ok:
                m2p += 1
            elif skip[k] == k + 1:           # a leaf
                p2p += count[k]
            else:
                ch = k + 1
                while ch < skip[k]:
                    stack.append(ch)
                    ch = skip[ch]
    return m2p, p2p


@pytest.mark.parametrize("theta", [0.4, 0.8])
def test_lists_match_a_walk_from_the_definition(theta):
    cl = inputs.gaussian_cloud(60, 1.0, 1e-3, 1e-5, 22)
    r = oracle.Tree(cl.x, cl.q, theta, 0.01, leaf_cap=2, G=1, expansion=S).eval()
    m2p, p2p = _numpy_counts(cl.x, cl.q, theta, 2)
    assert (r["m2p"], r["p2p"]) == (m2p, p2p)


def test_error_falls_with_theta():
    cl = inputs.gaussian_cloud(3000, 1.0, 1e-3, 1e-5, 23)
    fd, _ = oracle.direct(cl.x, cl.q, 0.01)
    errs = [relrms(oracle.Tree(cl.x, cl.q, th, 0.01, expansion=S).eval(want_phi=False)["f"], fd)
            for th in (0.8, 0.5, 0.3, 0.15)]
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3


def test_species_trees_do_not_keep_lists():
    cl = inputs.gaussian_cloud(50, 1.0, 1e-3, 1e-5, 24)
    with pytest.raises(ValueError):
        oracle.Tree(cl.x, cl.q, 0.5, 0.01, keep_lists=True, expansion=S)
