"""Pins of the oracle's Kelbg pair law (Sec. 2.1, Eq. (3)).

The electron-ion pair interacts through V = C (1 - exp(-r/lambda)) / r with
C = q_i q_j; like pairs through the (softened, eps = 0: bare) Coulomb law.
The oracle evaluates the force bracket 1 - e^{-u}(1 + u) and the potential
bracket 1 - e^{-u} (u = r/lambda) by Taylor series below u = 1/4 and directly
above.  These tests pin it to things fixed independently of that code: the
derivative of V taken by finite differences, numpy's expm1, the asymptotes
the paper states (C/lambda (1 - r/(2 lambda)) for r << lambda, C/r for
r >> lambda), the bare Coulomb law, momentum conservation and the tree at
theta = 0.
"""
import numpy as np
import pytest

import oracle
from paper_0709_3331_amd import inputs

K = oracle.PAIR_KELBG


def pair(r, lam, qi=1.0, qj=-1.0, eps=0.0):
    """Oracle force on particle 0 and potential at particle 0 for two particles
    a distance r apart along a fixed oblique direction."""
    d = np.array([0.48, -0.6, 0.64])   # unit vector
    x = np.stack([np.zeros(3), -r * d])
    f, phi = oracle.direct_pair(x, np.array([qi, qj]), eps, K, lam)
    return f[0], phi[0], d


def V(r, lam, C):
    return C * (-np.expm1(-r / lam)) / r


@pytest.mark.parametrize("u", [1e-3, 0.05, 0.2, 0.249, 0.251, 0.7, 3.0, 12.0])
def test_electron_ion_force_is_minus_dV_dr(u):
    lam = 0.02
    r = u * lam
    f, phi, d = pair(r, lam)
    # F_0 = -dV/dr along x_0 - x_1 = r d; central differences of V(r)
    h = 1e-4 * r
    dv = (V(r + h, lam, -1.0) - V(r - h, lam, -1.0)) / (2 * h)
    want = -dv * d
    np.testing.assert_allclose(f, want, rtol=2e-7, atol=0)
    # potential at particle 0: q_1 (1 - e^{-u}) / r
    assert phi == pytest.approx(-(-np.expm1(-u)) / r, rel=1e-13)


def test_short_range_asymptote_of_the_paper():
    # for r << lambda, V -> C / lambda (1 - r / (2 lambda)); the next term is
    # C r^2 / (6 lambda^3)
    lam = 0.01
    for u in (1e-6, 1e-4, 1e-2):
        _, phi, _ = pair(u * lam, lam, qi=1.0, qj=-1.0)
        approx = -(1.0 / lam) * (1.0 - u / 2)
        assert abs(phi - approx) <= 1.01 * (u * u / 6) / lam + 1e-15


def test_far_field_is_coulomb():
    lam = 1e-3
    r = 60 * lam                     # e^{-60}: below FP64 resolution of 1
    f, phi, d = pair(r, lam)
    np.testing.assert_allclose(f, -d / r ** 2, rtol=1e-15)
    assert phi == pytest.approx(-1.0 / r, rel=1e-15)


def test_coincident_electron_ion_pair():
    f, phi, _ = pair(0.0, 0.01)
    assert np.all(f == 0.0)
    assert phi == pytest.approx(-1.0 / 0.01, rel=1e-15)


@pytest.mark.parametrize("qi,qj", [(1.0, 1.0), (-1.0, -1.0)])
def test_like_pairs_take_bare_coulomb(qi, qj):
    r = 0.003
    f, phi, d = pair(r, 0.05, qi, qj, eps=0.0)
    np.testing.assert_allclose(f, qi * qj * d / r ** 2, rtol=1e-15)
    assert phi == pytest.approx(qj / r, rel=1e-15)


def test_like_pairs_keep_the_softening():
    r, eps = 0.003, 0.002
    f, phi, d = pair(r, 0.05, 1.0, 1.0, eps=eps)
    np.testing.assert_allclose(f, d * r / (r * r + eps * eps) ** 1.5, rtol=1e-14)


def test_momentum_is_conserved_and_small_lambda_is_coulomb():
    cl = inputs.gaussian_cloud(400, 1.0, 1e-3, 1e-5, 5)
    f, _ = oracle.direct_pair(cl.x, cl.q, 0.0, K, 0.01)
    assert np.abs(f.sum(axis=0)).max() / np.abs(f).sum() < 1e-14
    # lambda far below every separation: every pair is bare Coulomb, which the
    # softened law with a negligible eps reproduces
    fk, pk = oracle.direct_pair(cl.x, cl.q, 0.0, K, 1e-9)
    fc, pc = oracle.direct(cl.x, cl.q, 1e-12)
    np.testing.assert_allclose(fk, fc, rtol=1e-9, atol=1e-9 * np.abs(fc).max())
    np.testing.assert_allclose(pk, pc, rtol=1e-9, atol=1e-9 * np.abs(pc).max())


def test_kelbg_differs_from_plummer_only_for_electron_ion_pairs():
    cl = inputs.gaussian_cloud(300, 1.0, 1e-3, 1e-5, 6)
    ions = cl.q > 0
    x, q = cl.x[ions], cl.q[ions]      # ions only: every pair is like
    fk, pk = oracle.direct_pair(x, q, 0.01, K, 0.05)
    fp, pp = oracle.direct(x, q, 0.01)
    np.testing.assert_array_equal(fk, fp)
    np.testing.assert_array_equal(pk, pp)


def test_tree_at_theta0_equals_the_direct_sum():
    cl = inputs.gaussian_cloud(600, 1.0, 1e-3, 1e-5, 7)
    lam = 0.02
    t = oracle.Tree(cl.x, cl.q, 0.0, 0.0, leaf_cap=8, G=32, pair_law=K, lambda_ei=lam)
    r = t.eval(want_phi=True)
    fd, pd = oracle.direct_pair(cl.x, cl.q, 0.0, K, lam)
    np.testing.assert_allclose(r["f"], fd, rtol=1e-10, atol=1e-12 * np.abs(fd).max())
    np.testing.assert_allclose(r["phi"], pd, rtol=1e-10, atol=1e-12 * np.abs(pd).max())


def test_kelbg_tree_changes_only_the_near_field():
    # at theta > 0 the accepted boxes keep the softened expansion; the Kelbg
    # and Plummer trees then differ only through the opened leaves' pairs
    cl = inputs.gaussian_cloud(2000, 1.0, 1e-3, 1e-5, 8)
    tk = oracle.Tree(cl.x, cl.q, 0.5, 0.01, pair_law=K, lambda_ei=1e-9)
    tp = oracle.Tree(cl.x, cl.q, 0.5, 0.01)
    rk, rp = tk.eval(), tp.eval()
    # the opening test does not depend on the pair law: the same lists
    assert rk["p2p"] == rp["p2p"] and rk["m2p"] == rp["m2p"]
    assert np.isfinite(rk["f"]).all() and not np.array_equal(rk["f"], rp["f"])
    # the accepted boxes' share is the same in both: the difference is the
    # near field of the electron-ion pairs, so with every particle's partner
    # far (a dilute copy of the cloud) the two trees agree closely
    xs = cl.x * 50.0
    rk2 = oracle.Tree(xs, cl.q, 0.5, 0.01, pair_law=K, lambda_ei=1e-9).eval()
    rp2 = oracle.Tree(xs, cl.q, 0.5, 0.01).eval()
    assert np.linalg.norm(rk2["f"] - rp2["f"]) / np.linalg.norm(rp2["f"]) < 1e-3


def test_invalid_pair_laws_and_the_vjp_refuse():
    cl = inputs.gaussian_cloud(100, 1.0, 1e-3, 1e-5, 9)
    with pytest.raises(ValueError):
        oracle.direct_pair(cl.x, cl.q, 0.0, K, 0.0)
    with pytest.raises(ValueError):
        oracle.direct_pair(cl.x, cl.q, 0.0, 7, 0.1)
    t = oracle.Tree(cl.x, cl.q, 0.5, 0.01, keep_lists=True, pair_law=K, lambda_ei=0.01)
    with pytest.raises(Exception):
        t.vjp(np.ones((100, 3)))
