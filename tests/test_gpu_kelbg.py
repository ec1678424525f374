"""GPU parity of the Kelbg pair law (Sec. 2.1, Eq. (3)) against the oracle.

Under UCP_PAIR_KELBG the walk's particle-particle terms take the Kelbg law for
electron-ion pairs and the softened (eps = 0: bare) Coulomb law for like
pairs; accepted boxes keep the expansion.  The oracle tree with the same pair
law has the same lists, so FP64 must agree to rounding and SPLIT to its FP32
bar (1e-5 relative RMS).  theta = 0 is checked against the oracle's direct
sum, and the adjoint must refuse the law.
"""
import numpy as np
import pytest

import oracle
from paper_0709_3331_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0709_3331_amd import _lib as L  # noqa: E402
from paper_0709_3331_amd.tree import TreeSolver  # noqa: E402

K = L.UCP_PAIR_KELBG
TOL = {L.UCP_FP64: 1e-12, L.UCP_SPLIT: 1e-5}


def say(*a):
    print(*a, flush=True)


def relrms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


CASES = [
    # id, n, seed, theta, eps (like pairs), lambda, leaf_cap, G, group_mode
    ("bare-like", 3000, 41, 0.5, 0.0, 0.02, 8, 64, L.UCP_GROUP_CHUNK),
    ("soft-like", 2501 * 2, 42, 0.6, 0.01, 0.05, 24, 32, L.UCP_GROUP_NODE),
    ("per-particle", 800, 43, 0.7, 0.002, 0.3, 1, 1, L.UCP_GROUP_CHUNK),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_kelbg_tree_matches_oracle_tree(case):
    name, n, seed, theta, eps, lam, cap, G, gm = case
    say(f"[kelbg] case={name} n={n} theta={theta} eps={eps} lambda={lam}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, seed)
    ref = oracle.Tree(cl.x, cl.q, theta, eps, leaf_cap=cap, G=G, group_mode=gm, pair_law=K,
                      lambda_ei=lam).eval(want_phi=True)
    for prec in (L.UCP_FP64, L.UCP_SPLIT):
        ts = TreeSolver(n, theta=theta, eps=eps, leaf_cap=cap, group_size=G, group_mode=gm,
                        precision=prec, pair_law=K, lambda_ei=lam)
        f, phi = ts.tree_forces(dev(cl.x), dev(cl.q), want_phi=True)
        st = ts.stats()
        ef, ep = relrms(f.cpu().numpy(), ref["f"]), relrms(phi.cpu().numpy(), ref["phi"])
        say(f"[kelbg]   prec={prec} force {ef:.3e} phi {ep:.3e}")
        assert st["p2p"] == ref["p2p"] and st["m2p"] == ref["m2p"]
        assert ef < TOL[prec] and ep < TOL[prec]
        ts.close()


def test_kelbg_theta0_equals_direct_sum():
    n, lam = 1500, 0.01
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 44)
    fd, pd = oracle.direct_pair(cl.x, cl.q, 0.0, K, lam)
    ts = TreeSolver(n, theta=0.0, eps=0.0, precision=L.UCP_FP64, pair_law=K, lambda_ei=lam)
    f, phi = ts.tree_forces(dev(cl.x), dev(cl.q), want_phi=True)
    assert relrms(f.cpu().numpy(), fd) < 1e-12
    assert relrms(phi.cpu().numpy(), pd) < 1e-12
    ts.close()


def test_full_size_metric_cloud_sampled_groups():
    # the N = 524,288 cloud under the Kelbg law (bare like pairs,
    # lambda = 0.005), every 97th walk group against the oracle's groups
    cl, prm = inputs.metric(0)
    lam = 0.005
    say(f"[kelbg] metric cloud n={cl.n}")
    t = oracle.Tree(cl.x, cl.q, 0.5, 0.0, pair_law=K, lambda_ei=lam)
    gsel = np.arange(0, t.ngroups, 97)
    ref = t.eval_groups(gsel, want_phi=True)
    mask = ~np.isnan(ref["f"][:, 0])
    ts = TreeSolver(cl.n, theta=0.5, eps=0.0, precision=L.UCP_SPLIT, pair_law=K, lambda_ei=lam)
    f, phi = ts.tree_forces(dev(cl.x), dev(cl.q), want_phi=True)
    ts.stats()
    f, phi = f.cpu().numpy(), phi.cpu().numpy()
    ef = relrms(f[mask], ref["f"][mask])
    ep = relrms(phi[mask], ref["phi"][mask])
    say(f"[kelbg]   {mask.sum()} sampled particles: force {ef:.3e} phi {ep:.3e}")
    assert ef < 1e-5 and ep < 1e-5
    ts.close()


def test_switching_the_pair_law_without_a_rebuild():
    n, lam = 2000, 0.03
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 45)
    ts = TreeSolver(n, theta=0.5, eps=0.01, precision=L.UCP_FP64)
    ts.build(dev(cl.x), dev(cl.q))
    fp = ts.forces(n).cpu().numpy()
    ts.set_params(theta=0.5, eps=0.01, precision=L.UCP_FP64, pair_law=K, lambda_ei=lam)
    fk = ts.forces(n).cpu().numpy()
    ts.stats()
    rp = oracle.Tree(cl.x, cl.q, 0.5, 0.01).eval()["f"]
    rk = oracle.Tree(cl.x, cl.q, 0.5, 0.01, pair_law=K, lambda_ei=lam).eval()["f"]
    assert relrms(fp, rp) < 1e-12 and relrms(fk, rk) < 1e-12
    ts.close()


def test_kelbg_parameters_are_checked_and_the_vjp_refuses():
    with pytest.raises(L.UcpError) as ei:
        TreeSolver(100, pair_law=K, lambda_ei=0.0)
    assert ei.value.status == L.UCP_EINVAL
    with pytest.raises(L.UcpError):
        TreeSolver(100, eps=0.0)               # Plummer needs eps > 0
    with pytest.raises(L.UcpError):
        TreeSolver(100, pair_law=7, lambda_ei=0.1)
    cl = inputs.gaussian_cloud(200, 1.0, 1e-3, 1e-5, 46)
    ts = TreeSolver(200, eps=0.0, pair_law=K, lambda_ei=0.01)
    ts.build(dev(cl.x), dev(cl.q))
    with pytest.raises(L.UcpError) as ei:
        ts.vjp(torch.zeros((200, 3), dtype=torch.float64, device="cuda"))
    assert ei.value.status == L.UCP_EINVAL
    ts.close()
