"""GPU parity of the HIP TREE path against the FP64 CPU oracle.

Every comparison is made through the C-ABI on the same seeded inputs:
keys, permutation, topology, box centres, groups and per-group interaction
counts bit-exact; moments to 1e-13 of their natural scale; forces to 1e-12
relative RMS on the FP64 path and 1e-5 on the FP32/FP64 split path, and
particle by particle within the rounding bound of the terms each force is
summed from.
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

TOL_FP64 = 1e-12
TOL_SPLIT = 1e-5
# Per-particle bound.  The oracle returns A_i, the sum over the terms of E_i
# of each term's size (its sums over magnitudes) and of its Jacobian times
# the largest move of its offset when the offsets are rounded relative to a
# point of the group's bounding box.  Each term takes at most 32 roundings in
# sequence and the walk sums at most 64 terms in the working precision
# (unit roundoff u_w) before an FP64 accumulator, so
#     |F_i(GPU) - F_i(oracle)| <= K (u_w + 2^-53) |q_i| A_i,  K = 128,
# the 2^-53 term covering the oracle's own FP64 rounding.
K_BOUND = 128.0
U32, U64 = 2.0 ** -24, 2.0 ** -53


def say(*a):
    print(*a, flush=True)


def relrms(a, b):
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def force_bound_ratio(f, ref, cond, q, prec):
    """max_i |F_i - ref_i| / (per-particle bound); <= 1 passes."""
    uw = U32 if prec == L.UCP_SPLIT else U64
    m = ~np.isnan(ref[:, 0])
    tol = K_BOUND * (uw + U64) * np.abs(q[m]) * cond[m]
    err = np.linalg.norm(f[m] - ref[m], axis=1)
    return float(np.max(err / np.maximum(tol, 1e-300))) if err.size else 0.0


def per_particle_rel(f, ref):
    """median, 99th percentile and maximum of |F_i - ref_i| / |ref_i|."""
    m = ~np.isnan(ref[:, 0])
    r = np.linalg.norm(f[m] - ref[m], axis=1) / np.maximum(np.linalg.norm(ref[m], axis=1), 1e-300)
    return float(np.median(r)), float(np.quantile(r, 0.99)), float(r.max())


def check_topology(ts, t):
    """GPU build vs oracle tree t: keys, permutation, nodes, centres, groups."""
    np.testing.assert_array_equal(ts.debug("keys"), t.sorted_keys())
    np.testing.assert_array_equal(ts.debug("perm").astype(np.int64), t.perm())
    lv, fi, co, sk = t.nodes()
    ni = ts.debug("ninfo")
    assert ni.shape[0] == t.nnodes
    np.testing.assert_array_equal(ni[:, 0], fi)
    np.testing.assert_array_equal(ni[:, 1], co)
    np.testing.assert_array_equal(ni[:, 2], sk)
    np.testing.assert_array_equal(ni[:, 3] & 255, lv)
    np.testing.assert_array_equal((ni[:, 3] >> 8) & 1, (sk == np.arange(t.nnodes) + 1).astype(np.int32))
    geo = ts.debug("ngeo")
    np.testing.assert_array_equal(geo[:, :3], t.centres())
    lo, e = t.cube()
    np.testing.assert_array_equal(geo[:, 3], (2.0 ** (e - lv.astype(np.float64))) ** 2)
    gf, gc, gn = t.groups()
    gr = ts.debug("groups")
    np.testing.assert_array_equal(gr[:, 0], gf)
    np.testing.assert_array_equal(gr[:, 1], gc)
    np.testing.assert_array_equal(gr[:, 2], gn)


def check_moments(ts, t, x, q):
    ref = t.moments(x)
    got = ts.debug("moments")
    lv = t.nodes()[0]
    e = t.cube()[1]
    s = 2.0 ** (e - lv.astype(np.float64))
    # natural scale of each moment order: sum|q| * (box side)^order
    qa = np.abs(q).sum()
    scale = np.stack([np.full_like(s, qa)] + [qa * s] * 3 + [qa * s * s] * 6, axis=1)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)


NODE, CHUNK = L.UCP_GROUP_NODE, L.UCP_GROUP_CHUNK
CASES = [
    # id, n, seed, theta, eps, leaf_cap, G, key_bits, halo, group_mode
    ("small", 4096, 0, 0.5, 0.01, 8, 64, 63, 0.0, NODE),
    ("ragged", 3002, 1, 0.6, 0.01, 4, 32, 30, 0.0, NODE),
    ("per-particle", 1000, 2, 0.7, 0.02, 1, 1, 63, 0.0, NODE),
    ("halo", 20000, 3, 0.5, 0.005, 8, 64, 63, 0.05, NODE),
    ("tiles", 70002, 4, 0.3, 0.005, 16, 48, 63, 0.0, NODE),
    ("chunk-small", 4096, 0, 0.5, 0.01, 8, 64, 63, 0.0, CHUNK),
    ("chunk-ragged", 3002, 1, 0.6, 0.01, 4, 24, 30, 0.0, CHUNK),
    ("chunk-halo", 20000, 3, 0.5, 0.005, 8, 32, 63, 0.05, CHUNK),
    ("chunk-per-particle", 1000, 2, 0.7, 0.02, 1, 1, 63, 0.0, CHUNK),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tree_parity(case):
    name, n, seed, theta, eps, cap, G, kb, halo, gm = case
    say(f"[parity] case={name} n={n} seed={seed} theta={theta} G={G} leaf_cap={cap} bits={kb} "
        f"group_mode={gm}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, seed, halo_frac=halo)
    b = 21 if kb == 63 else 10
    t = oracle.Tree(cl.x, cl.q, theta, eps, b=b, leaf_cap=cap, G=G, group_mode=gm)
    ref = t.eval(group_counts=True, cond=True)
    x, q = dev(cl.x), dev(cl.q)
    for prec, tol in ((L.UCP_FP64, TOL_FP64), (L.UCP_SPLIT, TOL_SPLIT)):
        ts = TreeSolver(n, 1, theta=theta, eps=eps, leaf_cap=cap, group_size=G, key_bits=kb,
                        precision=prec, list_len=64, group_mode=gm)
        f, phi = ts.tree_forces(x, q, want_phi=True)
        st = ts.stats()
        say(f"[parity]   prec={prec} nodes={st['nodes']} groups={st['groups']} "
            f"p2p={st['p2p']} m2p={st['m2p']}")
        check_topology(ts, t)
        check_moments(ts, t, cl.x, cl.q)
        gs = ts.debug("gstat")
        np.testing.assert_array_equal(gs[:, 0], ref["gm2p"])
        np.testing.assert_array_equal(gs[:, 1], ref["gp2p"])
        assert st["p2p"] == ref["p2p"] and st["m2p"] == ref["m2p"]
        fa = f.cpu().numpy()
        ef = relrms(fa, ref["f"])
        ep = relrms(phi.cpu().numpy(), ref["phi"])
        ratio = force_bound_ratio(fa, ref["f"], ref["cond"], cl.q, prec)
        med, p99, mx = per_particle_rel(fa, ref["f"])
        say(f"[parity]   force rel RMS vs oracle tree {ef:.3e}, phi {ep:.3e}; per particle: "
            f"median {med:.2e} p99 {p99:.2e} max {mx:.2e}; max error / bound {ratio:.3e}")
        assert ef < tol and ep < tol
        assert ratio <= 1.0
        ts.close()


def test_theta0_equals_direct():
    n = 2048
    say(f"[parity] theta=0 vs direct n={n}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 7)
    fd, phid = oracle.direct(cl.x, cl.q, 0.01)
    for prec, tol in ((L.UCP_FP64, 1e-12), (L.UCP_SPLIT, 1e-5)):
        ts = TreeSolver(n, theta=0.0, eps=0.01, precision=prec)
        f, phi = ts.tree_forces(dev(cl.x), dev(cl.q), want_phi=True)
        st = ts.stats()
        assert st["m2p"] == 0 and st["p2p"] == n * n
        assert relrms(f.cpu().numpy(), fd) < tol
        assert relrms(phi.cpu().numpy(), phid) < tol
        ts.close()


def test_degenerate_inputs():
    say("[parity] degenerate: n=0, 1, 2, coincident")
    ts = TreeSolver(256, theta=0.5, eps=0.01, precision=L.UCP_FP64)
    x = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    f = ts.tree_forces(x, torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert f.shape == (0, 3)
    # one particle: no force, zero potential
    f, phi = ts.tree_forces(dev([[0.3, -0.2, 0.1]]), dev([1.0]), want_phi=True)
    assert f.abs().max().item() == 0.0 and phi.abs().max().item() == 0.0
    # two particles: closed form
    xx = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.0]])
    f, phi = ts.tree_forces(dev(xx), dev([1.0, -1.0]), want_phi=True)
    fd, pd = oracle.direct(xx, [1.0, -1.0], 0.01)
    np.testing.assert_allclose(f.cpu().numpy(), fd, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(phi.cpu().numpy(), pd, rtol=1e-14)
    # 100 coincident particles (one max-depth leaf chain) + 100 at another point
    xx = np.zeros((200, 3)); xx[100:] = [0.5, 0.25, -0.125]
    qq = np.where(np.arange(200) % 2 == 0, 1.0, -1.0)
    t = oracle.Tree(xx, qq, 0.5, 0.01, G=64)
    ref = t.eval()
    f, phi = ts.tree_forces(dev(xx), dev(qq), want_phi=True)
    check_topology(ts, t)
    assert relrms(f.cpu().numpy(), ref["f"]) < 1e-12 or np.abs(ref["f"]).max() < 1e-12
    np.testing.assert_allclose(phi.cpu().numpy(), ref["phi"], rtol=1e-12, atol=1e-9)
    ts.close()


def test_large_coincident_cluster():
    # 3000 coincident particles beside a cloud: a chain of internal nodes of
    # more than 1024 particles down to the maximum depth, each with one child,
    # whose ends and children come from the searches over the sorted keys and
    # whose moments come from their children, level by level
    say("[parity] 3000 coincident particles beside a cloud of 3000")
    cl = inputs.gaussian_cloud(6000, 1.0, 1e-3, 1e-5, 11)
    x = cl.x.copy()
    x[:3000] = [0.37, -0.41, 0.29]
    for cap in (8, 24):
        t = oracle.Tree(x, cl.q, 0.5, 0.01, leaf_cap=cap, G=64, group_mode=CHUNK)
        ref = t.eval(want_phi=True)
        lv, fi, co, sk = t.nodes()
        assert int(lv.max()) == 21 and int(co[sk != np.arange(len(lv)) + 1].max()) > 1024
        ts = TreeSolver(6000, theta=0.5, eps=0.01, leaf_cap=cap, group_size=64,
                        precision=L.UCP_FP64, group_mode=CHUNK)
        f, phi = ts.tree_forces(dev(x), dev(cl.q), want_phi=True)
        st = ts.stats()
        say(f"[parity]   leaf_cap={cap} nodes={st['nodes']} max level={int(lv.max())}")
        check_topology(ts, t)
        check_moments(ts, t, x, cl.q)
        assert relrms(f.cpu().numpy(), ref["f"]) < TOL_FP64
        assert relrms(phi.cpu().numpy(), ref["phi"]) < TOL_FP64
        ts.close()


def test_nonfinite_input_is_flagged():
    say("[parity] non-finite input")
    ts = TreeSolver(64, theta=0.5, eps=0.01)
    xx = np.random.default_rng(0).normal(size=(64, 3)); xx[5, 1] = np.nan
    ts.build(dev(xx), dev(np.ones(64)))
    with pytest.raises(L.UcpError) as ei:
        ts.stats()
    assert ei.value.status == L.UCP_ENONFINITE
    # the context recovers on the next good build
    xx[5, 1] = 0.0
    f = ts.tree_forces(dev(xx), dev(np.ones(64)))
    ts.stats()
    assert torch.isfinite(f).all()
    ts.close()


def test_flags_survive_later_builds_until_read():
    # a flag raised by one build stays visible after a later clean build
    # (as between the steps of one multi-step call) until ucp_get_stats reads it
    say("[parity] sticky flags")
    ts = TreeSolver(64, theta=0.5, eps=0.01)
    good = np.random.default_rng(2).normal(size=(64, 3))
    bad = good.copy(); bad[7, 2] = np.inf
    ts.build(dev(bad), dev(np.ones(64)))
    f = ts.tree_forces(dev(good), dev(np.ones(64)))
    with pytest.raises(L.UcpError) as ei:
        ts.stats()
    assert ei.value.status == L.UCP_ENONFINITE
    st = ts.stats()                      # read: the sticky word is clear
    assert st["flags"] == 0 and torch.isfinite(f).all()
    ts.close()


@pytest.mark.parametrize("gm", [NODE, CHUNK])
def test_batched_clouds_match_independent_clouds(gm):
    sizes = [100, 0, 2000, 74, 4096, 2]
    say(f"[parity] batched clouds sizes={sizes} group_mode={gm}")
    parts = [inputs.gaussian_cloud(s, 0.5 + 0.3 * k, 1e-3, 1e-5, 100 + k) if s else None
             for k, s in enumerate(sizes)]
    x = np.concatenate([p.x for p in parts if p is not None])
    q = np.concatenate([p.q for p in parts if p is not None])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    for prec, tol in ((L.UCP_FP64, TOL_FP64), (L.UCP_SPLIT, TOL_SPLIT)):
        ts = TreeSolver(n, len(sizes), theta=0.5, eps=0.01, precision=prec, group_size=32,
                        group_mode=gm)
        f, phi = ts.tree_forces(dev(x), dev(q), offsets=torch.from_numpy(off).cuda(), want_phi=True)
        st = ts.stats()
        f, phi = f.cpu().numpy(), phi.cpu().numpy()
        for k, p in enumerate(parts):
            if p is None:
                continue
            a, b = off[k], off[k + 1]
            ref = oracle.tree_forces(p.x, p.q, 0.5, 0.01, G=32, group_mode=gm)
            assert relrms(f[a:b], ref["f"]) < tol, k
            assert relrms(phi[a:b], ref["phi"]) < tol, k
        cube = ts.debug("cube")
        for k, p in enumerate(parts):
            if p is not None:
                lo, e = oracle.cube(p.x)
                np.testing.assert_array_equal(cube[k, :3], lo)
                assert cube[k, 3] == e
        assert st["clouds"] == len(sizes)
        # groups: each cloud's own groups, shifted by the cloud's offset
        gr = ts.debug("groups")
        want = []
        for k, p in enumerate(parts):
            if p is not None:
                gf, gc, _ = oracle.Tree(p.x, p.q, 0.5, 0.01, G=32, group_mode=gm).groups()
                want += [(off[k] + a, c) for a, c in zip(gf, gc)]
        assert [tuple(r) for r in gr[:, :2].tolist()] == [tuple(w) for w in np.array(want).tolist()]
        ts.close()


def test_bad_offsets_are_flagged():
    say("[parity] bad offsets")
    ts = TreeSolver(100, 3, theta=0.5, eps=0.01)
    x = dev(np.random.default_rng(1).normal(size=(100, 3)))
    q = dev(np.ones(100))
    ts.build(x, q, offsets=torch.tensor([0, 60, 40, 100], dtype=torch.int64, device="cuda"))
    with pytest.raises(L.UcpError) as ei:
        ts.stats()
    assert ei.value.status == L.UCP_EINVAL
    ts.close()


def test_rebuild_is_bitwise_deterministic():
    n = 30000
    say(f"[parity] determinism n={n}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 9)
    ts = TreeSolver(n, theta=0.5, eps=0.005)
    x, q = dev(cl.x), dev(cl.q)
    f1, p1 = ts.tree_forces(x, q, want_phi=True)
    m1 = ts.debug("moments")
    f2, p2 = ts.tree_forces(x, q, want_phi=True)
    m2 = ts.debug("moments")
    assert torch.equal(f1, f2) and torch.equal(p1, p2)
    np.testing.assert_array_equal(m1, m2)
    ts.close()


def test_verlet_and_energy_match_oracle():
    n, steps, dt, eps = 1024, 5, 1e-4, 0.01
    say(f"[parity] verlet n={n} steps={steps}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 11)
    ts = TreeSolver(n, theta=0.5, eps=eps, precision=L.UCP_FP64, group_size=32)
    x, v, q, m = dev(cl.x), dev(cl.v), dev(cl.q), dev(cl.m)
    f = ts.tree_forces(x, q)
    ts.step(x, v, f, q, m, dt, steps)
    xr, vr, fr = oracle.verlet(cl.x, cl.v, cl.q, cl.m, dt, steps, eps, mode="tree", theta=0.5, G=32)
    assert np.abs(x.cpu().numpy() - xr).max() < 1e-12
    assert relrms(v.cpu().numpy(), vr) < 1e-10
    assert relrms(f.cpu().numpy(), fr) < 1e-10
    # energies with the tree potential
    e = ts.energy(x, v, q, m).cpu().numpy()
    t = oracle.Tree(xr, cl.q, 0.5, eps, G=32)
    er = oracle.energy(vr, cl.q, cl.m, t.eval()["phi"])
    np.testing.assert_allclose(e, er, rtol=1e-10)
    ts.close()


def test_graph_replay_matches_eager_steps():
    n, dt = 4096, 1e-4
    say(f"[parity] graph replay n={n}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 12)
    ts = TreeSolver(n, theta=0.5, eps=0.01)
    q, m = dev(cl.q), dev(cl.m)
    runs = []
    for mode in ("eager", "graph"):
        x, v = dev(cl.x), dev(cl.v)
        f = ts.tree_forces(x, q)
        if mode == "eager":
            for _ in range(4):
                ts.step(x, v, f, q, m, dt, 1)
                torch.cuda.synchronize()
        else:
            ts.step(x, v, f, q, m, dt, 2)          # capture + two replays
            torch.cuda.synchronize()
            _ = (x * 1.0).sum().item()             # eager work between replays
            ts.step(x, v, f, q, m, dt, 2)
        torch.cuda.synchronize()
        runs.append((x.clone(), v.clone(), f.clone()))
    for a, b in zip(runs[0], runs[1]):
        assert torch.equal(a, b)
    ts.close()


def test_one_call_of_many_steps_matches_single_step_calls():
    # inside one call the closing kick of a step and the opening kick and
    # drift of the next are one kernel; the trajectory must be bitwise that of
    # one call per step
    n, dt, steps = 3000, 1e-4, 5
    say(f"[parity] {steps} steps in one call n={n}")
    cl = inputs.gaussian_cloud(n, 1.0, 1e-3, 1e-5, 13)
    ts = TreeSolver(n, theta=0.5, eps=0.01)
    q, m = dev(cl.q), dev(cl.m)
    runs = []
    for per_call in (1, steps):
        x, v = dev(cl.x), dev(cl.v)
        f = ts.tree_forces(x, q)
        for _ in range(steps // per_call):
            ts.step(x, v, f, q, m, dt, per_call)
        torch.cuda.synchronize()
        runs.append((x.clone(), v.clone(), f.clone()))
    for a, b in zip(runs[0], runs[1]):
        assert torch.equal(a, b)
    ts.close()


@pytest.mark.parametrize("gm,G", [(NODE, 64), (CHUNK, 64), (CHUNK, 32)])
def test_full_size_metric_cloud(gm, G):
    c, prm = inputs.metric(0)
    n = c.n
    say(f"[parity] metric cloud n={n} theta={prm['theta']} group_mode={gm} G={G}")
    t = oracle.Tree(c.x, c.q, prm["theta"], prm["eps"], G=G, group_mode=gm)
    ts = TreeSolver(n, theta=prm["theta"], eps=prm["eps"], group_size=G, group_mode=gm)
    x, q = dev(c.x), dev(c.q)
    f = ts.tree_forces(x, q)
    st = ts.stats()
    say(f"[parity]   nodes={st['nodes']} groups={st['groups']} p2p/N={st['p2p'] / n:.1f} "
        f"m2p/N={st['m2p'] / n:.1f}")
    check_topology(ts, t)
    ref = t.eval(group_counts=True, cond=True)
    gs = ts.debug("gstat")
    np.testing.assert_array_equal(gs[:, 0], ref["gm2p"])
    np.testing.assert_array_equal(gs[:, 1], ref["gp2p"])
    fa = f.cpu().numpy()
    ef = relrms(fa, ref["f"])
    ratio = force_bound_ratio(fa, ref["f"], ref["cond"], c.q, L.UCP_SPLIT)
    med, p99, mx = per_particle_rel(fa, ref["f"])
    say(f"[parity]   split force rel RMS vs oracle tree {ef:.3e}; per particle: median "
        f"{med:.2e} p99 {p99:.2e} max {mx:.2e}; max error / bound {ratio:.3e}")
    assert ef < TOL_SPLIT
    assert ratio <= 1.0
    ts.close()


def test_wave_clocks_of_a_timed_walk():
    # with timing on, every wave of the persistent walk stamps its start and
    # end; they lie inside the walk's own HIP-event span
    cl = inputs.gaussian_cloud(20000, 1.0, 1e-3, 1e-5, 31)
    x, q = torch.from_numpy(cl.x).cuda(), torch.from_numpy(cl.q).cuda()
    ts = TreeSolver(cl.n, theta=0.5, eps=0.01)
    ts.build(x, q)
    ts.timing(True)
    ts.forces(cl.n)
    ms, launches = ts.timing_read()
    t, unit = ts.wave_clock(units=True)
    ts.timing(False)
    ts.stats()
    ts.close()
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    cus, counts = np.unique(unit, return_counts=True)
    say(f"[clock] waves={t.shape[0]} span {t[:, 1].max():.1f} us, event {1e3 * ms:.1f} us; "
        f"{cus.shape[0]} units of {ncu} CUs, waves per unit {counts.min()}-{counts.max()}")
    assert launches == 1
    assert t.shape[0] % 4 == 0 and np.all(t[:, 1] >= t[:, 0]) and t[:, 0].min() == 0.0
    assert t[:, 1].max() <= 1e3 * ms + 20.0
    # the units name the CUs: every CU runs waves of the launch (8 blocks of
    # 4 waves per CU), and no unit ever holds more waves at once than a CU can
    # (4 per SIMD under the walk's LDS)
    assert cus.shape[0] == ncu
    for u in cus:
        iv = t[unit == u]
        ev = np.concatenate([np.stack([iv[:, 0], np.ones(len(iv))], 1),
                             np.stack([iv[:, 1], -np.ones(len(iv))], 1)])
        ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]   # at equal times, ends first
        assert np.cumsum(ev[:, 1]).max() <= 16, f"unit {u} holds more than 16 waves at once"
