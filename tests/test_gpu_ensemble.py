"""The batched ensemble at full size and the walk autotuner, on the GPU.

The 64-cloud ensemble (N_c = 2 U[4096, 65536], sigma_c = U[0.5, 2]) is built
and walked in one batched call; a sample of its clouds is compared with the
FP64 oracle tree of each cloud alone.  The autotuner must return one of its
candidates, the fastest it measured, and read it back from its cache.
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
from paper_0709_3331_amd import autotune  # noqa: E402
from paper_0709_3331_amd.tree import TreeSolver  # noqa: E402


def say(*a):
    print(*a, flush=True)


def relrms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_full_ensemble_sampled_clouds_match_oracle():
    ens, off, prm = inputs.ensemble()
    n, clouds = int(off[-1]), len(off) - 1
    say(f"[ensemble] clouds={clouds} n={n}")
    x, q = torch.from_numpy(ens.x).cuda(), torch.from_numpy(ens.q).cuda()
    offs = torch.from_numpy(off).cuda()
    sizes = np.diff(off)
    pick = [int(np.argmin(sizes)), 7, int(np.argmax(sizes))]
    for prec, tol in ((L.UCP_FP64, 1e-12), (L.UCP_SPLIT, 1e-5)):
        ts = TreeSolver(n, clouds, theta=prm["theta"], eps=prm["eps"], precision=prec)
        f = ts.tree_forces(x, q, offs).cpu().numpy()
        st = ts.stats()
        assert st["clouds"] == clouds
        # above 2^20 particles the sort's passes (cloud digits included) take
        # 4096-key tiles: each sampled cloud's keys and order bit-exact
        keys, perm = ts.debug("keys"), ts.debug("perm").astype(np.int64)
        for c in pick:
            a, b = off[c], off[c + 1]
            t = oracle.Tree(ens.x[a:b], ens.q[a:b], prm["theta"], prm["eps"])
            np.testing.assert_array_equal(keys[a:b], t.sorted_keys())
            np.testing.assert_array_equal(perm[a:b] - a, t.perm())
            ref = oracle.tree_forces(ens.x[a:b], ens.q[a:b], prm["theta"], prm["eps"], G=64)
            e = relrms(f[a:b], ref["f"])
            say(f"[ensemble]   prec={prec} cloud {c} (N={b - a}) rel RMS {e:.3e}")
            assert e < tol
        ts.close()


def test_batched_graph_step_matches_oracle_and_eager_steps():
    # ucp_step_batched on ragged clouds (one empty, one of 3 particles): calls
    # of 3 steps replay the captured graphs (a first call captures them);
    # positions and velocities against the oracle's Verlet run of each cloud
    # alone (FP64), and the graph path bitwise against the directly enqueued
    # steps (timing on) of the same calls.
    sizes = [900, 0, 2400, 64, 3]
    dt, theta, eps, steps, calls = 1e-4, 0.5, 0.01, 3, 2
    say(f"[ensemble] batched graph step sizes={sizes} calls={calls}x{steps}")
    parts = [inputs.gaussian_cloud(s, 0.7 + 0.2 * k, 1e-3, 1e-5, 60 + k) if s % 2 == 0 and s else None
             for k, s in enumerate(sizes)]
    tiny = np.random.default_rng(9).normal(size=(3, 3))
    xs = [p.x if p is not None else (tiny if s == 3 else np.zeros((0, 3)))
          for p, s in zip(parts, sizes)]
    vs = [p.v if p is not None else np.zeros((s, 3)) for p, s in zip(parts, sizes)]
    qs = [p.q if p is not None else np.array([1.0, -1.0, 1.0])[:s] for p, s in zip(parts, sizes)]
    ms = [p.m if p is not None else np.ones(s) for p, s in zip(parts, sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    cat = lambda a: torch.from_numpy(np.ascontiguousarray(np.concatenate(a))).cuda()  # noqa: E731
    q, m, offs = cat(qs), cat(ms), torch.from_numpy(off).cuda()
    ts = TreeSolver(n, len(sizes), theta=theta, eps=eps, precision=L.UCP_FP64, group_size=32)
    runs = []
    for mode in ("graph", "eager"):
        x, v = cat(xs), cat(vs)
        f = ts.tree_forces(x, q, offs)
        ts.timing(mode == "eager")
        for c in range(calls):
            ts.step(x, v, f, q, m, dt, steps, offsets=offs)
            torch.cuda.synchronize()
            _ = (x * 1.0).sum().item()          # eager work between the calls
        ts.timing(False)
        ts.timing_read()
        ts.stats()
        runs.append((x.clone(), v.clone(), f.clone()))
    for a, b in zip(runs[0], runs[1]):
        assert torch.equal(a, b)
    xg, vg = runs[0][0].cpu().numpy(), runs[0][1].cpu().numpy()
    for k in range(len(sizes)):
        a, b = off[k], off[k + 1]
        if b - a == 0:
            continue
        xr, vr, _ = oracle.verlet(xs[k], vs[k], qs[k], ms[k], dt, calls * steps, eps, mode="tree",
                                  theta=theta, G=32)
        dx = np.abs(xg[a:b] - xr).max()
        dv = np.linalg.norm(vg[a:b] - vr) / max(np.linalg.norm(vr), 1e-300)
        say(f"[ensemble]   cloud {k} (N={b - a}): max |dx| {dx:.2e}, v rel RMS {dv:.2e}")
        assert dx < 1e-12 and dv < 1e-12, k
    ts.close()


def test_autotune_picks_fastest_admitted_candidate_and_caches(tmp_path):
    sizes = [6000, 10000]
    parts = [inputs.gaussian_cloud(s, 1.0, 1e-3, 1e-5, 40 + k) for k, s in enumerate(sizes)]
    xn = np.concatenate([p.x for p in parts])
    qn = np.concatenate([p.q for p in parts])
    x = torch.from_numpy(xn).cuda()
    q = torch.from_numpy(qn).cuda()
    offs = torch.tensor([0, sizes[0], sum(sizes)], dtype=torch.int64, device="cuda")
    cache = str(tmp_path / "tune.json")
    cand = {"group_size": (32, 64), "list_len": (64, 128), "group_mode": (L.UCP_GROUP_CHUNK,),
            "leaf_cap": (24,)}
    r = autotune.tune(x, q, offs, theta=0.5, eps=0.01, candidates=cand, reps=2, cache_path=cache)
    say(f"[autotune] chose G={r['group_size']} L={r['list_len']} error vs direct "
        f"{r['rel_force_err_vs_direct']:.3e} (bound {r['err_bound']:.3e}, per-particle walk "
        f"{r['per_particle_walk_err_vs_direct']:.3e})")
    assert not r["cached"]
    assert len(r["candidates"]) == 4
    ok = [c for c in r["candidates"] if c["admitted"]]
    assert ok and r["walk_ms"] == min(c["walk_ms"] for c in ok)
    assert all(c["admitted"] == (c["rel_force_err_vs_direct"] <= r["err_bound"])
               for c in r["candidates"])
    assert (r["group_size"], r["list_len"]) in [(G, Lq) for G in (32, 64) for Lq in (64, 128)]
    # the tuner's direct-sum reference is the direct sum: check the errors it
    # reports against the oracle's direct sum of each cloud
    ref = np.concatenate([oracle.direct(p.x, p.q, 0.01)[0] for p in parts])
    ts = TreeSolver(sum(sizes), 2, theta=0.5, eps=0.01, group_size=r["group_size"],
                    list_len=r["list_len"], group_mode=r["group_mode"], leaf_cap=r["leaf_cap"])
    f = ts.tree_forces(x, q, offs).cpu().numpy()
    ts.stats()
    ts.close()
    e = relrms(f, ref)
    assert abs(e - r["rel_force_err_vs_direct"]) <= 1e-6 * e + 1e-9
    assert 0.0 < r["per_particle_walk_err_vs_direct"] < 1e-2
    r2 = autotune.tune(x, q, offs, theta=0.5, eps=0.01, candidates=cand, cache_path=cache)
    assert r2["cached"] and r2["group_size"] == r["group_size"] and r2["list_len"] == r["list_len"]
