"""Autotuner for the walk's group size G, list length L, group rule and leaf
capacity.

G, the group rule and the leaf capacity decide which targets share one
traversal and where the near field starts, so they change the accepted sets
(and the force error at truncation level), not only the speed; L changes only
the FP64 summation order.  The tuner therefore times the walk for every
candidate on the caller's own workload and measures every candidate's force
error against the direct sum of Eq. (1)-(2) on the same input (the
library's FP64 evaluation at theta = 0, where no box is accepted).  A
candidate is admitted only if its error does not exceed the error of the
per-particle walk over a tree of single-particle leaves (G = 1, leaf capacity
1: the tree and walk of Sec. 3) at the same theta, times `err_factor`; the
fastest admitted candidate is chosen.

Timing uses the library's own HIP events around each walk launch
(ucp_set_timing / ucp_timing_read).  Results are cached in a JSON file keyed by
device, particle count, cloud count, theta, eps and precision.
"""
from __future__ import annotations

import json
import os

import torch

from . import _lib as L
from .tree import TreeSolver

DEFAULT_CANDIDATES = {
    "group_size": (32, 48, 64),
    "list_len": (64, 128, 256),
    "group_mode": (L.UCP_GROUP_CHUNK, L.UCP_GROUP_NODE),
    "leaf_cap": (8, 16, 24, 32),
}


def default_cache_path():
    return os.environ.get("UCP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ucptree", "tune.json"))


def _key(n, clouds, theta, eps, precision):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return f"{dev}|n={n}|clouds={clouds}|theta={theta:g}|eps={eps:g}|precision={precision}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def _time_walk(x, q, offsets, reps, **params):
    """Walk time per launch, interactions per particle and the forces."""
    n = x.shape[0]
    clouds = 1 if offsets is None else offsets.numel() - 1
    ts = TreeSolver(n, clouds, **params)
    try:
        f = ts.tree_forces(x, q, offsets)      # warm-up (and graph-free first build)
        ts.stats()
        ts.timing(True)
        torch.cuda.synchronize()
        for _ in range(reps):
            ts.tree_forces(x, q, offsets)
        torch.cuda.synchronize()
        ms, cnt = ts.timing_read()
        st = ts.stats()
        ts.timing(False)
    finally:
        ts.close()
    return ms / max(cnt, 1), (st["p2p"] + st["m2p"]) / max(n, 1), f


def _forces(x, q, offsets, **params):
    n = x.shape[0]
    clouds = 1 if offsets is None else offsets.numel() - 1
    ts = TreeSolver(n, clouds, **params)
    try:
        f = ts.tree_forces(x, q, offsets)
        ts.stats()
    finally:
        ts.close()
    return f


def tune(x, q, offsets=None, *, theta, eps, precision=L.UCP_SPLIT, candidates=None, reps=3,
         cache_path=None, use_cache=True, err_factor=1.0):
    """Pick (group_size, list_len, group_mode, leaf_cap) for this workload.

    x, q: float64 GPU tensors ((N, 3), (N,)); offsets: int64 GPU tensor of
    cloud offsets or None.  Every candidate is timed and its relative RMS
    force error against the FP64 direct sum is measured; candidates whose
    error exceeds err_factor times that of the FP64 per-particle walk (G = 1,
    leaf capacity 1) are rejected, and the fastest of the others is chosen.
    Returns the chosen parameters, its walk time and error, the reference
    errors and bound, and every candidate's row."""
    n = x.shape[0]
    clouds = 1 if offsets is None else offsets.numel() - 1
    path = cache_path or default_cache_path()
    key = _key(n, clouds, theta, eps, precision)
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        return dict(cache[key], cached=True)
    cand = dict(DEFAULT_CANDIDATES)
    cand.update(candidates or {})
    # references: the direct sum (theta = 0 accepts no box) and the paper's
    # per-particle walk at this theta, both FP64
    fd = _forces(x, q, offsets, theta=0.0, eps=eps, precision=L.UCP_FP64)
    fpp = _forces(x, q, offsets, theta=theta, eps=eps, precision=L.UCP_FP64, group_size=1,
                  group_mode=L.UCP_GROUP_CHUNK, leaf_cap=1)
    err_pp = _rel(fpp, fd)
    bound = err_factor * err_pp
    rows = []
    for lc in cand["leaf_cap"]:
        for gm in cand["group_mode"]:
            for G in cand["group_size"]:
                for Lq in cand["list_len"]:
                    ms, ipp, f = _time_walk(x, q, offsets, reps, theta=theta, eps=eps,
                                            precision=precision, group_size=G, list_len=Lq,
                                            group_mode=gm, leaf_cap=lc)
                    err = _rel(f, fd)
                    rows.append({"group_size": G, "list_len": Lq, "group_mode": gm,
                                 "leaf_cap": lc, "walk_ms": ms,
                                 "interactions_per_particle": ipp,
                                 "rel_force_err_vs_direct": err,
                                 "rel_force_diff_vs_per_particle_fp64": _rel(f, fpp),
                                 "admitted": err <= bound})
                    del f
    ok = [r for r in rows if r["admitted"]]
    if not ok:
        raise RuntimeError(f"autotune: no candidate within {bound:.3e} of the direct sum")
    best = min(ok, key=lambda r: r["walk_ms"])
    out = {"group_size": best["group_size"], "list_len": best["list_len"],
           "group_mode": best["group_mode"], "leaf_cap": best["leaf_cap"],
           "walk_ms": best["walk_ms"],
           "rel_force_err_vs_direct": best["rel_force_err_vs_direct"],
           "rel_force_diff_vs_per_particle_fp64": best["rel_force_diff_vs_per_particle_fp64"],
           "per_particle_walk_err_vs_direct": err_pp, "err_bound": bound,
           "candidates": rows}
    if use_cache:
        cache = _load(path)
        cache[key] = out
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    return dict(out, cached=False)
