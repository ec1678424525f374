"""Seeded synthetic plasma clouds (numpy PCG64), shared by the tests, the
benchmark and the smoke check.

This module only draws random numbers: it holds none of the force, tree or
integrator arithmetic.  Units are reduced (e^2/4 pi eps0 = 1, k_B = 1).  Ions
occupy indices [0, N/2) with q = +1, m = 1; electrons [N/2, N) with q = -1,
m = 1/1836.  The clouds stand in for the paper's simulated ultracold plasmas
(Sec. 5): spherical, roughly symmetric, radially non-uniform (Sec. 4.1).

Draw order for every cloud: positions (N, 3) standard normal x sigma; then,
if present, halo radii and halo directions; then velocities (N, 3) standard
normal x sqrt(T/m) per species.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

M_ELECTRON = 1.0 / 1836.0


@dataclass
class Cloud:
    x: np.ndarray            # (N, 3) float64
    v: np.ndarray            # (N, 3) float64
    q: np.ndarray            # (N,) float64
    m: np.ndarray            # (N,) float64
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[0]


def _species(n_ion: int, n_el: int):
    q = np.concatenate([np.ones(n_ion), -np.ones(n_el)])
    m = np.concatenate([np.ones(n_ion), np.full(n_el, M_ELECTRON)])
    return q, m


def gaussian_cloud(n: int, sigma: float = 1.0, t_e: float = 1e-3, t_i: float = 1e-5,
                   seed: int = 0, halo_frac: float = 0.0, halo_r: tuple = (2.0, 3.0),
                   hot_frac: float = 0.0, t_hot: float = 1e-2) -> Cloud:
    """Two-component Gaussian cloud of n particles (n even: n/2 ions, n/2 electrons).

    halo_frac: per species, round(halo_frac * n/2) particles are moved to a
    shell [halo_r[0] sigma, halo_r[1] sigma], uniform in volume (the last ones
    of each species block).
    hot_frac: the first round(hot_frac * n/2) electrons get temperature t_hot.
    """
    if n % 2:
        raise ValueError("n must be even (equal ions and electrons)")
    rng = np.random.default_rng(seed)
    ns = n // 2
    x = rng.standard_normal((n, 3)) * sigma
    nh = int(round(halo_frac * ns))
    if nh > 0:
        r0, r1 = halo_r[0] * sigma, halo_r[1] * sigma
        u = rng.random(2 * nh)
        rad = np.cbrt(r0 ** 3 + u * (r1 ** 3 - r0 ** 3))
        d = rng.standard_normal((2 * nh, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        idx = np.concatenate([np.arange(ns - nh, ns), np.arange(n - nh, n)])
        x[idx] = d * rad[:, None]
    q, m = _species(ns, ns)
    temp = np.where(q > 0, t_i, t_e)
    nhot = int(round(hot_frac * ns))
    if nhot > 0:
        temp[ns:ns + nhot] = t_hot
    v = rng.standard_normal((n, 3)) * np.sqrt(temp / m)[:, None]
    meta = dict(kind="gaussian", n=n, sigma=sigma, t_e=t_e, t_i=t_i, seed=seed,
                halo_frac=halo_frac, halo_r=halo_r, hot_frac=hot_frac, t_hot=t_hot)
    return Cloud(x, v, q, m, meta)


# Workloads.  Each returns a Cloud plus the method parameters it is run with.
def small(seed: int = 0):
    """N = 4096 Gaussian cloud, sigma = 1, eps = 0.01, theta = 0.5, dt = 1e-4."""
    c = gaussian_cloud(4096, 1.0, 1e-3, 1e-5, seed)
    return c, dict(theta=0.5, eps=0.01, dt=1e-4, steps=100)


def metric(seed: int = 0):
    """N = 524,288: per species 249,037 Gaussian (sigma = 1) + 13,107 in a halo
    shell [2, 3] sigma; eps = 0.005, theta = 0.5, dt = 5e-5."""
    c = gaussian_cloud(524288, 1.0, 1e-3, 1e-5, seed, halo_frac=13107 / 262144)
    return c, dict(theta=0.5, eps=0.005, dt=5e-5, steps=1000)


def large(seed: int = 0):
    """N = 4,194,304 Gaussian cloud with 10% of electrons hot (T = 1e-2);
    eps = 0.002, theta = 0.5, dt = 5e-5."""
    c = gaussian_cloud(4194304, 1.0, 1e-3, 1e-5, seed, hot_frac=0.1, t_hot=1e-2)
    return c, dict(theta=0.5, eps=0.002, dt=5e-5, steps=50)


def adjoint(seed: int = 0):
    """N = 65,536 Gaussian cloud for rollout differentiation; theta = 0.5,
    eps = 0.01, dt = 1e-4, 200 steps, checkpoint every 20."""
    c = gaussian_cloud(65536, 1.0, 1e-3, 1e-5, seed)
    return c, dict(theta=0.5, eps=0.01, dt=1e-4, steps=200, ckpt=20)


def ensemble_sizes(clouds: int = 64, seed: int = 0, lo: int = 4096, hi: int = 65536):
    """Per-cloud N_c = 2 * U_int[lo, hi] and sigma_c = U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    ns, sig = [], []
    for _ in range(clouds):
        ns.append(2 * int(rng.integers(lo, hi, endpoint=True)))
        sig.append(float(rng.uniform(0.5, 2.0)))
    return ns, sig


def ensemble(clouds: int = 64, seed: int = 0, lo: int = 4096, hi: int = 65536):
    """Concatenated independent clouds; cloud c is drawn with seed 1000 + c.
    Returns (Cloud with all particles, offsets int64[clouds+1], params)."""
    ns, sig = ensemble_sizes(clouds, seed, lo, hi)
    parts = [gaussian_cloud(n, s, 1e-3, 1e-5, 1000 + c) for c, (n, s) in enumerate(zip(ns, sig))]
    x = np.concatenate([p.x for p in parts])
    v = np.concatenate([p.v for p in parts])
    q = np.concatenate([p.q for p in parts])
    m = np.concatenate([p.m for p in parts])
    off = np.zeros(clouds + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)
    meta = dict(kind="ensemble", clouds=clouds, sizes=ns, sigmas=sig, seed=seed)
    return Cloud(x, v, q, m, meta), off, dict(theta=0.5, eps=0.01, dt=1e-4, steps=200)
