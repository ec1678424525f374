"""Torch-facing convenience layer over the C-ABI (marshalling only).

``TreeSolver`` owns one library context.  Tensors are CUDA (HIP) float64,
contiguous; positions/velocities/forces are (n, 3).  All work is enqueued on
torch's current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _chk(t, shape_tail, name):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    if tuple(t.shape[1:]) != shape_tail:
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    return t


class TreeSolver:
    """One TREE context: build, forces, Verlet steps, energies, stats."""

    def __init__(self, n_max, clouds_max=1, **params):
        self.params = L.default_params(**params)
        self.h = L.ucp_create(int(n_max), int(clouds_max), self.params)
        self.n_max = n_max

    def close(self):
        if getattr(self, "h", None):
            L.ucp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **params):
        for k, v in params.items():
            setattr(self.params, k, v)
        L.ucp_set_params(self.h, self.params)

    # -- the method
    def build(self, x, q, offsets=None):
        _chk(x, (3,), "x")
        if offsets is None:
            L.ucp_build_tree(self.h, _ptr(x), _ptr(q), x.shape[0], _stream())
        else:
            L.ucp_build_tree_batched(self.h, _ptr(x), _ptr(q), _ptr(offsets), offsets.numel() - 1,
                                     x.shape[0], _stream())

    def forces(self, n, want_phi=False, device="cuda"):
        f = torch.empty((n, 3), dtype=torch.float64, device=device)
        phi = torch.empty(n, dtype=torch.float64, device=device) if want_phi else None
        L.ucp_compute_forces(self.h, _ptr(f), _ptr(phi), _stream())
        return (f, phi) if want_phi else f

    def tree_forces(self, x, q, offsets=None, want_phi=False):
        self.build(x, q, offsets)
        return self.forces(x.shape[0], want_phi, x.device)

    def step(self, x, v, f, q, m, dt, nsteps, offsets=None):
        if offsets is None:
            L.ucp_step(self.h, _ptr(x), _ptr(v), _ptr(f), _ptr(q), _ptr(m), x.shape[0], dt, nsteps,
                       _stream())
        else:
            L.ucp_step_batched(self.h, _ptr(x), _ptr(v), _ptr(f), _ptr(q), _ptr(m), _ptr(offsets),
                               offsets.numel() - 1, x.shape[0], dt, nsteps, _stream())

    def energy(self, x, v, q, m):
        out = torch.zeros(5, dtype=torch.float64, device=x.device)
        L.ucp_energy(self.h, _ptr(x), _ptr(v), _ptr(q), _ptr(m), x.shape[0], _ptr(out), _stream())
        return out

    def vjp(self, u, noalloc=False):
        """(dF/dx)^T u of the last build; noalloc=True uses the library's
        static adjoint scratch (ucp_force_vjp_noalloc) instead of buffers
        allocated by the first call."""
        xb = torch.empty_like(u)
        fn = L.ucp_force_vjp_noalloc if noalloc else L.ucp_force_vjp
        fn(self.h, _ptr(u), _ptr(xb), _stream())
        return xb

    def stats(self, raise_on_flag=True):
        st, rc = L.ucp_get_stats(self.h, _stream(), raise_on_flag)
        return {k: getattr(st, k) for k, _ in L.ucp_stats._fields_} | {"status": rc}

    def check(self):
        """Raise UcpError if the device flagged a problem in any build, walk
        or adjoint since the last check (synchronises the stream)."""
        self.stats(raise_on_flag=True)

    def timing(self, on=True):
        L.ucp_set_timing(self.h, on)

    def timing_read(self):
        return L.ucp_timing_read(self.h)

    def wave_clock(self, units=False):
        """Start and end (microseconds, from the first start) of every wave of
        the last force walk launched with timing on: array [waves, 2].  With
        units=True also the compute unit each wave ran on, as one integer per
        wave (XCD * 256 + bits 8-15 of the wave's HW_ID: CU, shader array and
        shader engine)."""
        cu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        w = self.params.walk_waves if self.params.walk_waves > 0 else 32
        waves = 4 * ((cu * w + 3) // 4)
        out = np.zeros((waves, 3), dtype=np.uint64)
        L.ucp_debug_copy(self.h, 8, out.ctypes.data_as(C.c_void_p), out.nbytes, _stream())
        t = out[:, :2].astype(np.float64) / 100.0   # 100 MHz real-time counter
        t = t - t[:, 0].min()
        if not units:
            return t
        ids = out[:, 2]
        unit = ((ids >> np.uint64(32)) & np.uint64(0xF)) * np.uint64(256) + \
            ((ids >> np.uint64(8)) & np.uint64(0xFF))
        return t, unit.astype(np.int64)

    # -- introspection (host numpy arrays)
    def debug(self, which):
        st = self.stats(raise_on_flag=False)
        n, nodes, groups, clouds = st["n"], st["nodes"], st["groups"], st["clouds"]
        spec = {"keys": (0, np.uint64, (n,)), "perm": (1, np.uint32, (n,)),
                "ninfo": (2, np.int32, (nodes, 4)), "ngeo": (3, np.float64, (nodes, 4)),
                "moments": (4, np.float64, (nodes, 10)), "groups": (5, np.int32, (groups, 4)),
                "gstat": (6, np.int32, (groups, 2)), "cube": (7, np.float64, (clouds, 4))}
        w, dt, shape = spec[which]
        out = np.zeros(shape, dtype=dt)
        if out.nbytes:
            L.ucp_debug_copy(self.h, w, out.ctypes.data_as(C.c_void_p), out.nbytes, _stream())
        return out
