"""ctypes binding of libucptree.so -- the C-ABI of include/ucp.h, same names.

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Loading fails loudly when the library has not been
built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("UCP_LIBPATH") or os.path.join(_HERE, "libucptree.so")

UCP_OK, UCP_EINVAL, UCP_ENOMEM, UCP_EHIP, UCP_ECAPACITY, UCP_ENOTBUILT, UCP_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6
UCP_FP64, UCP_SPLIT = 0, 1
UCP_GROUP_NODE, UCP_GROUP_CHUNK = 0, 1
UCP_PAIR_PLUMMER, UCP_PAIR_KELBG = 0, 1
UCP_EXPANSION_QUADRUPOLE, UCP_EXPANSION_SPECIES = 0, 1
UCP_CURVE_MORTON, UCP_CURVE_HILBERT = 0, 1
UCP_FLAG_NODE_OVERFLOW, UCP_FLAG_NONFINITE, UCP_FLAG_BAD_OFFSETS, UCP_FLAG_BAD_CUBE = 1, 2, 4, 8
UCP_FLAG_INTERNAL, UCP_FLAG_WALK_STACK = 16, 32
STATUS_NAMES = {0: "UCP_OK", -1: "UCP_EINVAL", -2: "UCP_ENOMEM", -3: "UCP_EHIP",
                -4: "UCP_ECAPACITY", -5: "UCP_ENOTBUILT", -6: "UCP_ENONFINITE"}

# the symbols declared in include/ucp.h
EXPORTS = ["ucp_default_params", "ucp_create", "ucp_destroy", "ucp_set_params", "ucp_get_params",
           "ucp_build_tree", "ucp_build_tree_batched", "ucp_compute_forces", "ucp_step",
           "ucp_step_batched", "ucp_energy", "ucp_force_vjp", "ucp_force_vjp_noalloc",
           "ucp_get_stats", "ucp_debug_copy",
           "ucp_set_timing", "ucp_timing_read", "ucp_last_error", "ucp_version"]


class ucp_params(C.Structure):
    _fields_ = [("theta", C.c_double), ("eps", C.c_double), ("key_bits", C.c_int32),
                ("leaf_cap", C.c_int32), ("group_size", C.c_int32), ("list_len", C.c_int32),
                ("precision", C.c_int32), ("walk_waves", C.c_int32), ("group_mode", C.c_int32),
                ("pair_law", C.c_int32), ("lambda_ei", C.c_double), ("expansion", C.c_int32),
                ("curve", C.c_int32)]


class ucp_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("clouds", C.c_int64), ("nodes", C.c_int64),
                ("groups", C.c_int64), ("max_level", C.c_int64), ("p2p", C.c_int64),
                ("m2p", C.c_int64), ("flags", C.c_int64)]


class UcpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libucptree.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build() "
                           "(or python paper_0709_3331_amd/build.py); there is no CPU fallback")
    lib = C.CDLL(LIBPATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pp = C.POINTER(ucp_params)
    sig = {
        "ucp_default_params": (None, [pp]),
        "ucp_create": (i32, [C.POINTER(vp), i64, i32, pp]),
        "ucp_destroy": (None, [vp]),
        "ucp_set_params": (i32, [vp, pp]),
        "ucp_get_params": (i32, [vp, pp]),
        "ucp_build_tree": (i32, [vp, vp, vp, i64, vp]),
        "ucp_build_tree_batched": (i32, [vp, vp, vp, vp, i32, i64, vp]),
        "ucp_compute_forces": (i32, [vp, vp, vp, vp]),
        "ucp_step": (i32, [vp, vp, vp, vp, vp, vp, i64, dbl, i32, vp]),
        "ucp_step_batched": (i32, [vp, vp, vp, vp, vp, vp, vp, i32, i64, dbl, i32, vp]),
        "ucp_energy": (i32, [vp, vp, vp, vp, vp, i64, vp, vp]),
        "ucp_force_vjp": (i32, [vp, vp, vp, vp]),
        "ucp_force_vjp_noalloc": (i32, [vp, vp, vp, vp]),
        "ucp_get_stats": (i32, [vp, C.POINTER(ucp_stats), vp]),
        "ucp_debug_copy": (i32, [vp, i32, vp, i64, vp]),
        "ucp_set_timing": (i32, [vp, i32]),
        "ucp_timing_read": (i32, [vp, C.POINTER(dbl), C.POINTER(i64)]),
        "ucp_last_error": (C.c_char_p, [vp]),
        "ucp_version": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, ctx=None):
    if status != UCP_OK:
        msg = load().ucp_last_error(ctx)
        raise UcpError(status, msg.decode() if msg else "")
    return status


def default_params(**over) -> ucp_params:
    p = ucp_params()
    load().ucp_default_params(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


# --- thin same-name wrappers: pointers are ints (torch .data_ptr()), stream an int
def ucp_create(n_max, clouds_max, params):
    h = C.c_void_p()
    check(load().ucp_create(C.byref(h), int(n_max), int(clouds_max), C.byref(params)))
    return h


def ucp_destroy(h):
    load().ucp_destroy(h)


def ucp_set_params(h, params):
    return check(load().ucp_set_params(h, C.byref(params)), h)


def ucp_get_params(h):
    p = ucp_params()
    check(load().ucp_get_params(h, C.byref(p)), h)
    return p


def ucp_build_tree(h, x, q, n, stream):
    return check(load().ucp_build_tree(h, x, q, int(n), stream), h)


def ucp_build_tree_batched(h, x, q, offsets, clouds, n, stream):
    return check(load().ucp_build_tree_batched(h, x, q, offsets, int(clouds), int(n), stream), h)


def ucp_compute_forces(h, f, phi, stream):
    return check(load().ucp_compute_forces(h, f, phi, stream), h)


def ucp_step(h, x, v, f, q, m, n, dt, nsteps, stream):
    return check(load().ucp_step(h, x, v, f, q, m, int(n), float(dt), int(nsteps), stream), h)


def ucp_step_batched(h, x, v, f, q, m, offsets, clouds, n, dt, nsteps, stream):
    return check(load().ucp_step_batched(h, x, v, f, q, m, offsets, int(clouds), int(n), float(dt),
                                         int(nsteps), stream), h)


def ucp_energy(h, x, v, q, m, n, out, stream):
    return check(load().ucp_energy(h, x, v, q, m, int(n), out, stream), h)


def ucp_force_vjp(h, u, xbar, stream):
    return check(load().ucp_force_vjp(h, u, xbar, stream), h)


def ucp_force_vjp_noalloc(h, u, xbar, stream):
    return check(load().ucp_force_vjp_noalloc(h, u, xbar, stream), h)


def ucp_get_stats(h, stream, raise_on_flag=True):
    st = ucp_stats()
    rc = load().ucp_get_stats(h, C.byref(st), stream)
    if raise_on_flag:
        check(rc, h)
    return st, rc


def ucp_debug_copy(h, which, dst_ptr, nbytes, stream):
    return check(load().ucp_debug_copy(h, int(which), dst_ptr, int(nbytes), stream), h)


def ucp_set_timing(h, on):
    return check(load().ucp_set_timing(h, int(bool(on))), h)


def ucp_timing_read(h):
    ms, cnt = C.c_double(0.0), C.c_int64(0)
    check(load().ucp_timing_read(h, C.byref(ms), C.byref(cnt)), h)
    return ms.value, cnt.value


def ucp_last_error(h=None):
    r = load().ucp_last_error(h)
    return r.decode() if r else ""


def ucp_version():
    return int(load().ucp_version())
