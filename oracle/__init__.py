"""FP64 CPU oracle for the two-component plasma TREE force evaluation.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the GPU path.  Each wrapper below names the part of the method it
follows; the arithmetic lives in ``ucp_oracle.c``.

Arrays are numpy, C-contiguous: positions/velocities/forces are (n, 3) float64
in the caller's particle order; charges and masses are (n,) float64.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libucp_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIBPATH)
    i64, i32, dbl, vp = C.c_int64, C.c_int, C.c_double, C.c_void_p
    sig = {
        "orc_version": (i32, []),
        "orc_max_threads": (i32, []),
        "orc_set_threads": (None, [i32]),
        "orc_direct": (None, [i64, _dp, _dp, dbl, _dp, vp]),
        "orc_direct_pair": (i32, [i64, _dp, _dp, dbl, i32, dbl, _dp, vp]),
        "orc_tree_set_pair": (i32, [vp, i32, dbl]),
        "orc_tree_set_expansion": (i32, [vp, i32]),
        "orc_direct_targets": (None, [i64, _dp, _dp, dbl, i64, _i64p, _dp, vp]),
        "orc_direct_vjp": (None, [i64, _dp, _dp, dbl, _dp, _dp]),
        "orc_cube": (i32, [i64, _dp, _dp, C.POINTER(C.c_int)]),
        "orc_keys": (None, [i64, _dp, _dp, i32, i32, i32, _u64p]),
        "orc_sort": (None, [i64, _u64p, _i64p]),
        "orc_tree_new": (vp, [i64, _dp, _dp, dbl, dbl, i32, i32, i32, i32, i32, i32]),
        "orc_tree_free": (None, [vp]),
        "orc_tree_nnodes": (i64, [vp]),
        "orc_tree_ngroups": (i64, [vp]),
        "orc_tree_cube": (None, [vp, _dp, C.POINTER(C.c_int)]),
        "orc_tree_perm": (None, [vp, _i64p]),
        "orc_tree_sorted_keys": (None, [vp, _u64p]),
        "orc_tree_nodes": (None, [vp, _i32p, _i64p, _i64p, _i64p]),
        "orc_tree_centres": (None, [vp, _dp]),
        "orc_tree_groups": (None, [vp, _i64p, _i64p, _i64p]),
        "orc_tree_moments": (None, [vp, _dp, _dp, _dp]),
        "orc_tree_eval": (None, [vp, _dp, _dp, _dp, vp, vp, vp, vp, vp]),
        "orc_tree_vjp": (i32, [vp, _dp, _dp, _dp, _dp, vp, vp]),
        "orc_tree_eval_groups": (i32, [vp, _dp, _dp, i64, _i64p, _dp, vp, vp, vp, vp]),
        "orc_tree_arch_series": (i64, [vp, _i64p]),
        "orc_rebuild": (i64, [i64, _i64p, i64, _i64p, _i64p]),
        "orc_verlet": (i32, [i64, _dp, _dp, _dp, _dp, i32, dbl, dbl, i32, i32, i32, i32, i32,
                             dbl, i32, _dp, i32]),
        "orc_energy": (None, [i64, _dp, _dp, _dp, _dp, _dp]),
        "orc_cell_eval": (None, [_dp, _dp, dbl, _dp, _dp]),
        "orc_cell_jacobian": (None, [_dp, _dp, dbl, _dp]),
        "orc_tree_lists": (i32, [vp, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64), vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


# --------------------------------------------------------------------------
# C-1 direct sum: Eq. (1)-(2) in reduced units with Plummer softening.
# --------------------------------------------------------------------------
def direct(x, q, eps):
    """Direct-sum forces F (n,3) and potentials phi (n,) [self pair excluded]."""
    x = _f64(x, (-1, 3)); q = _f64(q)
    n = x.shape[0]
    f = np.zeros((n, 3)); phi = np.zeros(n)
    _load().orc_direct(n, x, q, float(eps), f, _ptr(phi))
    return f, phi


PAIR_PLUMMER, PAIR_KELBG = 0, 1
EXP_QUADRUPOLE, EXP_SPECIES = 0, 1
CURVE_MORTON, CURVE_HILBERT = 0, 1


def direct_pair(x, q, eps, pair_law=PAIR_PLUMMER, lambda_ei=0.0):
    """Direct-sum F and phi under a pair law (Sec. 2.1): PAIR_PLUMMER applies the
    softened Coulomb law to every pair; PAIR_KELBG applies the modified law of
    Eq. (3) with length lambda_ei to electron-ion pairs and the softened
    Coulomb law (eps = 0: bare) to like pairs."""
    x = _f64(x, (-1, 3)); q = _f64(q)
    n = x.shape[0]
    f = np.zeros((n, 3)); phi = np.zeros(n)
    if _load().orc_direct_pair(n, x, q, float(eps), int(pair_law), float(lambda_ei), f,
                               _ptr(phi)) != 0:
        raise ValueError("oracle direct_pair: invalid pair law")
    return f, phi


def direct_targets(x, q, eps, targets):
    """Direct-sum F and phi for the particles listed in ``targets`` only."""
    x = _f64(x, (-1, 3)); q = _f64(q)
    t = np.ascontiguousarray(targets, dtype=np.int64)
    f = np.zeros((t.size, 3)); phi = np.zeros(t.size)
    _load().orc_direct_targets(x.shape[0], x, q, float(eps), t.size, t, f, _ptr(phi))
    return f, phi


def direct_vjp(x, q, eps, u):
    """(dF/dx)^T u of the direct-sum force map (minus the Hessian of U times u)."""
    x = _f64(x, (-1, 3)); q = _f64(q); u = _f64(u, (-1, 3))
    xb = np.zeros_like(x)
    _load().orc_direct_vjp(x.shape[0], x, q, float(eps), u, xb)
    return xb


# --------------------------------------------------------------------------
# C-2 tree pieces.
# --------------------------------------------------------------------------
def cube(x):
    """Enclosing cube: (lo[3], e) with side 2**e (Sec. 3)."""
    x = _f64(x, (-1, 3))
    lo = np.zeros(3); e = C.c_int(0)
    rc = _load().orc_cube(x.shape[0], x, lo, C.byref(e))
    if rc != 0:
        raise ValueError("cube: empty or non-finite input")
    return lo, e.value


def keys(x, lo, e, b, curve=CURVE_MORTON):
    """Keys for key depth b (10 or 21): Morton (per-bit interleave, x-major) or
    Hilbert (Skilling's transform, then the same interleave)."""
    x = _f64(x, (-1, 3))
    k = np.zeros(x.shape[0], dtype=np.uint64)
    _load().orc_keys(x.shape[0], x, _f64(lo), int(e), int(b), int(curve), k)
    return k


def stable_order(key):
    """Stable ordering of particles by key (ties: ascending index)."""
    key = np.ascontiguousarray(key, dtype=np.uint64)
    p = np.zeros(key.size, dtype=np.int64)
    _load().orc_sort(key.size, key, p)
    return p


class Tree:
    """Oracle Barnes-Hut tree (C-2): cube, keys, recursive preorder build,
    centres, walk groups and (optionally) frozen interaction lists.

    group_mode 0: node groups (a node of at most G particles whose parent holds
    more); group_mode 1: consecutive runs of G key-sorted particles.  curve:
    the order of the keys (CURVE_MORTON or CURVE_HILBERT); it changes the
    order of the boxes and of the particles, not the boxes themselves."""

    def __init__(self, x, q, theta, eps, b=21, leaf_cap=24, G=64, keep_lists=False, group_mode=1,
                 pair_law=PAIR_PLUMMER, lambda_ei=0.0, expansion=EXP_QUADRUPOLE,
                 curve=CURVE_HILBERT):
        lib = _load()
        self.x = _f64(x, (-1, 3)); self.q = _f64(q)
        self.n = self.x.shape[0]
        self.theta, self.eps, self.b, self.leaf_cap, self.G = theta, eps, b, leaf_cap, G
        self.group_mode, self.curve = group_mode, curve
        h = lib.orc_tree_new(self.n, self.x, self.q, float(theta), float(eps), int(b),
                             int(leaf_cap), int(G), int(group_mode), int(bool(keep_lists)),
                             int(curve))
        if not h:
            raise ValueError("oracle tree: invalid parameters or non-finite input")
        self._h = h
        self.keep_lists = keep_lists
        self.pair_law, self.lambda_ei = pair_law, lambda_ei
        if lib.orc_tree_set_pair(h, int(pair_law), float(lambda_ei)) != 0:
            raise ValueError("oracle tree: invalid pair law")
        self.expansion = expansion
        if lib.orc_tree_set_expansion(h, int(expansion)) != 0:
            raise ValueError("oracle tree: invalid expansion (species pseudo-particles do not "
                             "keep lists)")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_tree_free(h)
            self._h = None

    @property
    def nnodes(self):
        return int(_lib.orc_tree_nnodes(self._h))

    @property
    def ngroups(self):
        return int(_lib.orc_tree_ngroups(self._h))

    def cube(self):
        lo = np.zeros(3); e = C.c_int(0)
        _lib.orc_tree_cube(self._h, lo, C.byref(e))
        return lo, e.value

    def perm(self):
        p = np.zeros(self.n, dtype=np.int64)
        _lib.orc_tree_perm(self._h, p)
        return p

    def sorted_keys(self):
        k = np.zeros(self.n, dtype=np.uint64)
        _lib.orc_tree_sorted_keys(self._h, k)
        return k

    def nodes(self):
        """(level, first, count, skip) of every node, preorder."""
        M = self.nnodes
        lv = np.zeros(M, dtype=np.int32)
        fi, co, sk = (np.zeros(M, dtype=np.int64) for _ in range(3))
        _lib.orc_tree_nodes(self._h, lv, fi, co, sk)
        return lv, fi, co, sk

    def centres(self):
        c = np.zeros((self.nnodes, 3))
        _lib.orc_tree_centres(self._h, c)
        return c

    def groups(self):
        ng = self.ngroups
        fi, co, nd = (np.zeros(ng, dtype=np.int64) for _ in range(3))
        _lib.orc_tree_groups(self._h, fi, co, nd)
        return fi, co, nd

    def moments(self, x=None):
        """(M, 10): Q, p[3], Sxx, Syy, Szz, Sxy, Sxz, Syz about each centre."""
        x = self.x if x is None else _f64(x, (-1, 3))
        m = np.zeros((self.nnodes, 10))
        _lib.orc_tree_moments(self._h, x, self.q, m)
        return m

    def eval(self, x=None, want_phi=True, group_counts=False, cond=False):
        """Tree forces (C-2.8).  Returns dict f, phi, p2p, m2p[, gm2p, gp2p]
        [, cond].  cond: per particle the size A_i of the terms its field is
        summed from, so that an evaluation in a precision of unit roundoff u_w
        errs by a small multiple of u_w A_i in E_i (and |q_i| u_w A_i in F_i)."""
        x = self.x if x is None else _f64(x, (-1, 3))
        f = np.zeros((self.n, 3))
        phi = np.zeros(self.n) if want_phi else None
        st = np.zeros(2, dtype=np.int64)
        gm = gp = None
        if group_counts:
            gm = np.zeros(self.ngroups, dtype=np.int64)
            gp = np.zeros(self.ngroups, dtype=np.int64)
        cd = np.zeros(self.n) if cond else None
        _lib.orc_tree_eval(self._h, x, self.q, f, _ptr(phi), _ptr(st), _ptr(gm), _ptr(gp), _ptr(cd))
        out = {"f": f, "phi": phi, "p2p": int(st[0]), "m2p": int(st[1])}
        if group_counts:
            out["gm2p"], out["gp2p"] = gm, gp
        if cond:
            out["cond"] = cd
        return out

    def eval_groups(self, gsel, x=None, want_phi=False, cond=False):
        """Tree forces of the members of the selected groups only.  Returns
        dict f, phi (caller order; rows of other particles are NaN) and the
        per-selected-group list lengths gm2p, gp2p [, cond as in eval]."""
        x = self.x if x is None else _f64(x, (-1, 3))
        gsel = np.ascontiguousarray(gsel, dtype=np.int64)
        f = np.full((self.n, 3), np.nan)
        phi = np.full(self.n, np.nan) if want_phi else None
        gm = np.zeros(gsel.size, dtype=np.int64)
        gp = np.zeros(gsel.size, dtype=np.int64)
        cd = np.full(self.n, np.nan) if cond else None
        if _lib.orc_tree_eval_groups(self._h, x, self.q, gsel.size, gsel, f, _ptr(phi), _ptr(gm),
                                     _ptr(gp), _ptr(cd)) != 0:
            raise ValueError("group index out of range")
        out = {"f": f, "phi": phi, "gm2p": gm, "gp2p": gp}
        if cond:
            out["cond"] = cd
        return out

    def vjp(self, u, x=None, extras=False):
        """(dF/dx)^T u with the lists of the build held fixed and the cube
        origin's dependence on the minimum particles included; needs
        keep_lists=True.  extras=True returns (xbar, cond, lobar): cond the
        per-particle term sizes B_j, lobar the cube-origin cotangent (xyz),
        the size of its terms and the size of the chain-rule terms this oracle
        sums to get it (its own rounding scales with the latter)."""
        x = self.x if x is None else _f64(x, (-1, 3))
        u = _f64(u, (-1, 3))
        xb = np.zeros_like(x)
        cd = np.zeros(self.n) if extras else None
        lob = np.zeros(5)
        if _lib.orc_tree_vjp(self._h, x, self.q, u, xb, _ptr(lob), _ptr(cd)) != 0:
            raise ValueError("tree vjp needs keep_lists=True and the Plummer pair law")
        return (xb, cd, lob) if extras else xb

    def lists(self, g):
        """Frozen lists of group g: (accepted cells, opened leaves); keep_lists only."""
        nm, np_ = C.c_int64(0), C.c_int64(0)
        if _lib.orc_tree_lists(self._h, int(g), C.byref(nm), C.byref(np_), None, None) != 0:
            raise ValueError("lists need keep_lists=True and a valid group")
        mo = np.zeros(max(nm.value, 1), dtype=np.int64)
        po = np.zeros(max(np_.value, 1), dtype=np.int64)
        _lib.orc_tree_lists(self._h, int(g), C.byref(nm), C.byref(np_), _ptr(mo), _ptr(po))
        return mo[:nm.value], po[:np_.value]

    def arch_series(self):
        """Architecture series of Sec. 4.3 (node number = preorder index + 1)."""
        out = np.zeros(2 * max(self.nnodes, 1), dtype=np.int64)
        L = _lib.orc_tree_arch_series(self._h, out)
        return out[:L]


def cell_eval(mom, r, eps):
    """C-2.7 expansion of one cell (mom: Q, p[3], Sxx, Syy, Szz, Sxy, Sxz, Syz)
    at offset r = x - c: returns (E[3], phi)."""
    E = np.zeros(3); ph = np.zeros(1)
    _load().orc_cell_eval(_f64(mom), _f64(r), float(eps), E, ph)
    return E, float(ph[0])


def cell_jacobian(mom, r, eps):
    """dE/dr of the C-2.7 expansion (3x3)."""
    J = np.zeros(9)
    _load().orc_cell_jacobian(_f64(mom), _f64(r), float(eps), J)
    return J.reshape(3, 3)


def rebuild(series, cap):
    """Decode an architecture series: (parent, nchild) per node number."""
    s = np.ascontiguousarray(series, dtype=np.int64)
    par = np.full(cap, -7, dtype=np.int64); nch = np.zeros(cap, dtype=np.int64)
    m = _load().orc_rebuild(s.size, s, int(cap), par, nch)
    if m < 0:
        raise ValueError("malformed architecture series")
    return par[:m], nch[:m]


def tree_forces(x, q, theta, eps, b=21, leaf_cap=24, G=64, want_phi=True, group_mode=1,
                pair_law=PAIR_PLUMMER, lambda_ei=0.0, expansion=EXP_QUADRUPOLE,
                curve=CURVE_HILBERT):
    """Convenience: build the oracle tree and evaluate it."""
    t = Tree(x, q, theta, eps, b, leaf_cap, G, group_mode=group_mode, pair_law=pair_law,
             lambda_ei=lambda_ei, expansion=expansion, curve=curve)
    r = t.eval(want_phi=want_phi)
    r["nodes"] = t.nnodes
    r["groups"] = t.ngroups
    return r


# --------------------------------------------------------------------------
# C-3 Verlet and energies.
# --------------------------------------------------------------------------
def verlet(x, v, q, m, dt, nsteps, eps, mode="direct", theta=0.5, b=21, leaf_cap=24, G=64,
           f=None, group_mode=1, curve=CURVE_HILBERT):
    """KDK velocity Verlet; returns (x, v, f) after nsteps (copies)."""
    x = _f64(x, (-1, 3)).copy(); v = _f64(v, (-1, 3)).copy()
    q = _f64(q); m = _f64(m)
    fv = 1 if f is not None else 0
    f = np.zeros_like(x) if f is None else _f64(f, (-1, 3)).copy()
    rc = _load().orc_verlet(x.shape[0], x, v, q, m, 0 if mode == "direct" else 1, float(theta),
                            float(eps), int(b), int(leaf_cap), int(G), int(group_mode), int(curve),
                            float(dt),
                            int(nsteps), f, fv)
    if rc != 0:
        raise ValueError("verlet failed")
    return x, v, f


def energy(v, q, m, phi):
    """(K, U, E, K_ion, K_electron) from velocities and potentials."""
    v = _f64(v, (-1, 3))
    out = np.zeros(5)
    _load().orc_energy(v.shape[0], v, _f64(q), _f64(m), _f64(phi), out)
    return out
