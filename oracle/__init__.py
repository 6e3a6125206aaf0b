"""Oracle for the FMM evaluation pass: plain FP64 CPU code (``fmm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
package.  It shares no code with the HIP path and never calls it; the product
package never imports it.

This module marshals numpy arrays into the C library, where every step of
the method lives (``fmm_oracle.c``; its header names the passages of the
paper each function follows).  One step is written here instead:
:func:`compressed_unit_ops`, the truncated SVD of each far-offset operator
(Sec. 2.1.2), which calls numpy's LAPACK SVD on the C library's dense
operators and keeps the singular values at or above eps times the largest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_pint = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile ``fmm_oracle.c`` into ``liboracle.so`` with gcc (OpenMP, no FP
    contraction).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_direct.argtypes = [_pd, _i64, _pd, _pd, _pd]
    lib.oracle_direct_sampled.argtypes = [_pd, _i64, _pd, _pi64, _i64, _pd, _pd]
    lib.oracle_direct_k.argtypes = [_pd, _i64, _pd, _pd, _pd, ctypes.c_int]
    lib.oracle_direct_sampled_k.argtypes = [_pd, _i64, _pd, _pi64, _i64, _pd, _pd,
                                            ctypes.c_int]
    lib.oracle_cheb_nodes.argtypes = [ctypes.c_int, _pd]
    lib.oracle_cheb_S.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.oracle_cheb_S.restype = ctypes.c_double
    lib.oracle_cheb_dS.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.oracle_cheb_dS.restype = ctypes.c_double
    lib.oracle_p2m.argtypes = [ctypes.c_int, _i64, _pd, _pd, _pd, ctypes.c_double, _pd]
    lib.oracle_m2m.argtypes = [ctypes.c_int, ctypes.c_int, _pd, _pd]
    lib.oracle_l2l.argtypes = [ctypes.c_int, ctypes.c_int, _pd, _pd]
    lib.oracle_l2p.argtypes = [ctypes.c_int, _i64, _pd, _pd, _pd, ctypes.c_double,
                               _pd, _pd, _pd]
    lib.oracle_m2l_matrix.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      _pint, _pd]
    lib.oracle_m2l_matrix_k.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        _pint, _pd, ctypes.c_int]
    lib.oracle_tree_build.argtypes = [_pd, _i64, ctypes.c_int]
    lib.oracle_tree_build.restype = ctypes.c_void_p
    lib.oracle_tree_free.argtypes = [ctypes.c_void_p]
    lib.oracle_tree_info.argtypes = [ctypes.c_void_p, _pi64]
    lib.oracle_tree_box.argtypes = [ctypes.c_void_p, _pd]
    lib.oracle_tree_keys.argtypes = [ctypes.c_void_p, _pu64]
    lib.oracle_tree_perm.argtypes = [ctypes.c_void_p, _pi64]
    lib.oracle_tree_leaf_start.argtypes = [ctypes.c_void_p, _pi64]
    lib.oracle_tree_cell_keys.argtypes = [ctypes.c_void_p, ctypes.c_int, _pu64]
    lib.oracle_tree_near.argtypes = [ctypes.c_void_p, _pi64, _pi64]
    lib.oracle_tree_far.argtypes = [ctypes.c_void_p, ctypes.c_int, _pi64, _pi64]
    lib.oracle_fmm.argtypes = [ctypes.c_void_p, ctypes.c_int, _pd, _pi64, _i64,
                               _pd, _pd, _pd, _pd, _pd, _pd]
    lib.oracle_fmm_ops.argtypes = [ctypes.c_void_p, ctypes.c_int, _pd, _pi64, _i64, _pd,
                                   _pd, _pd, _pd, _pd, _pd, _pd, ctypes.c_int]
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, t=_pd):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def direct(pos, q, kernel=1):
    """Direct O(N^2) potentials and forces (Eq. 1-2) for the kernel
    |x - y|^-kernel (1: the paper's 1/r; 2: 1/r^2)."""
    pos = _f64(pos)
    n = pos.shape[0]
    q = _f64(q, (n,))
    phi = np.empty(n)
    f = np.empty((n, 3))
    rc = _load().oracle_direct_k(_ptr(pos), n, _ptr(q), _ptr(phi), _ptr(f), int(kernel))
    if rc != 0:
        raise ValueError("oracle_direct failed")
    return phi, f


def direct_sampled(pos, q, idx, kernel=1):
    """Exact sums at the targets ``idx`` over all sources."""
    pos = _f64(pos)
    n = pos.shape[0]
    q = _f64(q, (n,))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    s = idx.shape[0]
    phi = np.empty(s)
    f = np.empty((s, 3))
    rc = _load().oracle_direct_sampled_k(_ptr(pos), n, _ptr(q), _ptr(idx, _pi64), s,
                                         _ptr(phi), _ptr(f), int(kernel))
    if rc != 0:
        raise ValueError("oracle_direct_sampled failed")
    return phi, f


def cheb_nodes(l):
    xi = np.empty(l)
    if _load().oracle_cheb_nodes(l, _ptr(xi)) != 0:
        raise ValueError("bad order")
    return xi


def cheb_S(l, m, u):
    return float(_load().oracle_cheb_S(l, m, float(u)))


def cheb_dS(l, m, u):
    return float(_load().oracle_cheb_dS(l, m, float(u)))


def p2m(l, pos, q, center, a, W=None):
    pos = _f64(pos)
    n = pos.shape[0]
    q = _f64(q, (n,))
    c = _f64(center, (3,))
    W = np.zeros(l ** 3) if W is None else _f64(W, (l ** 3,)).copy()
    if _load().oracle_p2m(l, n, _ptr(pos), _ptr(q), _ptr(c), float(a), _ptr(W)) != 0:
        raise ValueError("oracle_p2m failed")
    return W


def m2m(l, octant, Wc, Wp=None):
    Wc = _f64(Wc, (l ** 3,))
    Wp = np.zeros(l ** 3) if Wp is None else _f64(Wp, (l ** 3,)).copy()
    if _load().oracle_m2m(l, octant, _ptr(Wc), _ptr(Wp)) != 0:
        raise ValueError("oracle_m2m failed")
    return Wp


def l2l(l, octant, Lp, Lc=None):
    Lp = _f64(Lp, (l ** 3,))
    Lc = np.zeros(l ** 3) if Lc is None else _f64(Lc, (l ** 3,)).copy()
    if _load().oracle_l2l(l, octant, _ptr(Lp), _ptr(Lc)) != 0:
        raise ValueError("oracle_l2l failed")
    return Lc


def l2p(l, pos, q, center, a, Loc):
    pos = _f64(pos)
    n = pos.shape[0]
    q = _f64(q, (n,))
    c = _f64(center, (3,))
    Loc = _f64(Loc, (l ** 3,))
    phi = np.empty(n)
    f = np.empty((n, 3))
    if _load().oracle_l2p(l, n, _ptr(pos), _ptr(q), _ptr(c), float(a), _ptr(Loc),
                          _ptr(phi), _ptr(f)) != 0:
        raise ValueError("oracle_l2p failed")
    return phi, f


def m2l_matrix(l, a, w, t, kernel=1):
    tt = np.ascontiguousarray(t, dtype=np.int32)
    K = np.empty((l ** 3, l ** 3))
    if _load().oracle_m2l_matrix_k(l, float(a), float(w), tt.ctypes.data_as(_pint),
                                   _ptr(K), int(kernel)) != 0:
        raise ValueError("oracle_m2l_matrix failed")
    return K


class Tree:
    """Octree of height ``h`` over ``pos`` built by the oracle."""

    def __init__(self, pos, h):
        self._pos = _f64(pos)
        if self._pos.ndim != 2 or self._pos.shape[1] != 3:
            raise ValueError("positions must be (n, 3)")
        self.n = self._pos.shape[0]
        self.h = int(h)
        lib = _load()
        self._h = lib.oracle_tree_build(_ptr(self._pos), self.n, self.h)
        if not self._h:
            raise ValueError("oracle_tree_build rejected the input")
        info = np.zeros(3 + self.h, dtype=np.int64)
        lib.oracle_tree_info(self._h, _ptr(info, _pi64))
        self.n_leaf = int(info[2])
        self.ncell = [int(x) for x in info[3:]]
        box = np.zeros(4)
        lib.oracle_tree_box(self._h, _ptr(box))
        self.lo = box[:3].copy()
        self.L = float(box[3])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_tree_free(h)
            self._h = None

    def keys(self):
        out = np.empty(self.n, dtype=np.uint64)
        _load().oracle_tree_keys(self._h, _ptr(out, _pu64))
        return out

    def perm(self):
        out = np.empty(self.n, dtype=np.int64)
        _load().oracle_tree_perm(self._h, _ptr(out, _pi64))
        return out

    def leaf_start(self):
        out = np.empty(self.n_leaf + 1, dtype=np.int64)
        _load().oracle_tree_leaf_start(self._h, _ptr(out, _pi64))
        return out

    def cell_keys(self, level):
        out = np.empty(self.ncell[level], dtype=np.uint64)
        if _load().oracle_tree_cell_keys(self._h, level, _ptr(out, _pu64)) != 0:
            raise ValueError("bad level")
        return out

    def near(self):
        off = np.empty(self.n_leaf + 1, dtype=np.int64)
        lib = _load()
        lib.oracle_tree_near(self._h, _ptr(off, _pi64), None)
        idx = np.empty(int(off[-1]), dtype=np.int64)
        lib.oracle_tree_near(self._h, _ptr(off, _pi64), _ptr(idx, _pi64))
        return off, idx

    def far(self, level):
        off = np.empty(self.ncell[level] + 1, dtype=np.int64)
        lib = _load()
        if lib.oracle_tree_far(self._h, level, _ptr(off, _pi64), None) != 0:
            raise ValueError("bad level")
        idx = np.empty(int(off[-1]), dtype=np.int64)
        lib.oracle_tree_far(self._h, level, _ptr(off, _pi64), _ptr(idx, _pi64))
        return off, idx

    def fmm(self, l, q, targets=None, parts=False, unit_ops=None, kernel=1):
        """FMM potentials and forces for the kernel |x - y|^-kernel; near +
        far, or the four parts.  With ``unit_ops`` (from
        :func:`compressed_unit_ops`, for the same kernel) M2L uses those
        operators instead of the exact kernel matrices."""
        q = _f64(q, (self.n,))
        if unit_ops is not None:
            unit_ops = np.ascontiguousarray(unit_ops, dtype=np.float64)
            if unit_ops.shape != (343, l ** 3, l ** 3):
                raise ValueError("unit_ops must be (343, l^3, l^3)")
        if targets is None:
            nt = self.n
            tptr = None
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int64)
            nt = targets.shape[0]
            tptr = _ptr(targets, _pi64)
        phi = np.empty(nt)
        f = np.empty((nt, 3))
        pn = np.empty(nt) if parts else None
        fn = np.empty((nt, 3)) if parts else None
        pf = np.empty(nt) if parts else None
        ff = np.empty((nt, 3)) if parts else None
        rc = _load().oracle_fmm_ops(self._h, int(l), _ptr(q), tptr, nt, _ptr(unit_ops),
                                    _ptr(phi), _ptr(f), _ptr(pn), _ptr(fn), _ptr(pf),
                                    _ptr(ff), int(kernel))
        if rc != 0:
            raise ValueError(f"oracle_fmm failed ({rc})")
        if parts:
            return phi, f, pn, fn, pf, ff
        return phi, f


def fmm(pos, q, h, l, targets=None, kernel=1):
    """Convenience: build the tree and evaluate."""
    return Tree(pos, h).fmm(l, q, targets=targets, kernel=kernel)


def far_offsets():
    """The 316 far-field offsets t (|t|_inf in {2, 3}) and their ids."""
    out = []
    for tx in range(-3, 4):
        for ty in range(-3, 4):
            for tz in range(-3, 4):
                if max(abs(tx), abs(ty), abs(tz)) >= 2:
                    out.append(((tx, ty, tz), (tx + 3) * 49 + (ty + 3) * 7 + (tz + 3)))
    return out


_ops_cache = {}


def compressed_unit_ops(l, eps, kernel=1):
    """Compressed M2L of Sec. 2.1.2: for every far offset t, the unit
    operator (cells of half-width 1) replaced by its truncated SVD, keeping
    the singular values s_k >= eps * s_1 (eps = 0 keeps all).  Each offset's
    operator is decomposed on its own (numpy's LAPACK SVD; no symmetry is
    used).  Returns (ops[343][l^3][l^3], {offset: rank})."""
    key = (l, float(eps), int(kernel))
    if key in _ops_cache:
        return _ops_cache[key]
    l3 = l ** 3
    ops = np.zeros((343, l3, l3))
    ranks = {}
    for t, i in far_offsets():
        K = m2l_matrix(l, 1.0, 2.0, t, kernel)
        U, s, Vt = np.linalg.svd(K)
        r = int(np.sum(s >= eps * s[0]))
        ops[i] = (U[:, :r] * s[:r]) @ Vt[:r]
        ranks[t] = r
    _ops_cache[key] = (ops, ranks)
    return ops, ranks
