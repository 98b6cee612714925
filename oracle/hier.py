"""ctypes binding of the plain FP64 hierarchical oracle (``oracle/hier.c``).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the bench's
CPU-baseline leg, never by the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "hier.c")
LIB = os.path.join(_HERE, "liboracle_hier.so")

_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def load(path: str | None = None):
    """Load the oracle library (building it first if absent or stale)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    if path is None:
        build(force=False)
        path = LIB
    lib = ctypes.CDLL(path)
    lib.or_build.restype = ctypes.c_void_p
    lib.or_build.argtypes = [_dp, _i64]
    lib.or_build_s.restype = ctypes.c_void_p
    lib.or_build_s.argtypes = [_dp, _i64, _i64]
    lib.or_free.argtypes = [ctypes.c_void_p]
    lib.or_free.restype = None
    for f in ("or_n", "or_rows", "or_num_internal"):
        getattr(lib, f).restype = _i64
        getattr(lib, f).argtypes = [ctypes.c_void_p]
    lib.or_max_kappa.restype = ctypes.c_double
    lib.or_max_kappa.argtypes = [ctypes.c_void_p]
    lib.or_perm.argtypes = [ctypes.c_void_p, _i64p]
    lib.or_perm.restype = None
    lib.or_tree.argtypes = [ctypes.c_void_p, _i64p, _i64p, _i64p]
    lib.or_tree.restype = None
    lib.or_codes.argtypes = [_dp, _i64, _u64p]
    lib.or_codes.restype = None
    lib.or_node.argtypes = [ctypes.c_void_p, _i64, _i64p, _dp]
    lib.or_node.restype = None
    lib.or_apply.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int, _i64]
    lib.or_apply.restype = None
    lib.or_apply_full.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int, _i64, _dp]
    lib.or_apply_full.restype = None
    lib.or_up_infosets.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.or_up_infosets.restype = None
    lib.or_explicit.argtypes = [ctypes.c_void_p, _dp]
    lib.or_explicit.restype = None
    lib.or_explicit_full.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.or_explicit_full.restype = None
    if path == LIB:
        _lib = lib
    return lib


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def codes(pos) -> np.ndarray:
    """Quantised z-y-x interleaved box codes of one body's beads (user order)."""
    lib = load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    out = np.zeros(len(pos), dtype=np.uint64)
    lib.or_codes(_ptr(pos), len(pos), _ptr(out, _u64p))
    return out


class Node:
    __slots__ = ("first", "last", "x", "y", "n", "k", "dim", "off", "bucket", "c", "T22",
                 "sx", "sy", "kappa", "G")


class Body:
    """One rigid body: the oracle's tree, transforms and products.  Leaves
    hold at most ``s`` beads (s = 1: one bead per leaf)."""

    def __init__(self, pos, lib=None, s=1):
        self.lib = lib if lib is not None else load()
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.n = len(self.pos)
        self.s = int(s)
        if self.n < 2:
            raise ValueError("a body needs at least 2 beads")
        if self.s < 1:
            raise ValueError("s must be >= 1")
        self._h = self.lib.or_build_s(_ptr(self.pos), self.n, self.s)
        if not self._h:
            raise RuntimeError("oracle build failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.lib.or_free(h)
            self._h = None

    @property
    def rows(self):
        return 3 * self.n - 6

    @property
    def num_internal(self):
        return int(self.lib.or_num_internal(self._h))

    @property
    def max_kappa(self):
        return float(self.lib.or_max_kappa(self._h))

    def perm(self):
        out = np.zeros(self.n, dtype=np.int64)
        self.lib.or_perm(self._h, _ptr(out, _i64p))
        return out

    def tree(self):
        """(first, last, split) of every internal node: its sorted-position
        range and the last position of its x child."""
        k = self.num_internal
        f, l, s = (np.zeros(k, dtype=np.int64) for _ in range(3))
        self.lib.or_tree(self._h, _ptr(f, _i64p), _ptr(l, _i64p), _ptr(s, _i64p))
        return f, l, s

    def node(self, i) -> Node:
        ints = np.zeros(9, dtype=np.int64)
        dbl = np.zeros(96, dtype=np.float64)
        self.lib.or_node(self._h, int(i), _ptr(ints, _i64p), _ptr(dbl))
        nd = Node()
        (nd.first, nd.last, nd.x, nd.y, nd.n, nd.k, nd.dim, nd.off, nd.bucket) = (int(t) for t in ints)
        nd.c = dbl[0:3].copy()
        nd.T22 = dbl[3:12].reshape(3, 3).copy()
        nd.sx, nd.sy, nd.kappa = float(dbl[12]), float(dbl[13]), float(dbl[14])
        nd.G = dbl[15:96].reshape(9, 9)[: nd.k, : nd.k].copy()
        return nd

    def nodes(self):
        return [self.node(i) for i in range(self.num_internal)]

    def apply(self, v, transpose=False, root=None):
        """Q~ v (transpose=False, v: 3n x R) or Q~^T w (w: (3n-6) x R).
        With ``root`` (6 x R array) the full Q = [Q_Z; Q~] is used: it receives
        Q_Z v, or supplies the root Velocity-set."""
        v = np.asarray(v, dtype=np.float64)
        vec = v.ndim == 1
        R = 1 if vec else v.shape[1]
        v2 = np.ascontiguousarray(v.reshape(v.shape[0], R))
        if not transpose:
            assert v2.shape[0] == 3 * self.n
            out = np.zeros((self.rows, R))
        else:
            assert v2.shape[0] == self.rows
            out = np.zeros((3 * self.n, R))
        if root is not None:
            root_arr = np.ascontiguousarray(np.asarray(root, dtype=np.float64).reshape(6, R))
            self.lib.or_apply_full(self._h, _ptr(v2), _ptr(out), int(bool(transpose)), R, _ptr(root_arr))
            if not transpose and isinstance(root, np.ndarray) and root.flags.c_contiguous and root.size == 6 * R:
                root.reshape(6, R)[...] = root_arr
            return (out[:, 0] if vec else out), root_arr
        self.lib.or_apply(self._h, _ptr(v2), _ptr(out), int(bool(transpose)), R)
        return out[:, 0] if vec else out

    def up_infosets(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        out = np.zeros(self.rows)
        M = np.zeros((self.num_internal, 6))
        self.lib.or_up_infosets(self._h, _ptr(f), _ptr(out), _ptr(M))
        return out, M

    def explicit(self, with_root_u=False):
        Q = np.zeros((self.rows, 3 * self.n))
        if with_root_u:
            U = np.zeros((3, 3 * self.n))
            self.lib.or_explicit_full(self._h, _ptr(Q), _ptr(U))
            return Q, U
        self.lib.or_explicit(self._h, _ptr(Q))
        return Q


class Batch:
    """Block-diagonal Q~ = diag(Q~^1, ..., Q~^m) over bodies given by offsets."""

    def __init__(self, pos, offsets, s=1):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.bodies = [Body(self.pos[self.offsets[j]:self.offsets[j + 1]], s=s)
                       for j in range(len(self.offsets) - 1)]
        sizes = np.diff(self.offsets)
        self.row_off = np.zeros(len(sizes) + 1, dtype=np.int64)
        np.cumsum(3 * sizes - 6, out=self.row_off[1:])

    @property
    def rows(self):
        return int(self.row_off[-1])

    def apply(self, v, transpose=False):
        v = np.asarray(v, dtype=np.float64)
        R = 1 if v.ndim == 1 else v.shape[1]
        v2 = v.reshape(v.shape[0], R)
        N = int(self.offsets[-1])
        out = np.zeros(((3 * N) if transpose else self.rows, R))
        for j, b in enumerate(self.bodies):
            b0, b1 = 3 * self.offsets[j], 3 * self.offsets[j + 1]
            r0, r1 = self.row_off[j], self.row_off[j + 1]
            if transpose:
                out[b0:b1] = b.apply(v2[r0:r1], True)
            else:
                out[r0:r1] = b.apply(v2[b0:b1], False)
        return out.reshape((out.shape[0],) + v.shape[1:])
