"""Hierarchical orthogonal complements of rigid-body Z-matrices on MI355X.

Thin Python binding of the C ABI in ``include/hq.h`` (``libhq.so``): argument
marshalling only.  Every step of the method runs in the library's HIP kernels;
PyTorch supplies device memory and the current stream.

    h = build(positions, offsets)          # tree + FP64 transforms
    y = h.apply(v)                         # Q~ v      (v: 3N x R, float64/float32)
    z = h.apply(w, transpose=True)         # Q~^T w    (w: rows x R)
    Q = h.explicit(body)                   # dense Q~ of one body

Fang, Huang, Huber, McCammon, Zhang, "Hierarchical Orthogonal Matrix
Generation and Matrix-Vector Multiplications in Rigid Body Simulations"
(Sections 3-4, Algorithms 1-3).
"""
from __future__ import annotations

import ctypes
import hashlib

import numpy as np

from . import _lib
from ._lib import (HQ_BODY_DEGENERATE, HQ_BODY_ILLCOND, HQ_FLAG_BOUNDS, HQ_FLAG_NONFINITE, HQ_FLAG_PHASES,
                   HQ_FLAG_STACK, HQ_FP32, HQ_FP64, Info, Options)

__all__ = ["HQError", "Handle", "build", "build_into", "workspace_bytes", "load", "HQ_FP64", "HQ_FP32"]


class HQError(RuntimeError):
    def __init__(self, status, where):
        lib = _lib.load()
        self.status = int(status)
        msg = lib.hq_last_error().decode(errors="replace")
        name = lib.hq_status_string(status).decode()
        super().__init__(f"{where}: {name}: {msg}")


def load():
    return _lib.load()


def _check(st, where):
    if st != 0:
        raise HQError(st, where)


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


# vector layouts of hq_apply_layout (hq_layout)
LAYOUTS = {"rows": _lib.HQ_ROWS, "triples": _lib.HQ_TRIPLES}


def _prec(dtype):
    torch = _torch()
    if dtype == torch.float64:
        return HQ_FP64
    if dtype == torch.float32:
        return HQ_FP32
    raise TypeError(f"unsupported dtype {dtype}: use float64 or float32")


def _check_dev(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check_f64(t, name, count, shape=None):
    """A contiguous float64 device tensor of ``count`` values (and ``shape``)."""
    torch = _torch()
    _check_dev(t, name)
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.numel() != count or (shape is not None and tuple(t.shape) != shape):
        want = shape if shape is not None else f"{count} values"
        raise ValueError(f"{name} must hold {want}, got {tuple(t.shape)}")


class Handle:
    """A built set of bodies (owns the library's device state)."""

    def __init__(self, raw, offsets, stream=None):
        self._raw = raw
        self.offsets = np.asarray(offsets, dtype=np.int64)
        sizes = np.diff(self.offsets)
        self.row_offsets = np.concatenate([[0], np.cumsum(3 * sizes - 6)]).astype(np.int64)

    @property
    def N(self):
        return int(self.offsets[-1])

    @property
    def m(self):
        return len(self.offsets) - 1

    @property
    def rows(self):
        return int(self.row_offsets[-1])

    def _h(self):
        if not self._raw:
            raise RuntimeError("handle was destroyed")
        return self._raw

    def destroy(self):
        if self._raw:
            _lib.load().hq_destroy(self._raw)
            self._raw = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # -- products ---------------------------------------------------------
    def apply(self, v, transpose=False, out=None, stream=None, timed=False, layout="rows", noalloc=False):
        """Q~ v (v: 3N x R) or Q~^T w (w: rows x R); R = 1 for a 1-D v.
        layout="triples": v and out are (rows / 3, R, 3) tensors, row triple
        t's right-hand side r at [t, r, :] (hq_apply_layout, HQ_TRIPLES).
        With timed=True returns (out, per-phase launch ms) via hq_apply_timed.
        noalloc=True calls hq_apply_noalloc (the library allocates nothing;
        pass ``out`` to allocate nothing here either)."""
        torch = _torch()
        _check_dev(v, "v")
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        nin, nout = (self.rows, 3 * self.N) if transpose else (3 * self.N, self.rows)
        squeeze = False
        if layout == "triples":
            if v.dim() != 3 or v.shape[0] * 3 != nin or v.shape[2] != 3:
                raise ValueError(f"v must be ({nin // 3}, R, 3) in the triples layout, got {tuple(v.shape)}")
            R = v.shape[1]
            v2, oshape = v, (nout // 3, R, 3)
        else:
            squeeze = v.dim() == 1
            v2 = v.reshape(v.shape[0], 1) if squeeze else v
            R = v2.shape[1]
            if v2.shape[0] != nin:
                raise ValueError(f"v has {v2.shape[0]} rows, expected {nin}")
            oshape = (nout, R)
        if not v2.is_contiguous():
            raise ValueError("v must be contiguous")
        if out is None:
            out = torch.empty(oshape, dtype=v.dtype, device=v.device)
        else:
            _check_dev(out, "out")
            if tuple(out.shape) != oshape and not (squeeze and out.shape == (nout,)):
                raise ValueError("out has the wrong shape")
            if out.dtype != v.dtype:
                raise TypeError("out and v must have the same dtype")
            if not out.is_contiguous():
                raise ValueError("out must be contiguous")
        lib = _lib.load()
        lay = LAYOUTS[layout]
        if timed:
            ms = (ctypes.c_float * 64)()
            nph = ctypes.c_int32()
            _check(lib.hq_apply_timed(self._h(), _ptr(v2), _ptr(out), int(bool(transpose)), R, _prec(v.dtype),
                                      lay, _stream(stream), ms, 64, ctypes.byref(nph)), "hq_apply_timed")
            res = out.reshape(nout) if squeeze else out
            return res, [ms[i] for i in range(nph.value)]
        fn, name = (lib.hq_apply_noalloc, "hq_apply_noalloc") if noalloc else (lib.hq_apply_layout, "hq_apply_layout")
        _check(fn(self._h(), _ptr(v2), _ptr(out), int(bool(transpose)), R, _prec(v.dtype), lay, _stream(stream)), name)
        return out.reshape(nout) if squeeze else out

    def apply_full(self, v, transpose=False, root=None, out=None, stream=None, layout="rows"):
        """The full Q = [Q_Z; Q~] (hq_apply_full).  transpose=False: returns
        (Q~ v, Q_Z v) with Q_Z v as 6 rows per body ((6m, R), or (2m, R, 3)
        in the triples layout).  transpose=True: ``root`` (the same shape)
        supplies the root Velocity-sets; returns Q_Z^T root + Q~^T v."""
        torch = _torch()
        _check_dev(v, "v")
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        nin, nout = (self.rows, 3 * self.N) if transpose else (3 * self.N, self.rows)
        if layout == "triples":
            if v.dim() != 3 or v.shape[0] * 3 != nin or v.shape[2] != 3:
                raise ValueError(f"v must be ({nin // 3}, R, 3) in the triples layout, got {tuple(v.shape)}")
            R = v.shape[1]
            oshape, rshape = (nout // 3, R, 3), (2 * self.m, R, 3)
        else:
            if v.dim() != 2 or v.shape[0] != nin:
                raise ValueError(f"v must be ({nin}, R), got {tuple(v.shape)}")
            R = v.shape[1]
            oshape, rshape = (nout, R), (6 * self.m, R)
        if root is None:
            if transpose:
                raise ValueError("transpose=True needs root (the root Velocity-sets)")
            root = torch.empty(rshape, dtype=v.dtype, device=v.device)
        else:
            _check_dev(root, "root")
            if tuple(root.shape) != rshape or root.dtype != v.dtype or not root.is_contiguous():
                raise ValueError(f"root must be a contiguous {rshape} tensor of v's dtype")
        if out is None:
            out = torch.empty(oshape, dtype=v.dtype, device=v.device)
        else:
            _check_dev(out, "out")
            if tuple(out.shape) != oshape or out.dtype != v.dtype:
                raise ValueError(f"out must be a contiguous {oshape} tensor of v's dtype")
        if not v.is_contiguous():
            raise ValueError("v must be contiguous")
        _check(_lib.load().hq_apply_full(self._h(), _ptr(v), _ptr(out), _ptr(root), int(bool(transpose)), R,
                                         _prec(v.dtype), LAYOUTS[layout], _stream(stream)), "hq_apply_full")
        return out if transpose else (out, root)

    def apply_rotated(self, rot, v, transpose=False, out=None, work=None, stream=None, layout="rows"):
        """hq_apply_rotated: products of the bodies after rigid rotations
        ``rot`` ((m, 3, 3) or (m, 9) float64, device) since the last build or
        rebuild, with the handle's transforms (no rebuild).  Shapes as for
        apply(); ``work`` (the upward product's rotated input) is allocated
        when not given."""
        torch = _torch()
        _check_dev(v, "v")
        _check_dev(rot, "rot")
        if rot.dtype != torch.float64 or rot.numel() != 9 * self.m or not rot.is_contiguous():
            raise ValueError("rot must be a contiguous float64 tensor of m x 9 (or m x 3 x 3) values")
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        nin, nout = (self.rows, 3 * self.N) if transpose else (3 * self.N, self.rows)
        if layout == "triples":
            if v.dim() != 3 or v.shape[0] * 3 != nin or v.shape[2] != 3:
                raise ValueError(f"v must be ({nin // 3}, R, 3) in the triples layout")
            R = v.shape[1]
            oshape = (nout // 3, R, 3)
        else:
            if v.dim() != 2 or v.shape[0] != nin:
                raise ValueError(f"v must be ({nin}, R)")
            R = v.shape[1]
            oshape = (nout, R)
        if not v.is_contiguous():
            raise ValueError("v must be contiguous")
        if out is None:
            out = torch.empty(oshape, dtype=v.dtype, device=v.device)
        else:
            _check_dev(out, "out")
            if tuple(out.shape) != oshape or out.dtype != v.dtype:
                raise ValueError(f"out must be a contiguous {oshape} tensor of v's dtype")
        wp = None
        if not transpose:
            if work is None:
                work = torch.empty_like(v)
            else:
                _check_dev(work, "work")
                if work.shape != v.shape or work.dtype != v.dtype:
                    raise ValueError("work must be a contiguous tensor like v")
            wp = _ptr(work)
        _check(_lib.load().hq_apply_rotated(self._h(), _ptr(rot), _ptr(v), _ptr(out), wp, int(bool(transpose)), R,
                                            _prec(v.dtype), LAYOUTS[layout], _stream(stream)), "hq_apply_rotated")
        return out

    def node_phase(self):
        """Tile phase of every internal node (handle order)."""
        ph = np.zeros(self.N - self.m, dtype=np.int32)
        _check(_lib.load().hq_node_phase(self._h(), ph.ctypes.data_as(_lib.P_i32)), "hq_node_phase")
        return ph

    def reserve(self, nrhs, dtype):
        _check(_lib.load().hq_reserve(self._h(), int(nrhs), _prec(dtype)), "hq_reserve")

    def rebuild(self, positions, stream=None):
        _check_f64(positions, "positions", 3 * self.N, (self.N, 3))
        _check(_lib.load().hq_rebuild(self._h(), _ptr(positions), _stream(stream)), "hq_rebuild")

    def rigid_update(self, positions, rot, trans, stream=None):
        """Positions (N, 3) float64 in place; rot m x 9 (or m x 3 x 3) and
        trans m x 3 float64, all on the device."""
        _check_f64(positions, "positions", 3 * self.N, (self.N, 3))
        _check_f64(rot, "rot", 9 * self.m)
        _check_f64(trans, "trans", 3 * self.m)
        _check(_lib.load().hq_rigid_update(self._h(), _ptr(positions), _ptr(rot), _ptr(trans), _stream(stream)),
               "hq_rigid_update")

    def rigid_motion(self, positions, out, rot, trans, centers, stream=None):
        """hq_rigid_motion: out = Rot_j (positions - c_j) + c_j + t_j per body
        (out may be positions); positions and out (N, 3), rot m x 9, trans
        and centers m x 3, float64 on the device."""
        _check_f64(positions, "positions", 3 * self.N, (self.N, 3))
        _check_f64(out, "out", 3 * self.N, (self.N, 3))
        _check_f64(rot, "rot", 9 * self.m)
        _check_f64(trans, "trans", 3 * self.m)
        _check_f64(centers, "centers", 3 * self.m)
        _check(_lib.load().hq_rigid_motion(self._h(), _ptr(positions), _ptr(out), _ptr(rot), _ptr(trans),
                                           _ptr(centers), _stream(stream)), "hq_rigid_motion")

    # -- explicit Q~ --------------------------------------------------------
    def explicit(self, body=0, stream=None):
        """Dense Q~ of one body: (3n-6) x 3n float64 on the device."""
        torch = _torch()
        n = int(self.offsets[body + 1] - self.offsets[body])
        out = torch.empty((max(3 * n - 6, 0), 3 * n), dtype=torch.float64, device="cuda")
        _check(_lib.load().hq_explicit(self._h(), int(body), _ptr(out), 3 * n, _stream(stream)), "hq_explicit")
        return out

    def explicit_blocks_size(self, body=0):
        """(blocks, values) of the block-sparse Q~ of one body."""
        nb, nv = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib.load().hq_explicit_blocks_size(self._h(), int(body), ctypes.byref(nb), ctypes.byref(nv)),
               "hq_explicit_blocks_size")
        return nb.value, nv.value

    def explicit_blocks(self, body=0, dtype=None, stream=None):
        """Block-sparse Q~ of one body: (values, val_off, row_off, bead_first,
        rows, cols); see hq_explicit_blocks."""
        torch = _torch()
        dtype = dtype or torch.float64
        lib = _lib.load()
        nb, nv = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib.hq_explicit_blocks_size(self._h(), int(body), ctypes.byref(nb), ctypes.byref(nv)),
               "hq_explicit_blocks_size")
        nb, nv = nb.value, nv.value
        values = torch.empty(max(nv, 1), dtype=dtype, device="cuda")
        val_off = np.zeros(nb + 1, dtype=np.int64)
        row_off = np.zeros(max(nb, 1), dtype=np.int64)
        bead_first = np.zeros(max(nb, 1), dtype=np.int64)
        rows = np.zeros(max(nb, 1), dtype=np.int32)
        cols = np.zeros(max(nb, 1), dtype=np.int32)
        _check(lib.hq_explicit_blocks(self._h(), int(body), _prec(dtype), _ptr(values),
                                      val_off.ctypes.data_as(_lib.P_i64), row_off.ctypes.data_as(_lib.P_i64),
                                      bead_first.ctypes.data_as(_lib.P_i64), rows.ctypes.data_as(_lib.P_i32),
                                      cols.ctypes.data_as(_lib.P_i32), _stream(stream)), "hq_explicit_blocks")
        return values[:nv], val_off, row_off[:nb], bead_first[:nb], rows[:nb], cols[:nb]

    def sorted_beads(self, body=0):
        n = int(self.offsets[body + 1] - self.offsets[body])
        out = np.zeros(n, dtype=np.int64)
        _check(_lib.load().hq_sorted_beads(self._h(), int(body), out.ctypes.data_as(_lib.P_i64)),
               "hq_sorted_beads")
        return out

    # -- introspection ------------------------------------------------------
    def query(self):
        info = Info()
        _check(_lib.load().hq_query(self._h(), ctypes.byref(info)), "hq_query")
        return {f: getattr(info, f) for f, _ in Info._fields_}

    def body_info(self):
        flags = np.zeros(self.m, dtype=np.int32)
        kappa = np.zeros(self.m, dtype=np.float64)
        _check(_lib.load().hq_body_info(self._h(), flags.ctypes.data_as(_lib.P_i32),
                                        kappa.ctypes.data_as(_lib.P_f64)), "hq_body_info")
        return flags, kappa

    def node_data(self, with_G=True, with_geometry=True):
        """Per-node tree and transform data (G needs the FP64 transforms;
        centroids and T22 after a rebuild need keep_node_data)."""
        NI = self.N - self.m
        a = {k: np.zeros(NI, dtype=np.int32) for k in ("first", "last", "x", "y", "body", "n", "k", "row")}
        cen = np.zeros((NI, 3)) if with_geometry else None
        T22 = np.zeros((NI, 3, 3)) if with_geometry else None
        G = np.zeros((NI, 9, 9)) if with_G else None
        P = _lib.P_i32
        f64 = (lambda x: x.ctypes.data_as(_lib.P_f64) if x is not None else None)
        _check(_lib.load().hq_node_data(self._h(), a["first"].ctypes.data_as(P), a["last"].ctypes.data_as(P),
                                        a["x"].ctypes.data_as(P), a["y"].ctypes.data_as(P),
                                        a["body"].ctypes.data_as(P), a["n"].ctypes.data_as(P),
                                        f64(cen), f64(T22), f64(G), a["k"].ctypes.data_as(P),
                                        a["row"].ctypes.data_as(P)), "hq_node_data")
        a.update(centroid=cen, T22=T22, G=G)
        return a


def _offsets(positions, offsets):
    _check_dev(positions, "positions")
    torch = _torch()
    if positions.dtype != torch.float64:
        raise TypeError("positions must be float64")
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or len(off) < 2:
        raise ValueError("offsets must hold m + 1 entries")
    if positions.dim() != 2 or positions.shape[1] != 3 or positions.shape[0] != int(off[-1]):
        raise ValueError("positions must be N x 3 with N = offsets[-1]")
    return off


def _options(kw):
    names = [f for f, _ in Options._fields_]
    unknown = set(kw) - set(names)
    if unknown:
        raise TypeError(f"unknown options {sorted(unknown)}")
    return Options(*[int(kw.get(f, 0)) for f in names])


def build(positions, offsets, stream=None, **options):
    """Build the tree and FP64 transforms for bodies given by ``offsets``
    (host, m + 1 int64) over ``positions`` (device, N x 3 float64).
    ``options``: hq_options fields (tile_units, store, run_nodes, ...)."""
    off = _offsets(positions, offsets)
    opt = _options(options)
    raw = ctypes.c_void_p()
    lib = _lib.load()
    _check(lib.hq_build(_ptr(positions), off.ctypes.data_as(_lib.P_i64), len(off) - 1, ctypes.byref(opt),
                        _stream(stream), ctypes.byref(raw)), "hq_build")
    return Handle(raw, off)


def workspace_bytes(offsets, **options):
    """hq_workspace_bytes: device bytes of a handle built by build_into."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or len(off) < 2:
        raise ValueError("offsets must hold m + 1 entries")
    opt = _options(options)
    n = ctypes.c_size_t(0)
    _check(_lib.load().hq_workspace_bytes(off.ctypes.data_as(_lib.P_i64), len(off) - 1, ctypes.byref(opt),
                                          ctypes.byref(n)), "hq_workspace_bytes")
    return int(n.value)


def build_into(positions, offsets, workspace=None, stream=None, **options):
    """hq_build_into: build with every piece of device state in ``workspace``
    (a 256-byte aligned torch uint8 tensor of at least workspace_bytes bytes;
    allocated here with torch when None).  The handle keeps a reference to it
    and the library allocates no device memory for this handle."""
    torch = _torch()
    off = _offsets(positions, offsets)
    opt = _options(options)
    need = workspace_bytes(off, **options)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=positions.device)
    _check_dev(workspace, "workspace")
    nbytes = workspace.numel() * workspace.element_size()
    raw = ctypes.c_void_p()
    _check(_lib.load().hq_build_into(_ptr(positions), off.ctypes.data_as(_lib.P_i64), len(off) - 1,
                                     ctypes.byref(opt), _ptr(workspace), nbytes, _stream(stream), ctypes.byref(raw)),
           "hq_build_into")
    h = Handle(raw, off)
    h.workspace = workspace
    return h


def constrained_solve(h, dapply, F, layout="rows", rtol=1e-8, max_iter=500, stream=None, check_every=4):
    """hq_constrained_solve: the constraint forces g of Eq. 1.5 by conjugate
    gradients on Q~ D Q~^T and the rigid-body velocities V of Eq. 1.6.
    ``dapply(x, y)`` writes D x into y (torch tensors of the vector shape
    (3N, R), or (N, R, 3) in the triples layout) on the current stream.
    ``F``: (6m, R) or (2m, R, 3).  The host checks convergence every
    ``check_every`` iterations.  Returns (V, g, info dict)."""
    torch = _torch()
    _check_dev(F, "F")
    if layout not in LAYOUTS:
        raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
    if layout == "triples":
        if F.dim() != 3 or F.shape[0] != 2 * h.m or F.shape[2] != 3:
            raise ValueError(f"F must be ({2 * h.m}, R, 3) in the triples layout")
        R = F.shape[1]
        bshape, gshape = (h.N, R, 3), (h.rows // 3, R, 3)
    else:
        if F.dim() != 2 or F.shape[0] != 6 * h.m:
            raise ValueError(f"F must be ({6 * h.m}, R)")
        R = F.shape[1]
        bshape, gshape = (3 * h.N, R), (h.rows, R)
    if not F.is_contiguous():
        raise ValueError("F must be contiguous")
    dx = torch.empty(bshape, dtype=F.dtype, device=F.device)
    dy = torch.empty(bshape, dtype=F.dtype, device=F.device)
    V = torch.empty_like(F)
    g = torch.empty(gshape, dtype=F.dtype, device=F.device)
    errors = []
    ts = stream or torch.cuda.current_stream()

    def cb(x, y, nrhs, user, s):
        try:
            with torch.cuda.stream(ts):
                dapply(dx, dy)
            return 0
        except Exception as e:  # reported through the status below
            errors.append(e)
            return 1

    fn = _lib.DAPPLY_FN(cb)
    if not 1 <= int(check_every) <= 64:
        raise ValueError("check_every must be in [1, 64]")
    info = _lib.KrylovInfo(int(max_iter), float(rtol), 0, 0.0, int(check_every))
    st = _lib.load().hq_constrained_solve(h._h(), fn, None, _ptr(F), _ptr(V), _ptr(g), R, _prec(F.dtype),
                                          LAYOUTS[layout], _ptr(dx), _ptr(dy), ctypes.byref(info), _stream(ts))
    if errors:
        raise errors[0]
    _check(st, "hq_constrained_solve")
    return V, g, {"iters": info.iters, "max_rel_residual": info.max_rel_residual}


_TUNED = {}


def autotune(positions, offsets, nrhs, dtype=None, include_rebuild=True, stream=None, layout="rows", **base):
    """hq_autotune: the tile size, run length and later-phase waves per CU
    with the shortest measured (rebuild +) upward + downward round for this
    workload.  Returns a dict of hq_options fields plus ``ms``; results are
    remembered per (offsets, nrhs, dtype, include_rebuild, base options) for
    the life of the process."""
    torch = _torch()
    dtype = dtype or torch.float32
    off = _offsets(positions, offsets)
    if layout not in LAYOUTS:
        raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
    key = (hashlib.sha1(off.tobytes()).hexdigest(), int(nrhs), str(dtype), bool(include_rebuild), layout,
           tuple(sorted(base.items())))
    if key in _TUNED:
        return dict(_TUNED[key])
    names = [f for f, _ in Options._fields_]
    b = _options(base)
    best = Options()
    ms = ctypes.c_double()
    _check(_lib.load().hq_autotune(_ptr(positions), off.ctypes.data_as(_lib.P_i64), len(off) - 1, int(nrhs),
                                   _prec(dtype), LAYOUTS[layout], int(bool(include_rebuild)), ctypes.byref(b),
                                   _stream(stream),
                                   ctypes.byref(best), ctypes.byref(ms)), "hq_autotune")
    res = {f: getattr(best, f) for f in names}
    res["ms"] = ms.value
    _TUNED[key] = res
    return dict(res)


def capture_begin(stream=None):
    _check(_lib.load().hq_capture_begin(_stream(stream)), "hq_capture_begin")


def capture_end(stream=None):
    ex = ctypes.c_void_p()
    _check(_lib.load().hq_capture_end(_stream(stream), ctypes.byref(ex)), "hq_capture_end")
    return Graph(ex)


class Graph:
    """A captured stream sequence (hipGraphExec), replayed by launch()."""

    def __init__(self, ex):
        self._ex = ex

    def launch(self, stream=None):
        _check(_lib.load().hq_graph_launch(self._ex, _stream(stream)), "hq_graph_launch")

    def destroy(self):
        if self._ex:
            _lib.load().hq_graph_destroy(self._ex)
            self._ex = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
