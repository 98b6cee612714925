"""The full Q = [Q_Z; Q~] (hq_apply_full): the root Info-sets Q_Z v that the
upward sweep otherwise drops, and a given root Velocity-set in the downward
sweep, against the hierarchical oracle's own full-Q mode.

* FP64, bodies of 2 to 2,600 beads, tile sizes 4 and 32 (one to many tile
  phases), 1 to 40 right-hand sides (narrow and wide sweeps), both vector
  layouts: Q~ v and Q_Z v, and Q_Z^T r + Q~^T w, against the oracle body by
  body (<= 1e-12 relative per body and RHS for bodies without an
  ill-conditioned node); for every body the round trip Q^T (Q v) = v
  (basis-free, <= 1e-12).
* FP32 on the benchmark's workload (4,096 bodies, R = 32): round trip
  <= 1e-5 and sampled bodies' Q_Z v against the oracle <= 1e-5.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hier

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


def to_layout(a, layout):
    if layout == "rows":
        return np.ascontiguousarray(a)
    return np.ascontiguousarray(a.reshape(a.shape[0] // 3, 3, a.shape[1]).transpose(0, 2, 1))


def from_layout(t, layout):
    if layout == "rows":
        return t
    return np.ascontiguousarray(t.transpose(0, 2, 1).reshape(3 * t.shape[0], t.shape[1]))


def rel(a, b, scale):
    if a.size == 0:
        return 0.0
    return float((np.linalg.norm(a - b, axis=0) / np.maximum(scale, 1e-300)).max())


@pytest.mark.parametrize("S,R,layout", [(32, 1, "rows"), (4, 5, "rows"), (32, 32, "rows"), (4, 40, "triples"),
                                        (32, 32, "triples"), (16, 3, "triples")])
def test_full_q_fp64_against_oracle(hq, S, R, layout):
    w = W.small_batch(31, [2, 3, 4, 7, 33, 129, 500, 1500, 2600])
    rng = np.random.default_rng(40 + R)
    v = rng.standard_normal((3 * w.N, R))
    wv = rng.standard_normal((w.rows, R))
    r = rng.standard_normal((6 * w.m, R))
    print(f"[gpu] full Q S={S} R={R} {layout}", flush=True)
    h = hq.build(_dev(w.pos), w.offsets, tile_units=S)
    up, root = h.apply_full(_dev(to_layout(v, layout)), layout=layout)
    up, root = from_layout(up.cpu().numpy(), layout), from_layout(root.cpu().numpy(), layout)
    dn = from_layout(h.apply_full(_dev(to_layout(wv, layout)), transpose=True, root=_dev(to_layout(r, layout)),
                                  layout=layout).cpu().numpy(), layout)
    # round trip through the full Q (basis-free)
    back = from_layout(h.apply_full(_dev(to_layout(up, layout)), transpose=True, root=_dev(to_layout(root, layout)),
                                    layout=layout).cpu().numpy(), layout)
    assert h.query()["device_flags"] == 0
    assert np.abs(back - v).max() <= 1e-12 * np.abs(v).max() * 10
    rows = h.row_offsets
    for j, b in enumerate(hier.Batch(w.pos, w.offsets).bodies):
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        r0, r1 = rows[j], rows[j + 1]
        vj = v[b0:b1]
        eps_o, root_o = b.apply(vj, root=np.zeros((6, R)))
        out_o, _ = b.apply(wv[r0:r1], transpose=True, root=r[6 * j:6 * j + 6])
        if b.max_kappa > 1e4:
            continue
        scale_v = np.linalg.norm(vj, axis=0)
        assert rel(up[r0:r1], eps_o, scale_v) <= 1e-12
        assert rel(root[6 * j:6 * j + 6], root_o, scale_v) <= 1e-12
        scale_w = np.sqrt(np.linalg.norm(wv[r0:r1], axis=0) ** 2 + np.linalg.norm(r[6 * j:6 * j + 6], axis=0) ** 2)
        assert rel(dn[b0:b1], out_o, scale_w) <= 1e-12


def test_full_q_fp32_bd_workload(hq):
    w = W.bd_m4096()
    rng = np.random.default_rng(43)
    f = rng.standard_normal((3 * w.N, w.nrhs))
    print(f"[gpu] full Q FP32 bd N={w.N}", flush=True)
    h = hq.build(_dev(w.pos), w.offsets, store=2)
    ft = _dev(to_layout(f, "triples"), torch.float32)
    eps, root = h.apply_full(ft, layout="triples")
    back = h.apply_full(eps, transpose=True, root=root, layout="triples")
    assert h.query()["device_flags"] == 0
    back = from_layout(back.cpu().numpy(), "triples").astype(np.float64)
    err = np.linalg.norm(back - f, axis=0) / np.linalg.norm(f, axis=0)
    assert err.max() <= 1e-5
    root = from_layout(root.cpu().numpy(), "triples").astype(np.float64)
    for j in np.random.default_rng(8).choice(w.m, 12, replace=False):
        b0, b1 = w.offsets[j], w.offsets[j + 1]
        bo = hier.Body(w.pos[b0:b1])
        _, root_o = bo.apply(f[3 * b0:3 * b1], root=np.zeros((6, w.nrhs)))
        assert rel(root[6 * j:6 * j + 6], root_o, np.linalg.norm(f[3 * b0:3 * b1], axis=0)) <= 1e-5


def test_full_q_argument_errors(hq):
    w = W.small_batch(32, [10, 20])
    h = hq.build(_dev(w.pos), w.offsets)
    v = torch.zeros((3 * w.N, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        h.apply_full(torch.zeros((w.rows, 2), dtype=torch.float64, device="cuda"), transpose=True)  # no root
    with pytest.raises(ValueError):
        h.apply_full(v, root=torch.zeros((6 * w.m, 3), dtype=torch.float64, device="cuda"))
    from paper_1708_08427_amd import _lib
    import ctypes
    out = torch.zeros((w.rows, 2), dtype=torch.float64, device="cuda")
    st = _lib.load().hq_apply_full(h._h(), ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr()), None, 0,
                                   2, _lib.HQ_FP64, _lib.HQ_ROWS, None)
    assert st == 1
    assert h.query()["device_flags"] == 0
