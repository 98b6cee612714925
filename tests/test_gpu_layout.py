"""Vectors in the triples layout (hq_apply_layout with HQ_TRIPLES): each row
triple's R right-hand sides stored as R contiguous 3-vectors.

* Small batches, R = 1 .. 70 (narrow and wide sweeps), FP64 against the
  hierarchical oracle (<= 1e-12 relative 2-norm per body and RHS).
* The same products as the rows layout, bit for bit: the layout changes only
  where values are read and written, not the arithmetic.
* The benchmark's workload (4,096 bodies, R = 32, FP32 and FP64 wide sweeps)
  after a rigid motion and a rebuild: triples and rows agree bit for bit.
* Argument errors: an unknown layout and ill-shaped tensors are rejected.
"""
import ctypes

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


def to_triples(a):
    """(3T, R) rows -> (T, R, 3) triples."""
    return np.ascontiguousarray(a.reshape(a.shape[0] // 3, 3, a.shape[1]).transpose(0, 2, 1))


def from_triples(t):
    """(T, R, 3) triples -> (3T, R) rows."""
    return np.ascontiguousarray(t.transpose(0, 2, 1).reshape(3 * t.shape[0], t.shape[1]))


def rel_per_body(a, b, offsets):
    worst = 0.0
    for j in range(len(offsets) - 1):
        r0, r1 = offsets[j], offsets[j + 1]
        if r1 == r0:
            continue
        d = np.linalg.norm(a[r0:r1] - b[r0:r1], axis=0)
        n = np.maximum(np.linalg.norm(b[r0:r1], axis=0), 1e-300)
        worst = max(worst, float((d / n).max()))
    return worst


def test_layout_converters_are_inverse():
    a = np.arange(6 * 5, dtype=np.float64).reshape(6, 5)
    t = to_triples(a)
    assert t.shape == (2, 5, 3)
    assert t[1, 4, 2] == a[5, 4] and t[0, 2, 1] == a[1, 2]
    assert np.array_equal(from_triples(t), a)


@pytest.mark.parametrize("R", [1, 5, 16, 32, 64, 70])
def test_triples_fp64_against_oracle_and_rows(hq, R):
    w = W.small_batch(12, [40, 700, 1200])
    rng = np.random.default_rng(200 + R)
    v = rng.standard_normal((3 * w.N, R))
    wv = rng.standard_normal((w.rows, R))
    print(f"[gpu] triples R={R} N={w.N}", flush=True)
    h = hq.build(_dev(w.pos), w.offsets, tile_units=128)
    bt = hier.Batch(w.pos, w.offsets)
    up_o, dn_o = bt.apply(v), bt.apply(wv, transpose=True)
    up_t = from_triples(h.apply(_dev(to_triples(v)), layout="triples").cpu().numpy())
    dn_t = from_triples(h.apply(_dev(to_triples(wv)), transpose=True, layout="triples").cpu().numpy())
    assert h.query()["device_flags"] == 0
    assert rel_per_body(up_t, up_o, h.row_offsets) <= 1e-12
    assert rel_per_body(dn_t, dn_o, 3 * np.asarray(w.offsets)) <= 1e-12
    up_r = h.apply(_dev(v)).cpu().numpy()
    dn_r = h.apply(_dev(wv), transpose=True).cpu().numpy()
    assert np.array_equal(up_t, up_r)
    assert np.array_equal(dn_t, dn_r)
    # FP32: the same bits as the rows layout
    up32_t = from_triples(h.apply(_dev(to_triples(v), torch.float32), layout="triples").cpu().numpy())
    up32_r = h.apply(_dev(v, torch.float32)).cpu().numpy()
    assert np.array_equal(up32_t, up32_r)
    assert h.query()["device_flags"] == 0


def test_triples_bd_workload_equals_rows(hq):
    w = W.bd_m4096()
    rng = np.random.default_rng(41)
    f = rng.standard_normal((3 * w.N, w.nrhs))
    rot, trans = W.rigid_motions(rng, 1, w.m)
    pos = _dev(w.pos)
    print(f"[gpu] triples bd N={w.N} m={w.m} R={w.nrhs}", flush=True)
    h = hq.build(pos, w.offsets, store=3)
    h.rigid_update(pos, _dev(rot.reshape(1, w.m, 9)[0]), _dev(trans[0]))
    h.rebuild(pos)
    for dt in (torch.float32, torch.float64):
        fr = _dev(f, dt)
        ft = _dev(to_triples(f), dt)
        yr = h.apply(fr)
        yt = h.apply(ft, layout="triples")
        assert np.array_equal(from_triples(yt.cpu().numpy()), yr.cpu().numpy())
        zr = h.apply(yr, transpose=True)
        zt = h.apply(yt, transpose=True, layout="triples")
        assert np.array_equal(from_triples(zt.cpu().numpy()), zr.cpu().numpy())
    assert h.query()["device_flags"] == 0


def test_triples_timed_matches_untimed(hq):
    w = W.small_batch(14, [300, 2000])
    rng = np.random.default_rng(3)
    v = _dev(to_triples(rng.standard_normal((3 * w.N, 32))), torch.float32)
    h = hq.build(_dev(w.pos), w.offsets)
    a = h.apply(v, layout="triples")
    b, ms = h.apply(v, layout="triples", timed=True)
    assert torch.equal(a, b)
    assert len(ms) >= h.query()["phases"] >= 1
    assert all(t >= 0 for t in ms)


def test_layout_argument_errors(hq):
    from paper_1708_08427_amd import _lib
    w = W.small_batch(15, [50, 60])
    h = hq.build(_dev(w.pos), w.offsets)
    v = torch.zeros((w.N, 4, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        h.apply(v, layout="columns")
    with pytest.raises(ValueError):
        h.apply(v.reshape(3 * w.N, 4), layout="triples")  # rows-shaped tensor
    with pytest.raises(ValueError):
        h.apply(v.transpose(1, 2).contiguous(), layout="triples")  # (N, 3, R)
    out = torch.zeros((w.rows // 3, 4, 3), dtype=torch.float64, device="cuda")
    lib = _lib.load()
    st = lib.hq_apply_layout(h._h(), ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(out.data_ptr()), 0, 4,
                             _lib.HQ_FP64, 2, None)
    assert st == 1 and b"layout" in lib.hq_last_error()
    assert h.query()["device_flags"] == 0
