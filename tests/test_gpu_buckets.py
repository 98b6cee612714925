"""Leaf boxes of up to s beads (hq_options.leaf_size) on the GPU against the
FP64 oracle with the same leaf size, and the fused upward sweep against the
per-phase one.

* Products of FP64 transforms and vectors <= 1e-12 relative per body and
  right-hand side where the oracle's nodes and leaves are well conditioned
  (else the basis-free projector), narrow and wide sweeps, both layouts,
  bodies smaller than a leaf, two-bead bodies.
* FP32 against FP64 <= 1e-5 and the leak; the full Q against the oracle's.
* A rebuild after a rigid motion equals a fresh build bit for bit.
* The fused upward sweep (one launch, arrival counters) equals the per-phase
  launches of the wide sweeps bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, hier

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


def _rel(a, b):
    return float((np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)).max())


SIZES = [2, 3, 5, 9, 16, 17, 40, 700, 1500, 2600]


@pytest.mark.parametrize("s", [2, 3, 4, 8, 11, 16])
@pytest.mark.parametrize("R", [1, 3, 32, 40])
def test_leaf_boxes_fp64_against_oracle(hq, s, R):
    w = W.small_batch(70 + s, SIZES)
    rng = np.random.default_rng(s * 100 + R)
    v = rng.standard_normal((3 * w.N, R))
    g = rng.standard_normal((w.rows, R))
    print(f"[gpu] leaf_size {s} R {R} N={w.N}", flush=True)
    h = hq.build(_dev(w.pos), w.offsets, leaf_size=s, tile_units=16)
    up = h.apply(_dev(v)).cpu().numpy()
    dn = h.apply(_dev(g), transpose=True).cpu().numpy()
    assert h.query()["device_flags"] == 0
    bt = hier.Batch(w.pos, w.offsets, s=s)
    up_o, dn_o = bt.apply(v), bt.apply(g, transpose=True)
    pr = h.apply(h.apply(_dev(v)), transpose=True).cpu().numpy()
    flags, _ = h.body_info()
    checked = 0
    for j, b in enumerate(bt.bodies):
        assert np.array_equal(h.sorted_beads(j), b.perm())
        r0, r1 = h.row_offsets[j], h.row_offsets[j + 1]
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        pj = w.pos[w.offsets[j]:w.offsets[j + 1]]
        assert bool(flags[j] & hq.HQ_BODY_DEGENERATE) == (dense.rank(pj) < 6), (j, flags[j])
        if b.max_kappa <= 1e4:
            if r1 > r0:
                assert _rel(up[r0:r1], up_o[r0:r1]) <= 1e-12, j
            assert _rel(dn[b0:b1], dn_o[b0:b1]) <= 1e-12 or r1 == r0, j
            checked += 1
        if dense.rank(pj) == 6:
            want = dense.project(pj, v[b0:b1])
            assert np.abs(pr[b0:b1] - want).max() <= 1e-12 * max(1.0, np.abs(v[b0:b1]).max())
    assert checked >= len(SIZES) - 1


@pytest.mark.parametrize("s", [4, 8])
def test_leaf_boxes_fp32_layouts_full_q(hq, s):
    w = W.small_batch(90 + s, SIZES)
    rng = np.random.default_rng(s)
    R = 32
    v = rng.standard_normal((3 * w.N, R))
    g = rng.standard_normal((w.rows, R))
    h = hq.build(_dev(w.pos), w.offsets, leaf_size=s)
    up64 = h.apply(_dev(v)).cpu().numpy()
    dn64 = h.apply(_dev(g), transpose=True).cpu().numpy()
    up32 = h.apply(_dev(v, torch.float32)).cpu().numpy().astype(np.float64)
    dn32 = h.apply(_dev(g, torch.float32), transpose=True).cpu().numpy().astype(np.float64)
    for j in range(w.m):
        r0, r1 = h.row_offsets[j], h.row_offsets[j + 1]
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        if r1 > r0:
            assert (np.linalg.norm(up32[r0:r1] - up64[r0:r1], axis=0) / np.linalg.norm(v[b0:b1], axis=0)).max() <= 1e-5
            assert (np.linalg.norm(dn32[b0:b1] - dn64[b0:b1], axis=0) / np.linalg.norm(g[r0:r1], axis=0)).max() <= 1e-5
        assert dense.leak(w.pos[w.offsets[j]:w.offsets[j + 1]], dn32[b0:b1]).max() <= 1e-5
    # the triples layout gives the same values
    vt = _dev(v).reshape(w.N, 3, R).transpose(1, 2).contiguous()
    upt = h.apply(vt, layout="triples").transpose(1, 2).reshape(w.rows, R).cpu().numpy()
    assert np.array_equal(upt, up64)
    # the full Q against the oracle's
    root = np.zeros((6 * w.m, R))
    eps, qz = h.apply_full(_dev(v))
    eps, qz = eps.cpu().numpy(), qz.cpu().numpy()
    bt = hier.Batch(w.pos, w.offsets, s=s)
    for j, b in enumerate(bt.bodies):
        if b.max_kappa > 1e4:
            continue
        _, ro = b.apply(v[3 * w.offsets[j]:3 * w.offsets[j + 1]], root=np.zeros((6, R)))
        assert np.abs(qz[6 * j:6 * j + 6] - ro).max() <= 1e-12 * np.abs(ro).max()
    back = h.apply_full(_dev(eps), transpose=True, root=_dev(qz)).cpu().numpy()
    assert np.abs(back - v).max() <= 1e-12 * np.abs(v).max()
    with pytest.raises(hq.HQError):
        h.explicit(3)
    assert h.query()["device_flags"] == 0


def test_leaf_boxes_rebuild_and_rotation(hq):
    w = W.small_batch(95, SIZES)
    rng = np.random.default_rng(95)
    rot, tr = W.rigid_motions(rng, 1, w.m)
    f = _dev(rng.standard_normal((3 * w.N, 32)))
    pos = _dev(w.pos)
    h = hq.build(pos, w.offsets, leaf_size=6)
    h.rigid_update(pos, _dev(rot.reshape(w.m, 9)), _dev(tr.reshape(w.m, 3)))
    h.rebuild(pos)
    a = h.apply(f)
    fresh = hq.build(pos.clone(), w.offsets, leaf_size=6)
    assert torch.equal(a, fresh.apply(f))
    # products of the moved bodies from the transforms before the motion
    h0 = hq.build(_dev(w.pos), w.offsets, leaf_size=6)
    pr = h0.apply_rotated(_dev(rot.reshape(w.m, 9)), h0.apply_rotated(_dev(rot.reshape(w.m, 9)), f), transpose=True)
    pw = fresh.apply(fresh.apply(f), transpose=True)
    assert float((pr - pw).abs().max()) <= 1e-12 * float(f.abs().max())
    assert h.query()["device_flags"] == 0


@pytest.mark.parametrize("R,layout", [(32, "triples"), (16, "rows"), (40, "rows"), (64, "rows")])
def test_fused_upward_equals_phase_launches(hq, R, layout):
    w = W.small_batch(96, [2, 3, 60, 700, 3000, 9000, 6100, 480])
    rng = np.random.default_rng(R)
    f = _dev(rng.standard_normal((3 * w.N, R)), torch.float32)
    if layout == "triples":
        f = f.reshape(w.N, 3, R).transpose(1, 2).contiguous()
    for S, S2 in ((32, 0), (16, 4), (64, 8)):
        pos = _dev(w.pos)
        a = hq.build(pos, w.offsets, tile_units=S, later_tile_units=S2, sweep_kernel=3)
        b = hq.build(pos, w.offsets, tile_units=S, later_tile_units=S2, fused_upward=1)
        ya, yb = a.apply(f, layout=layout), b.apply(f, layout=layout)
        assert torch.equal(ya, yb)
        # again, with the counters restored by the previous sweep
        assert torch.equal(b.apply(f, layout=layout), ya)
        assert b.query()["device_flags"] == 0
