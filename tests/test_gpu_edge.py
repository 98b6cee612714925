"""Edge cases of the method on the GPU path, through the C ABI.

* Collinear bodies (Section 2.2: Z has rank 5, so Q~ spans 3n-6 of the 3n-5
  dimensions of the complement): flagged HQ_BODY_DEGENERATE, no NaN, rows
  still orthonormal and orthogonal to Z, trace(P) - trace(Q~^T Q~) = 1 against
  the dense LAPACK projector; the regular bodies of the same batch match the
  hierarchical oracle element by element.
* Duplicate and coincident beads (equal codes split by the sorted position):
  bead order and tree bit-exact against the oracle, products against the
  oracle (element-wise where its nodes are well conditioned, else on the
  basis-free projector).
* Non-finite positions: hq_build fails with HQ_E_INVALID; hq_rebuild raises
  HQ_FLAG_NONFINITE.  hq_explicit above the dense limit: HQ_E_UNSUPPORTED.
* The 4,194,304-bead clustered body: bead order and tree bit-exact against
  the oracle at full size, and the block-sparse explicit Q~ in FP32 (value
  count, and blocks times v equal to the sweep on sampled blocks).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, hier

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HQ_E_INVALID = 1
HQ_E_UNSUPPORTED = 5


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


def _build(hq, w, **kw):
    print(f"[gpu] build {w.name} N={w.N} m={w.m} {kw}", flush=True)
    return hq.build(_dev(w.pos), w.offsets, **kw)


def _rel(a, b):
    return float((np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)).max())


def _gpu_tree(nd, j, n):
    """(first, last, split) of body j's internal nodes from hq_node_data,
    split = last sorted position of the x child, sorted by first then last."""
    sel = np.nonzero(nd["body"] == j)[0]
    first, last, x = nd["first"][sel], nd["last"][sel], nd["x"][sel]
    # x child: >= 0 a node index local to the body, < 0 a leaf -(pos) - 1
    base = sel.min() if len(sel) else 0
    split = np.where(x >= 0, nd["last"][np.clip(x, 0, None) + base], -(x + 1))
    t = np.stack([first, last, split], axis=1).astype(np.int64)
    return t[np.lexsort((t[:, 1], t[:, 0]))]


def _oracle_tree(b):
    f, l, s = b.tree()
    t = np.stack([f, l, s], axis=1)
    return t[np.lexsort((t[:, 1], t[:, 0]))]


MIXED = [("ellipsoid", 100), ("collinear", 3), ("ellipsoid", 700), ("collinear", 20),
         ("collinear", 500), ("ellipsoid", 64), ("collinear", 2), ("ellipsoid", 1500)]


@pytest.mark.parametrize("S", [8, 32])
def test_collinear_bodies_in_a_batch(hq, S):
    w = W.mixed_batch(21, MIXED)
    h = _build(hq, w, tile_units=S)
    q = h.query()
    assert q["device_flags"] == 0
    flags, kappa = h.body_info()
    bt = hier.Batch(w.pos, w.offsets)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3 * w.N, 3))
    g = rng.standard_normal((w.rows, 3))
    up = h.apply(_dev(v)).cpu().numpy()
    dn = h.apply(_dev(g), transpose=True).cpu().numpy()
    up32 = h.apply(_dev(v, torch.float32)).cpu().numpy()
    dn32 = h.apply(_dev(g, torch.float32), transpose=True).cpu().numpy()
    for a in (up, dn, up32, dn32):
        assert np.isfinite(a).all()
    up_o, dn_o = bt.apply(v), bt.apply(g, transpose=True)
    rows, beads3 = h.row_offsets, 3 * w.offsets
    ndeg = 0
    for j, (kind, n) in enumerate(MIXED):
        pj = w.pos[w.offsets[j]:w.offsets[j + 1]]
        r0, r1, b0, b1 = rows[j], rows[j + 1], beads3[j], beads3[j + 1]
        degenerate = dense.rank(pj) < 6
        assert degenerate == (kind == "collinear")
        assert bool(flags[j] & hq.HQ_BODY_DEGENERATE) == degenerate, (j, kind, flags[j], kappa[j])
        if not degenerate:
            assert bt.bodies[j].max_kappa <= 1e4
            assert _rel(up[r0:r1], up_o[r0:r1]) <= 1e-12
            assert _rel(dn[b0:b1], dn_o[b0:b1]) <= 1e-12
            continue
        ndeg += 1
        if n == 2:
            assert r1 == r0
            continue
        Q = h.explicit(j).cpu().numpy()
        assert np.isfinite(Q).all()
        # orthonormal rows, orthogonal to Z's row space
        assert np.abs(Q @ Q.T - np.eye(3 * n - 6)).max() <= 1e-12
        Z = dense.zmatrix_centroid(pj)
        assert np.linalg.norm(Z @ Q.T, 2) <= 1e-12 * np.linalg.norm(Z, 2)
        # the complement has 3n - 5 dimensions, Q~ spans 3n - 6 of them
        P = dense.projector(pj)
        assert abs(np.trace(P) - np.trace(Q.T @ Q) - 1.0) <= 1e-9
        # the sweeps apply that same Q~
        assert np.abs(up[r0:r1] - Q @ v[b0:b1]).max() <= 1e-12 * np.abs(v[b0:b1]).sum(axis=0).max()
        assert np.abs(dn[b0:b1] - Q.T @ g[r0:r1]).max() <= 1e-12 * np.abs(g[r0:r1]).sum(axis=0).max()
    assert ndeg == 4
    assert q["degenerate_bodies"] == ndeg


DUPS = [("duplicates", 300), ("ellipsoid", 200), ("cluster", 400), ("point", 8), ("point", 2),
        ("duplicates", 2500), ("point", 3)]


@pytest.mark.parametrize("S", [4, 32])
def test_duplicate_and_coincident_beads(hq, S):
    w = W.mixed_batch(22, DUPS)
    h = _build(hq, w, tile_units=S)
    assert h.query()["device_flags"] == 0
    flags, _ = h.body_info()
    nd = h.node_data(with_G=False, with_geometry=False)
    bt = hier.Batch(w.pos, w.offsets)
    rng = np.random.default_rng(4)
    v = rng.standard_normal((3 * w.N, 2))
    g = rng.standard_normal((w.rows, 2))
    up = h.apply(_dev(v)).cpu().numpy()
    dn = h.apply(_dev(g), transpose=True).cpu().numpy()
    pr = h.apply(h.apply(_dev(v)), transpose=True).cpu().numpy()
    assert np.isfinite(up).all() and np.isfinite(dn).all() and np.isfinite(pr).all()
    up_o, dn_o = bt.apply(v), bt.apply(g, transpose=True)
    rows, beads3 = h.row_offsets, 3 * w.offsets
    compared = projected = 0
    for j, (kind, n) in enumerate(DUPS):
        b = bt.bodies[j]
        pj = w.pos[w.offsets[j]:w.offsets[j + 1]]
        # index work: bit-exact
        assert np.array_equal(h.sorted_beads(j), b.perm())
        assert np.array_equal(_gpu_tree(nd, j, n), _oracle_tree(b))
        r0, r1, b0, b1 = rows[j], rows[j + 1], beads3[j], beads3[j + 1]
        full_rank = dense.rank(pj) == 6
        assert bool(flags[j] & hq.HQ_BODY_DEGENERATE) == (not full_rank), (j, kind)
        if b.max_kappa <= 1e4:
            assert _rel(up[r0:r1], up_o[r0:r1]) <= 1e-12
            assert _rel(dn[b0:b1], dn_o[b0:b1]) <= 1e-12
            compared += 1
        if full_rank:
            want = dense.project(pj, v[b0:b1])
            assert np.abs(pr[b0:b1] - want).max() <= 1e-12 * max(1.0, np.abs(v[b0:b1]).max())
            projected += 1
        elif n > 2:
            Q = h.explicit(j).cpu().numpy()
            assert np.abs(Q @ Q.T - np.eye(3 * n - 6)).max() <= 1e-12
            Z = dense.zmatrix_centroid(pj)
            assert np.linalg.norm(Z @ Q.T) <= 1e-12 * max(np.linalg.norm(Z), 1.0)
    print(f"[gpu] element-wise {compared}, projector {projected} of {len(DUPS)} bodies", flush=True)
    assert projected == 4


def test_nonfinite_positions(hq):
    w = W.small_batch(23, [50, 300, 20])
    for bad in (np.nan, np.inf, -np.inf):
        pos = w.pos.copy()
        pos[317, 1] = bad
        with pytest.raises(hq.HQError) as e:
            hq.build(_dev(pos), w.offsets)
        assert e.value.status == HQ_E_INVALID
    # a valid handle rebuilt on a non-finite position raises the device flag
    h = _build(hq, w)
    assert h.query()["device_flags"] == 0
    pos = w.pos.copy()
    pos[5, 2] = np.nan
    h.rebuild(_dev(pos))
    assert h.query()["device_flags"] & hq.HQ_FLAG_NONFINITE


def test_explicit_above_dense_limit(hq):
    w = W.small_batch(24, [40, 200])
    h = _build(hq, w, explicit_dense_max_n=100)
    assert h.explicit(0).shape == (114, 120)
    with pytest.raises(hq.HQError) as e:
        h.explicit(1)
    assert e.value.status == HQ_E_UNSUPPORTED


def test_large_clustered_tree_and_explicit_blocks(hq):
    """Full size: index work bit-exact, explicit blocks in FP32."""
    w = W.large_clustered()
    h = _build(hq, w)
    assert h.query()["device_flags"] == 0
    b = hier.Body(w.pos)
    print("[gpu] oracle tree built", flush=True)
    assert np.array_equal(h.sorted_beads(0), b.perm())
    nd = h.node_data(with_G=False, with_geometry=False)
    assert np.array_equal(_gpu_tree(nd, 0, w.N), _oracle_tree(b))
    del nd
    print("[gpu] tree bit-exact", flush=True)
    nb, nv = h.explicit_blocks_size(0)
    vals, val_off, row_off, bead_first, rows, cols = h.explicit_blocks(0, dtype=torch.float32)
    torch.cuda.synchronize()
    assert len(rows) == nb and val_off[-1] == nv
    assert nv == int(np.sum(rows.astype(np.int64) * cols.astype(np.int64)))
    print(f"[gpu] explicit blocks: {nb} blocks, {nv} values", flush=True)
    rng = np.random.default_rng(45)
    v = rng.standard_normal((3 * w.N, 1))
    vd = _dev(v, torch.float32)
    ref = h.apply(vd).reshape(-1)
    sb = torch.from_numpy(h.sorted_beads(0)).cuda()
    pick = np.concatenate([np.argsort(cols)[-8:], rng.choice(nb, 2000, replace=False)])
    worst = 0.0
    for bi in pick:
        r, c = int(rows[bi]), int(cols[bi])
        blk = vals[int(val_off[bi]):int(val_off[bi + 1])].reshape(r, c).double()
        beads = sb[int(bead_first[bi]):int(bead_first[bi]) + c // 3]
        idx = (3 * beads[:, None] + torch.arange(3, device="cuda")[None, :]).reshape(-1)
        got = blk @ vd.reshape(-1)[idx].double()
        want = ref[int(row_off[bi]):int(row_off[bi]) + r].double()
        worst = max(worst, float((got - want).norm() / vd.reshape(-1)[idx].double().norm()))
    print(f"[gpu] blocks x v against the sweep: {worst:.2e}", flush=True)
    assert worst <= 1e-5
