"""Node-parallel sweeps (hq_options.sweep_kernel = 2 in every phase; the
automatic choice in the phases after the first): a lane per (node,
right-hand side), each tile's levels resolved in LDS.

* FP64 products against the oracle <= 1e-12 per (body, RHS) for tiles of 2 to
  64 units, separate later-phase tile sizes, 1 to 40 right-hand sides (column
  passes of up to 8), both layouts, bodies of 2 to 2,600 beads.
* Against the lane-group-per-tile kernel (sweep_kernel = 1) and the wide
  sweeps on the benchmark's workload (FP64 <= 1e-13, FP32 <= 1e-5).
* Tiles above 64 units fall back to the lane group per tile; leaf boxes and
  the full Q go through the node-parallel phases above them.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hier
from tests.test_gpu_parity import _dev, build, check_fp64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


SIZES = [2, 3, 4, 7, 33, 129, 500, 1500, 2600]


@pytest.mark.parametrize("S,S2", [(2, 0), (4, 0), (16, 0), (32, 0), (64, 0), (32, 4), (64, 16), (8, 64)])
def test_np_fp64_tile_sizes(hq, S, S2):
    w = W.small_batch(11, SIZES)
    for R in (1, 3):
        h = check_fp64(hq, w, S=S, nrhs=R, S2=S2, sweep_kernel=2)
        assert h.query()["phases"] >= 1


@pytest.mark.parametrize("R", [1, 2, 5, 8, 13, 40])
def test_np_fp64_nrhs(hq, R):
    """Column passes of up to 8 right-hand sides."""
    w = W.small_batch(12, [40, 700, 1200, 3])
    check_fp64(hq, w, S=32, nrhs=R, sweep_kernel=2)


def test_np_automatic_below_8(hq):
    """The automatic choice at 1 and 5 right-hand sides (node-parallel) against
    the oracle, and a tile size above 64 units (lane group per tile)."""
    w = W.small_batch(14, SIZES)
    check_fp64(hq, w, S=32, nrhs=1)
    check_fp64(hq, w, S=128, nrhs=5)
    check_fp64(hq, w, S=16, S2=128, nrhs=1)


@pytest.mark.parametrize("layout", ["rows", "triples"])
def test_np_layouts_and_full_q(hq, layout):
    w = W.small_batch(15, [3, 90, 700, 2300])
    rng = np.random.default_rng(15)
    R = 3
    v = rng.standard_normal((3 * w.N, R))
    h = build(hq, w, tile_units=16, sweep_kernel=2)
    bt = hier.Batch(w.pos, w.offsets)
    vt = _dev(v)
    if layout == "triples":
        vt = vt.reshape(w.N, 3, R).transpose(1, 2).contiguous()
    eps, qz = h.apply_full(vt, layout=layout)
    if layout == "triples":
        eps = eps.transpose(1, 2).reshape(w.rows, R)
        qz = qz.transpose(1, 2).reshape(6 * w.m, R)
    eps, qz = eps.cpu().numpy(), qz.cpu().numpy()
    for j, b in enumerate(bt.bodies):
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        e_o, r_o = b.apply(v[b0:b1], root=np.zeros((6, R)))
        r0, r1 = h.row_offsets[j], h.row_offsets[j + 1]
        assert np.abs(eps[r0:r1] - e_o).max() <= 1e-12 * np.abs(e_o).max()
        assert np.abs(qz[6 * j:6 * j + 6] - r_o).max() <= 1e-12 * np.abs(r_o).max()
    back = h.apply_full(_dev(eps), transpose=True, root=_dev(qz)).cpu().numpy()
    assert np.abs(back - v).max() <= 1e-12 * np.abs(v).max()
    assert h.query()["device_flags"] == 0


@pytest.mark.parametrize("s", [4, 8])
def test_np_above_leaf_boxes(hq, s):
    """Leaf boxes (the first phase) under node-parallel later phases."""
    w = W.small_batch(16 + s, SIZES)
    rng = np.random.default_rng(s)
    v = rng.standard_normal((3 * w.N, 1))
    g = rng.standard_normal((w.rows, 1))
    h = build(hq, w, leaf_size=s, tile_units=16, sweep_kernel=2)
    up = h.apply(_dev(v)).cpu().numpy()
    dn = h.apply(_dev(g), transpose=True).cpu().numpy()
    bt = hier.Batch(w.pos, w.offsets, s=s)
    up_o, dn_o = bt.apply(v), bt.apply(g, transpose=True)
    checked = 0
    for j, b in enumerate(bt.bodies):
        if b.max_kappa > 1e4:
            continue
        r0, r1 = h.row_offsets[j], h.row_offsets[j + 1]
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        if r1 > r0:
            assert np.linalg.norm(up[r0:r1] - up_o[r0:r1]) <= 1e-12 * np.linalg.norm(up_o[r0:r1])
            assert np.linalg.norm(dn[b0:b1] - dn_o[b0:b1]) <= 1e-12 * np.linalg.norm(dn_o[b0:b1])
        checked += 1
    assert checked >= len(SIZES) - 1
    assert h.query()["device_flags"] == 0


def test_np_against_other_kernels_bd(hq):
    """The benchmark's workload at 4 right-hand sides: node-parallel, lane
    group per tile, and the wide sweeps' columns agree."""
    w = W.bd_m4096()
    rng = np.random.default_rng(9)
    f = rng.standard_normal((3 * w.N, 4))
    g = rng.standard_normal((w.rows, 4))
    pos = _dev(w.pos)
    hn = hq.build(pos, w.offsets, store=3, sweep_kernel=2)
    hl = hq.build(pos, w.offsets, store=3, sweep_kernel=1)
    for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
        a = hn.apply(_dev(f, dt)).double().cpu().numpy()
        b = hl.apply(_dev(f, dt)).double().cpu().numpy()
        assert np.abs(a - b).max() <= tol * np.abs(f).max()
        a = hn.apply(_dev(g, dt), transpose=True).double().cpu().numpy()
        b = hl.apply(_dev(g, dt), transpose=True).double().cpu().numpy()
        assert np.abs(a - b).max() <= tol * np.abs(g).max()
    # the automatic choice (the first phase with the lane-per-tile kernels of
    # exact wait counts, node-parallel later phases) against both, at 1 and 3
    # right-hand sides, in both precisions and directions
    ha = hq.build(pos, w.offsets, store=3)
    for R in (1, 3):
        for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
            fr, gr = _dev(f[:, :R], dt), _dev(g[:, :R], dt)
            a, b = ha.apply(fr), ha.apply(gr, transpose=True)
            for hx in (hn, hl):
                assert float((a - hx.apply(fr)).abs().max()) <= tol * float(fr.abs().max()), (R, dt)
                assert float((b - hx.apply(gr, transpose=True)).abs().max()) <= tol * float(gr.abs().max()), (R, dt)
    assert ha.query()["device_flags"] == 0
    assert hn.query()["device_flags"] == 0 and hl.query()["device_flags"] == 0


def test_np_results_independent_of_tile_size(hq):
    """Same arithmetic per node: FP64 results agree bitwise across tile sizes."""
    w = W.small_batch(13, [300, 900, 2000])
    rng = np.random.default_rng(5)
    v = _dev(rng.standard_normal((3 * w.N, 2)))
    outs = [build(hq, w, tile_units=S, later_tile_units=S2, sweep_kernel=2).apply(v).cpu().numpy()
            for S, S2 in ((4, 0), (16, 0), (64, 0), (32, 4), (8, 64))]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
