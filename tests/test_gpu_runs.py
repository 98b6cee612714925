"""Run tables and launch grids of the later tile phases on the GPU.

A later phase of at most 16,384 tiles is swept one tile per run; a phase
with more tiles is cut into runs of several tiles every few nodes.  The grid
of a later phase is sized from the tile count the build found in that phase,
and the kernels stride over whatever a rebuild puts there.

* Many small bodies (one second-phase tile per body root, more than 16,384
  of them): the wide sweeps against the lane-group kernel (the same FP64
  transforms, no run tables) <= 1e-13 per (body, RHS), the larger bodies
  against the oracle <= 1e-12, the projector on a sample <= 1e-12, FP32
  against FP64 <= 1e-5 in the triples layout.
* Batches with few later tiles (later tiles of 32, 16 and 4 units): FP64
  products <= 1e-12 per (body, RHS) against the oracle with the 32-column
  wide sweeps, FP32 against FP64 <= 1e-5 in the triples layout.
* A rebuild onto positions whose tree spreads its nodes over other phases
  than the build's equals a fresh build on those positions bit for bit
  (wide sweeps at 32 RHS, node-parallel and lane kernels at 1 RHS).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, hier
from tests.test_gpu_parity import _dev, check_fp64, rel_per_body

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


def _fp32_vs_fp64_triples(hq, w, R, **opts):
    rng = np.random.default_rng(5)
    v = rng.standard_normal((3 * w.N, R))
    g = rng.standard_normal((w.rows, R))
    h = hq.build(_dev(w.pos), w.offsets, **opts)
    up64 = h.apply(_dev(v)).cpu().numpy()
    dn64 = h.apply(_dev(g), transpose=True).cpu().numpy()
    vt = _dev(v, torch.float32).reshape(w.N, 3, R).transpose(1, 2).contiguous()
    gt = _dev(g, torch.float32).reshape(w.rows // 3, 3, R).transpose(1, 2).contiguous()
    up32 = h.apply(vt, layout="triples").transpose(1, 2).reshape(w.rows, R).cpu().numpy().astype(np.float64)
    dn32 = h.apply(gt, transpose=True, layout="triples").transpose(1, 2).reshape(3 * w.N, R).cpu().numpy()
    dn32 = dn32.astype(np.float64)
    assert h.query()["device_flags"] == 0
    worst = 0.0
    for j in range(w.m):
        r0, r1 = h.row_offsets[j], h.row_offsets[j + 1]
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        if r1 > r0:
            worst = max(worst, float((np.linalg.norm(up32[r0:r1] - up64[r0:r1], axis=0)
                                      / np.linalg.norm(v[b0:b1], axis=0)).max()))
            worst = max(worst, float((np.linalg.norm(dn32[b0:b1] - dn64[b0:b1], axis=0)
                                      / np.linalg.norm(g[r0:r1], axis=0)).max()))
    print(f"[gpu] FP32 triples against FP64: {worst:.2e}", flush=True)
    assert worst <= 1e-5
    return h


def test_later_phase_beyond_run_target(hq):
    # 16,500 bodies of 40 beads: each body root is a second-phase tile of one
    # node above two first-phase tiles, so the second phase holds more tiles
    # than the run-count target and is cut into runs of several tiles.
    # Some of these small bodies have a Q~ basis that the oracle itself moves
    # by up to 3e-12 when their positions change by 1e-15 relatively (the
    # transforms are generated from differences of nearby positions), so the
    # element-wise oracle bar is applied to the larger bodies; every body is
    # compared with the lane-group kernel, which sweeps the same FP64
    # transforms without run tables, and on the basis-free projector.
    w = W.small_batch(7, [40] * 16500 + [300] * 200 + [2, 3])
    R = 32
    rng = np.random.default_rng(11)
    v = rng.standard_normal((3 * w.N, R))
    g = rng.standard_normal((w.rows, R))
    pos = _dev(w.pos)
    h = hq.build(pos, w.offsets, tile_units=32)
    ref = hq.build(pos, w.offsets, tile_units=32, sweep_kernel=1)
    ph = h.node_phase()
    print(f"[gpu] phase sizes {np.bincount(ph).tolist()}", flush=True)
    assert int((ph == 2).sum()) >= 16500
    up, dn = h.apply(_dev(v)).cpu().numpy(), h.apply(_dev(g), transpose=True).cpu().numpy()
    up1, dn1 = ref.apply(_dev(v)).cpu().numpy(), ref.apply(_dev(g), transpose=True).cpu().numpy()
    assert h.query()["device_flags"] == 0 and ref.query()["device_flags"] == 0
    rows, b3 = h.row_offsets, 3 * np.asarray(w.offsets)
    assert rel_per_body(up, up1, w.offsets, rows) <= 1e-13
    assert rel_per_body(dn, dn1, w.offsets, b3) <= 1e-13
    # the oracle on the 300-bead bodies and the two smallest
    sel = list(range(16500, w.m))
    parts = [w.pos[w.offsets[j]:w.offsets[j + 1]] for j in sel]
    so = np.concatenate([[0], np.cumsum([len(p) for p in parts])])
    bt = hier.Batch(np.concatenate(parts), so)
    vs = np.concatenate([v[b3[j]:b3[j + 1]] for j in sel])
    gs = np.concatenate([g[rows[j]:rows[j + 1]] for j in sel])
    up_o, dn_o = bt.apply(vs), bt.apply(gs, transpose=True)
    ro = np.concatenate([[0], np.cumsum([rows[j + 1] - rows[j] for j in sel])])
    checked = 0
    for i, j in enumerate(sel):
        if bt.bodies[i].max_kappa > 1e4:
            continue
        if rows[j + 1] > rows[j]:
            assert rel_per_body(up[rows[j]:rows[j + 1]], up_o[ro[i]:ro[i + 1]], [0, 1], [0, ro[i + 1] - ro[i]]) <= 1e-12
            assert rel_per_body(dn[b3[j]:b3[j + 1]], dn_o[3 * so[i]:3 * so[i + 1]], [0, 1],
                                [0, 3 * (so[i + 1] - so[i])]) <= 1e-12
        checked += 1
    assert checked >= len(sel) - 2
    # the projector on every 8th body
    pr = h.apply(h.apply(_dev(v)), transpose=True).cpu().numpy()
    for j in range(0, w.m, 8):
        pj = w.pos[w.offsets[j]:w.offsets[j + 1]]
        if dense.rank(pj) < 6:
            continue
        want = dense.project(pj, v[b3[j]:b3[j + 1]])
        assert np.abs(pr[b3[j]:b3[j + 1]] - want).max() <= 1e-12 * max(1.0, np.abs(v[b3[j]:b3[j + 1]]).max())
    _fp32_vs_fp64_triples(hq, w, R, tile_units=32)


@pytest.mark.parametrize("S2", [32, 16, 4])
def test_later_phase_one_run_per_tile(hq, S2):
    rng = np.random.default_rng(S2)
    sizes = np.clip(np.round(rng.lognormal(np.log(500.0), 0.8, 300)), 2, 6000).astype(int).tolist()
    w = W.small_batch(40 + S2, sizes)
    check_fp64(hq, w, S=32, nrhs=32, S2=S2, min_checked=len(sizes) - 3)
    _fp32_vs_fp64_triples(hq, w, 32, tile_units=32, later_tile_units=S2)


@pytest.mark.parametrize("R", [32, 1])
def test_rebuild_moves_nodes_between_phases(hq, R):
    sizes = [2, 3, 70, 700, 2500, 5000, 1200, 40, 9000]
    a = W.small_batch(61, sizes)
    # the same bodies, each bunched into a few tight clusters: a different
    # tree shape, so the rebuild's nodes fall into other phases
    rng = np.random.default_rng(62)
    pos = a.pos.copy()
    for j in range(a.m):
        o0, o1 = a.offsets[j], a.offsets[j + 1]
        n = o1 - o0
        centers = rng.uniform(0.0, 100.0, (max(1, n // 300), 3))
        pos[o0:o1] = centers[rng.integers(0, len(centers), n)] + 0.5 * rng.standard_normal((n, 3))
    # phases reserved generously: the rebuild may need more than the build
    opts = dict(tile_units=16, later_tile_units=4, max_phases=24)
    h = hq.build(_dev(a.pos), a.offsets, **opts)
    ph0 = h.node_phase()
    p = _dev(pos)
    h.rebuild(p)
    fresh = hq.build(p.clone(), a.offsets, **opts)
    ph1 = fresh.node_phase()
    print(f"[gpu] phases built {np.bincount(ph0).tolist()} after the move {np.bincount(ph1).tolist()}", flush=True)
    assert not np.array_equal(ph0, ph1)
    f = _dev(np.random.default_rng(R).standard_normal((3 * a.N, R)), torch.float32)
    wv = _dev(np.random.default_rng(R + 1).standard_normal((a.rows, R)), torch.float32)
    assert torch.equal(h.apply(f), fresh.apply(f))
    assert torch.equal(h.apply(wv, transpose=True), fresh.apply(wv, transpose=True))
    assert h.query()["device_flags"] == 0 and fresh.query()["device_flags"] == 0
