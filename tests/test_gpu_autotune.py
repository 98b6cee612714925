"""The autotuner (hq_autotune): it returns one of its candidate launch
configurations, remembers it per workload, and a handle built with the chosen
options computes the same products (FP64 against the oracle, FP32 bitwise
equal to the default configuration's, since the arithmetic per node does not
depend on how tiles are grouped into runs or waves)."""
import numpy as np
import pytest

import workloads as W
from oracle import hier

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


def test_autotune_picks_a_candidate_and_keeps_parity(hq):
    w = W.small_batch(31, [2, 3, 60, 400, 1300, 2500, 900, 700, 5000], nrhs=32)
    rng = np.random.default_rng(31)
    f = rng.standard_normal((3 * w.N, 32))
    pos = torch.from_numpy(w.pos).cuda()
    print(f"[gpu] autotune N={w.N} m={w.m}", flush=True)
    t = hq.autotune(pos, w.offsets, 32, torch.float32, include_rebuild=True)
    assert t["tile_units"] in (16, 32, 64)
    assert t["run_nodes"] in (32, 48, 64)
    assert t["waves_per_cu"] in (8, 16, 32)
    assert t["ms"] > 0.0
    assert hq.autotune(pos, w.offsets, 32, torch.float32, include_rebuild=True) == t
    opts = {k: t[k] for k in ("tile_units", "run_nodes", "waves_per_cu")}
    h = hq.build(pos, w.offsets, store=3, **opts)
    up64 = h.apply(torch.from_numpy(f).cuda()).cpu().numpy()
    bt = hier.Batch(w.pos, w.offsets)
    ref = bt.apply(f)
    rows = h.row_offsets
    for j, b in enumerate(bt.bodies):
        if b.max_kappa > 1e4:
            continue
        r0, r1 = rows[j], rows[j + 1]
        e = np.linalg.norm(up64[r0:r1] - ref[r0:r1], axis=0) / np.maximum(np.linalg.norm(ref[r0:r1], axis=0), 1e-300)
        assert e.max() <= 1e-12
    # FP32: same results as the default run length and grid at the same tile size
    f32 = torch.from_numpy(f).float().cuda()
    h2 = hq.build(pos, w.offsets, store=2, tile_units=opts["tile_units"])
    a = h.apply(f32)
    b2 = h2.apply(f32)
    assert torch.equal(a, b2)
    assert torch.equal(h.apply(a, transpose=True), h2.apply(b2, transpose=True))
    assert h.query()["device_flags"] == 0 and h2.query()["device_flags"] == 0
