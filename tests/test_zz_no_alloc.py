"""hq_apply_noalloc (the exchange buffer in a static device array, no device
allocation) against hq_apply_layout on the same handle: the same kernels, so
the products agree bit for bit; and the FP64 products against the oracle
(<= 1e-12 relative per body and right-hand side).  Two calls in a row, the
second with a smaller input (fewer right-hand sides, then a smaller batch),
so the second call reuses the array the first one filled."""
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


def _rel(a, b):
    return float((np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)).max())


def _check(hq, w, h, R, dtype, layout, rng, oracle=None):
    v = rng.standard_normal((3 * w.N, R))
    g = rng.standard_normal((w.rows, R))
    vd = torch.from_numpy(v).to(dtype).cuda()
    gd = torch.from_numpy(g).to(dtype).cuda()
    if layout == "triples":
        vd = vd.reshape(w.N, 3, R).transpose(1, 2).contiguous()
        gd = gd.reshape(w.rows // 3, 3, R).transpose(1, 2).contiguous()
    # the noalloc call first, so the static array holds the previous call's
    # entries when it starts
    up_n = h.apply(vd, layout=layout, noalloc=True)
    dn_n = h.apply(gd, transpose=True, layout=layout, noalloc=True)
    up = h.apply(vd, layout=layout)
    dn = h.apply(gd, transpose=True, layout=layout)
    torch.cuda.synchronize()
    assert torch.equal(up_n, up) and torch.equal(dn_n, dn)
    assert h.query()["device_flags"] == 0
    if oracle is not None:
        if layout == "triples":
            up = up.transpose(1, 2).reshape(w.rows, R)
            dn = dn.transpose(1, 2).reshape(3 * w.N, R)
        up, dn = up.double().cpu().numpy(), dn.double().cpu().numpy()
        up_o, dn_o = oracle.apply(v), oracle.apply(g, transpose=True)
        tol = 1e-12 if dtype == torch.float64 else 1e-5
        for j in range(w.m):
            r0, r1 = h.row_offsets[j], h.row_offsets[j + 1]
            b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
            if r1 > r0:
                assert _rel(up[r0:r1], up_o[r0:r1]) <= tol
                assert _rel(dn[b0:b1], dn_o[b0:b1]) <= tol


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_noalloc_matches_apply_two_calls(hq, dtype):
    dt = getattr(torch, dtype)
    rng = np.random.default_rng(91)
    big = W.small_batch(92, [2, 3, 40, 700, 1500, 2600, 900])
    small = W.small_batch(93, [5, 300, 64])
    hb = hq.build(torch.from_numpy(big.pos).cuda(), big.offsets, tile_units=16)
    hs = hq.build(torch.from_numpy(small.pos).cuda(), small.offsets, tile_units=16)
    ob, os_ = hier.Batch(big.pos, big.offsets), hier.Batch(small.pos, small.offsets)
    print(f"[gpu] noalloc {dtype}: big N={big.N} then R=40 -> R=3 -> small N={small.N}", flush=True)
    # wide sweeps (40 RHS), then narrow ones (3 RHS) on the same handle, then
    # a smaller handle
    _check(hq, big, hb, 40, dt, "rows", rng, ob)
    _check(hq, big, hb, 3, dt, "rows", rng, ob)
    _check(hq, small, hs, 2, dt, "rows", rng, os_)
    _check(hq, big, hb, 32, dt, "triples", rng, ob)
    _check(hq, small, hs, 32, dt, "triples", rng, os_)


def test_noalloc_bench_workload_and_limit(hq):
    """The benchmark's workload (4,096 bodies, 32 FP32 right-hand sides,
    triples layout) fits the static array; 64 right-hand sides do not and
    are refused before anything is launched."""
    w = W.bd_m4096()
    h = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets, store=2)
    print(f"[gpu] noalloc bench workload tiles={h.query()['tiles']}", flush=True)
    rng = np.random.default_rng(94)
    _check(hq, w, h, 32, torch.float32, "triples", rng)
    v = torch.zeros((w.N, 64, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(hq.HQError) as e:
        h.apply(v, layout="triples", noalloc=True)
    assert e.value.status == 5
    # a smaller call after the refused one still matches
    _check(hq, w, h, 32, torch.float32, "triples", rng)
