"""hq_build_into: a handle whose device state lives in caller (torch) memory.

Its products, tree and explicit blocks equal those of a hq_build handle bit
for bit, its Krylov solve to rounding (the solve's dot products add partial
sums in no fixed order), and the library allocates no device memory for
it: the device's free memory (hipMemGetInfo) does not move across the build,
sweeps in both precisions and layouts, a rebuild after a rigid motion, the
explicit blocks and the Krylov solve.  Requests beyond the reserved sizes
fail instead of allocating."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HQ_E_INVALID, HQ_E_UNSUPPORTED = 1, 5


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


def _run(hq, h, pos, rot, tr, f64, g64, f32t, g32t, out):
    """Every kind of call on a handle; results into the preallocated ``out``."""
    h.apply(f64, out=out["up64"])
    h.apply(g64, transpose=True, out=out["dn64"])
    h.apply(f32t, layout="triples", out=out["up32"])
    h.apply(g32t, transpose=True, layout="triples", out=out["dn32"])
    h.apply_full(f64, root=out["root"], out=out["full"])
    h.rigid_update(pos, rot, tr)
    h.rebuild(pos)
    h.apply(f64, out=out["up64b"])
    h.apply_rotated(rot, f64, out=out["rot"], work=out["work"])


def test_build_into_equals_build_and_allocates_nothing(hq):
    w = W.small_batch(61, [2, 3, 40, 700, 1500, 2600, 900, 5000, 64])
    rng = np.random.default_rng(61)
    R = 32
    f = rng.standard_normal((3 * w.N, R))
    g = rng.standard_normal((w.rows, R))
    rot, tr = W.rigid_motions(rng, 1, w.m)
    dev = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    f64, g64 = dev(f), dev(g)
    f32t = dev(f, torch.float32).reshape(w.N, 3, R).transpose(1, 2).contiguous()
    g32t = dev(g, torch.float32).reshape(w.rows // 3, 3, R).transpose(1, 2).contiguous()
    rot_d, tr_d = dev(rot.reshape(w.m, 9)), dev(tr.reshape(w.m, 3))

    def outs():
        return {"up64": torch.empty((w.rows, R), dtype=torch.float64, device="cuda"),
                "dn64": torch.empty((3 * w.N, R), dtype=torch.float64, device="cuda"),
                "up32": torch.empty((w.rows // 3, R, 3), dtype=torch.float32, device="cuda"),
                "dn32": torch.empty((w.N, R, 3), dtype=torch.float32, device="cuda"),
                "root": torch.empty((6 * w.m, R), dtype=torch.float64, device="cuda"),
                "full": torch.empty((w.rows, R), dtype=torch.float64, device="cuda"),
                "up64b": torch.empty((w.rows, R), dtype=torch.float64, device="cuda"),
                "rot": torch.empty((w.rows, R), dtype=torch.float64, device="cuda"),
                "work": torch.empty((3 * w.N, R), dtype=torch.float64, device="cuda")}

    # reference: a library-allocated handle (this also loads every kernel)
    pos_a = dev(w.pos)
    ha = hq.build(pos_a, w.offsets, tile_units=16, store=3, keep_node_data=1)
    oa = outs()
    _run(hq, ha, pos_a, rot_d, tr_d, f64, g64, f32t, g32t, oa)
    nda = ha.node_data()
    ba = ha.explicit_blocks(4)
    torch.cuda.synchronize()

    # the workspace handle, everything preallocated by torch
    opts = dict(tile_units=16, store=3, keep_node_data=1, max_nrhs=R)
    need = hq.workspace_bytes(w.offsets, **opts)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    pos_b = dev(w.pos)
    ob = outs()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    hb = hq.build_into(pos_b, w.offsets, workspace=ws, **opts)
    _run(hq, hb, pos_b, rot_d, tr_d, f64, g64, f32t, g32t, ob)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"[gpu] workspace {need} bytes; device free memory moved by {free0 - free1} bytes", flush=True)
    assert free1 == free0
    for k in oa:
        if k != "work":  # scratch of the rotated product (unused by the wide sweeps)
            assert torch.equal(oa[k], ob[k]), k
    ndb = hb.node_data()
    for k in nda:
        if nda[k] is not None:
            assert np.array_equal(nda[k], ndb[k]), k
    bb = hb.explicit_blocks(4)
    assert torch.equal(ba[0], bb[0])
    for x, y in zip(ba[1:], bb[1:]):
        assert np.array_equal(x, y)
    assert hb.query()["device_flags"] == 0 and ha.query()["device_flags"] == 0
    # beyond the reserved right-hand sides: refused, nothing allocated
    with pytest.raises(hq.HQError) as e:
        hb.apply(torch.zeros((3 * w.N, R + 1), dtype=torch.float64, device="cuda"))
    assert e.value.status == HQ_E_UNSUPPORTED
    # FP32 entries are half the size: twice the right-hand sides fit
    hb.apply(torch.zeros((3 * w.N, 2 * R), dtype=torch.float32, device="cuda"))
    hb.destroy()
    ha.destroy()


def test_build_into_krylov_and_limits(hq):
    w = W.small_batch(62, [300, 1200, 64])
    rng = np.random.default_rng(62)
    R = 3
    pos = torch.from_numpy(w.pos).cuda()
    F = torch.from_numpy(rng.standard_normal((6 * w.m, R))).cuda()

    def dapply(x, y):  # a diagonal SPD mobility
        y.copy_(x * 1.5)

    ha = hq.build(pos, w.offsets)
    Va, ga, ia = hq.constrained_solve(ha, dapply, F, rtol=1e-10)
    opts = dict(krylov_nrhs=R)
    hb = hq.build_into(pos, w.offsets, **opts)
    Vb, gb, ib = hq.constrained_solve(hb, dapply, F, rtol=1e-10)
    # the CG dot products add block partials with atomics, so the last bits
    # of two solves may differ: the same iterations and the same solution
    assert ia["iters"] == ib["iters"] and ib["max_rel_residual"] <= 1e-10
    assert float((Va - Vb).norm() / Va.norm()) <= 1e-12
    assert float((ga - gb).norm() / ga.norm()) <= 1e-12
    # more right-hand sides than the workspace's Krylov vectors hold
    with pytest.raises(hq.HQError) as e:
        hq.constrained_solve(hb, dapply, torch.cat([F, F], dim=1).contiguous())
    assert e.value.status == HQ_E_UNSUPPORTED
    # no Krylov vectors reserved at all
    hc = hq.build_into(pos, w.offsets)
    with pytest.raises(hq.HQError) as e:
        hq.constrained_solve(hc, dapply, F)
    assert e.value.status == HQ_E_UNSUPPORTED
    # a workspace too small, or not 256-byte aligned
    need = hq.workspace_bytes(w.offsets)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(hq.HQError) as e:
        hq.build_into(pos, w.offsets, workspace=small)
    assert e.value.status == HQ_E_INVALID
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(hq.HQError) as e:
        hq.build_into(pos, w.offsets, workspace=big[16:])
    assert e.value.status == HQ_E_INVALID
    # a tile capacity below the tree's tiles
    with pytest.raises(hq.HQError) as e:
        hq.build_into(pos, w.offsets, tile_units=8, max_tiles=4)
    assert e.value.status == HQ_E_UNSUPPORTED
