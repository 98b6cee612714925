"""The Brownian-dynamics step on the GPU: rigid motion, rebuild and the FP32
sweep pair, eagerly and replayed from a captured hipGraph."""
import numpy as np
import pytest

import workloads as W
from oracle import dense, hier

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hq():
    import paper_1708_08427_amd as hq
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return hq


def _workload():
    w = W.small_batch(21, [2, 3, 60, 400, 1300, 2500, 900], nrhs=32)
    rng = np.random.default_rng(21)
    rot, trans = W.rigid_motions(rng, 4, w.m)
    f = rng.standard_normal((3 * w.N, 32))
    return w, rot, trans, f


def test_rigid_update_matches_numpy(hq):
    w, rot, trans, _ = _workload()
    pos = torch.from_numpy(w.pos).cuda()
    h = hq.build(pos, w.offsets)
    rot_d = torch.from_numpy(rot[0].reshape(w.m, 9)).cuda()
    tr_d = torch.from_numpy(trans[0]).cuda()
    h.rigid_update(pos, rot_d, tr_d)
    got = pos.cpu().numpy()
    for j in range(w.m):
        p = w.pos[w.offsets[j]:w.offsets[j + 1]]
        c = p.mean(axis=0)
        want = (p - c) @ rot[0, j].T + c + trans[0, j]
        assert np.abs(got[w.offsets[j]:w.offsets[j + 1]] - want).max() < 1e-9


def test_rebuild_equals_fresh_build(hq):
    w, rot, trans, f = _workload()
    pos = torch.from_numpy(w.pos).cuda()
    h = hq.build(pos, w.offsets, tile_units=32, later_tile_units=4)
    f64 = torch.from_numpy(f).cuda()
    moved = w.pos.copy()
    for j in range(w.m):
        sl = slice(w.offsets[j], w.offsets[j + 1])
        c = moved[sl].mean(axis=0)
        moved[sl] = (moved[sl] - c) @ rot[1, j].T + c + trans[1, j]
    pos2 = torch.from_numpy(moved).cuda()
    h.rebuild(pos2)
    a = h.apply(f64).cpu().numpy()
    h2 = hq.build(pos2, w.offsets, tile_units=32, later_tile_units=4)
    b = h2.apply(f64).cpu().numpy()
    assert h.query()["device_flags"] == 0
    assert np.array_equal(a, b)
    bt = hier.Batch(moved, w.offsets)
    o = bt.apply(f)
    assert np.abs(a - o).max() < 1e-10


def test_graph_replay_matches_eager(hq):
    """K steps captured once, replayed several times with eager work and
    synchronisations between replays; every replay equals the eager run."""
    w, rot, trans, f = _workload()
    K = 3
    rot_d = torch.from_numpy(rot.reshape(4, w.m, 9)).cuda()
    tr_d = torch.from_numpy(trans).cuda()
    f32 = torch.from_numpy(f).float().cuda()
    tmp = torch.empty((w.rows, 32), dtype=torch.float32, device="cuda")
    out = torch.empty((3 * w.N, 32), dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pos = torch.from_numpy(w.pos).cuda()
        h = hq.build(pos, w.offsets, tile_units=32, store=2, stream=s)
        h.reserve(32, torch.float32)

        def steps():
            for i in range(K):
                h.rigid_update(pos, rot_d[i], tr_d[i], stream=s)
                h.rebuild(pos, stream=s)
                h.apply(f32, out=tmp, stream=s)
                h.apply(tmp, transpose=True, out=out, stream=s)

        pos.copy_(torch.from_numpy(w.pos).cuda())
        steps()
        torch.cuda.synchronize()
        eager_out, eager_pos = out.cpu().numpy(), pos.cpu().numpy()

        pos.copy_(torch.from_numpy(w.pos).cuda())
        torch.cuda.synchronize()
        hq.capture_begin(s)
        steps()
        g = hq.capture_end(s)
        for rep in range(3):
            # the motion turns each body about the centroid of the handle's last
            # (re)build: restore positions and that state before a replay
            pos.copy_(torch.from_numpy(w.pos).cuda())
            h.rebuild(pos, stream=s)
            out.zero_()
            torch.cuda.synchronize()
            g.launch(s)
            torch.cuda.synchronize()
            assert np.array_equal(pos.cpu().numpy(), eager_pos), rep
            assert np.array_equal(out.cpu().numpy(), eager_out), rep
            # eager work between replays
            h.apply(f32, out=tmp, stream=s)
            torch.cuda.synchronize()
        g.destroy()
        assert h.query()["device_flags"] == 0
    # the replayed step is the projection P f on the moved bodies
    for j in range(w.m):
        if w.offsets[j + 1] - w.offsets[j] < 3:
            continue
        sl = slice(w.offsets[j], w.offsets[j + 1])
        b0, b1 = 3 * w.offsets[j], 3 * w.offsets[j + 1]
        want = dense.project(eager_pos[sl], f[b0:b1])
        got = eager_out[b0:b1].astype(np.float64)
        assert np.abs(got - want).max() <= 1e-4 * np.abs(f[b0:b1]).max()


def test_two_handle_pipeline_matches_sequence(hq):
    """Steps alternating between two handles of the same bodies on two
    streams (step i + 1's rebuild overlapping step i's sweeps, each motion
    turning the bodies about the centroid of the previous step's rebuild)
    give the positions and products of the one-handle sequence bit for bit,
    eagerly and replayed from a graph captured across both streams."""
    w, rot, trans, f = _workload()
    K = 4
    rot_d = torch.from_numpy(rot.reshape(K, w.m, 9)).cuda()
    tr_d = torch.from_numpy(trans).cuda()
    f32 = torch.from_numpy(f).float().cuda()
    s0, s1 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s0):
        pos = torch.from_numpy(w.pos).cuda()
        # the plain sequence on one handle and one stream
        h = hq.build(pos, w.offsets, tile_units=16, store=2, stream=s0)
        tmp = torch.empty((w.rows, 32), dtype=torch.float32, device="cuda")
        out = torch.empty((3 * w.N, 32), dtype=torch.float32, device="cuda")
        for i in range(K):
            h.rigid_update(pos, rot_d[i], tr_d[i], stream=s0)
            h.rebuild(pos, stream=s0)
            h.apply(f32, out=tmp, stream=s0)
            h.apply(tmp, transpose=True, out=out, stream=s0)
        torch.cuda.synchronize()
        want_pos, want_out = pos.cpu().numpy(), out.cpu().numpy()

        pos.copy_(torch.from_numpy(w.pos).cuda())
        hs = [hq.build(pos, w.offsets, tile_units=16, store=2, stream=s0) for _ in range(2)]
        for hx in hs:
            hx.reserve(32, torch.float32)
        ss = [s0, s1]
        tmps = [torch.empty_like(tmp) for _ in range(2)]
        outs = [torch.empty_like(out) for _ in range(2)]
        events = []

        def event(s):
            e = torch.cuda.Event()
            e.record(s)
            events.append(e)
            return e

        def steps():
            s1.wait_event(event(s0))
            rebuilt = None
            for i in range(K):
                x = i % 2
                if rebuilt is not None:
                    ss[x].wait_event(rebuilt)
                hs[(i - 1) % 2].rigid_update(pos, rot_d[i], tr_d[i], stream=ss[x])
                hs[x].rebuild(pos, stream=ss[x])
                rebuilt = event(ss[x])
                hs[x].apply(f32, out=tmps[x], stream=ss[x])
                hs[x].apply(tmps[x], transpose=True, out=outs[x], stream=ss[x])
            s0.wait_event(event(s1))

        torch.cuda.synchronize()
        steps()
        torch.cuda.synchronize()
        assert np.array_equal(pos.cpu().numpy(), want_pos)
        assert np.array_equal(outs[(K - 1) % 2].cpu().numpy(), want_out)

        hq.capture_begin(s0)
        steps()
        g = hq.capture_end(s0)
        for rep in range(2):
            # restore the positions and both handles' centroids before a replay
            pos.copy_(torch.from_numpy(w.pos).cuda())
            for hx in hs:
                hx.rebuild(pos, stream=s0)
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            g.launch(s0)
            torch.cuda.synchronize()
            assert np.array_equal(pos.cpu().numpy(), want_pos), rep
            assert np.array_equal(outs[(K - 1) % 2].cpu().numpy(), want_out), rep
        g.destroy()
        for hx in hs:
            assert hx.query()["device_flags"] == 0


def test_rigid_motion_matches_numpy(hq):
    """hq_rigid_motion about given centres, into another buffer and in place,
    against numpy; the input buffer is left untouched."""
    w, rot, trans, _ = _workload()
    pos = torch.from_numpy(w.pos).cuda()
    h = hq.build(pos, w.offsets)
    rng = np.random.default_rng(5)
    cen = rng.uniform(0.0, 100.0, (w.m, 3))
    rot_d = torch.from_numpy(rot[0].reshape(w.m, 9)).cuda()
    tr_d = torch.from_numpy(trans[0]).cuda()
    cen_d = torch.from_numpy(cen).cuda()
    out = torch.empty_like(pos)
    h.rigid_motion(pos, out, rot_d, tr_d, cen_d)
    torch.cuda.synchronize()
    assert np.array_equal(pos.cpu().numpy(), w.pos)
    got = out.cpu().numpy()
    for j in range(w.m):
        p = w.pos[w.offsets[j]:w.offsets[j + 1]]
        want = (p - cen[j]) @ rot[0, j].T + cen[j] + trans[0, j]
        assert np.abs(got[w.offsets[j]:w.offsets[j + 1]] - want).max() < 1e-9
    h.rigid_motion(pos, pos, rot_d, tr_d, cen_d)
    assert torch.equal(pos, out)
    with pytest.raises(ValueError):
        h.rigid_motion(pos, out, rot_d, tr_d, cen_d[:-1])


@pytest.mark.parametrize("P", [2, 3])
def test_position_buffers_equal_one_handle(hq, P):
    """Steps on P handles and P position buffers, step i moving buffer
    (i - 1) % P into buffer i % P about tracked centroids, so that a step
    waits only for the previous step's motion (consecutive rebuilds run
    concurrently): the positions and products of the one-handle sequence in
    place, bit for bit, eagerly and replayed from a graph captured across
    the streams."""
    w, rot, trans, f = _workload()
    K = 4
    rot_d = torch.from_numpy(rot.reshape(K, w.m, 9)).cuda()
    tr_d = torch.from_numpy(trans).cuda()
    sizes = np.diff(np.asarray(w.offsets))
    c0 = np.add.reduceat(w.pos, np.asarray(w.offsets[:-1]), axis=0) / sizes[:, None]
    cen = c0[None] + np.concatenate([np.zeros((1, w.m, 3)), np.cumsum(trans, axis=0)[:-1]], axis=0)
    cen_d = torch.from_numpy(np.ascontiguousarray(cen)).cuda()
    f32 = torch.from_numpy(f).float().cuda()
    s0, s1 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s0):
        pos = torch.from_numpy(w.pos).cuda()
        h = hq.build(pos, w.offsets, tile_units=16, store=2, stream=s0)
        tmp = torch.empty((w.rows, 32), dtype=torch.float32, device="cuda")
        out = torch.empty((3 * w.N, 32), dtype=torch.float32, device="cuda")
        for i in range(K):
            h.rigid_motion(pos, pos, rot_d[i], tr_d[i], cen_d[i], stream=s0)
            h.rebuild(pos, stream=s0)
            h.apply(f32, out=tmp, stream=s0)
            h.apply(tmp, transpose=True, out=out, stream=s0)
        torch.cuda.synchronize()
        want_pos, want_out = pos.cpu().numpy(), out.cpu().numpy()

        posb = [torch.from_numpy(w.pos).cuda() for _ in range(P)]
        hs = [hq.build(posb[0], w.offsets, tile_units=16, store=2, stream=s0) for _ in range(P)]
        for hx in hs:
            hx.reserve(32, torch.float32)
        ss = [s0, s1] + [torch.cuda.Stream() for _ in range(2, P)]
        tmps = [torch.empty_like(tmp) for _ in range(P)]
        outs = [torch.empty_like(out) for _ in range(P)]
        events = []

        def event(s):
            e = torch.cuda.Event()
            e.record(s)
            events.append(e)
            return e

        def steps():
            fork = event(s0)
            for s in ss[1:]:
                s.wait_event(fork)
            moved = None
            for i in range(K):
                x = i % P
                if moved is not None:
                    ss[x].wait_event(moved)
                hs[x].rigid_motion(posb[(i - 1) % P], posb[x], rot_d[i], tr_d[i], cen_d[i], stream=ss[x])
                moved = event(ss[x])
                hs[x].rebuild(posb[x], stream=ss[x])
                hs[x].apply(f32, out=tmps[x], stream=ss[x])
                hs[x].apply(tmps[x], transpose=True, out=outs[x], stream=ss[x])
            for s in ss[1:]:
                s0.wait_event(event(s))

        torch.cuda.synchronize()
        steps()
        torch.cuda.synchronize()
        assert np.array_equal(posb[(K - 1) % P].cpu().numpy(), want_pos)
        assert np.array_equal(outs[(K - 1) % P].cpu().numpy(), want_out)

        hq.capture_begin(s0)
        steps()
        g = hq.capture_end(s0)
        for rep in range(3):
            for b in posb:
                b.zero_()
            posb[P - 1].copy_(torch.from_numpy(w.pos).cuda())
            for o in outs:
                o.zero_()
            torch.cuda.synchronize()
            g.launch(s0)
            torch.cuda.synchronize()
            assert np.array_equal(posb[(K - 1) % P].cpu().numpy(), want_pos), rep
            assert np.array_equal(outs[(K - 1) % P].cpu().numpy(), want_out), rep
        g.destroy()
        for hx in hs:
            assert hx.query()["device_flags"] == 0


def test_first_phase_grid_cap_matches_uncapped(hq):
    """A capped first-phase grid (one wave per compute unit, grid-strided
    over more run pairs than it has waves) gives the uncapped sweeps' results
    bit for bit, both directions, both layouts."""
    w = W.small_batch(23, [2, 5, 700, 3000, 9000, 6100, 480], nrhs=32)
    rng = np.random.default_rng(23)
    f = torch.from_numpy(rng.standard_normal((3 * w.N, 32))).float().cuda()
    g = torch.from_numpy(rng.standard_normal((w.rows, 32))).float().cuda()
    pos = torch.from_numpy(w.pos).cuda()
    h0 = hq.build(pos, w.offsets, tile_units=16, run_nodes=8)
    h1 = hq.build(pos, w.offsets, tile_units=16, run_nodes=8, first_waves_per_cu=1)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    assert (w.N - w.m) // 8 // 2 > 2 * ncu  # more run pairs than the capped grid has waves
    for lay in ("rows", "triples"):
        fv = f if lay == "rows" else f.view(w.N, 3, 32).transpose(1, 2).contiguous()
        gv = g if lay == "rows" else g.view(w.rows // 3, 3, 32).transpose(1, 2).contiguous()
        for tr, v in ((False, fv), (True, gv)):
            a = h0.apply(v, transpose=tr, layout=lay)
            b = h1.apply(v, transpose=tr, layout=lay)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (lay, tr)
    assert h0.query()["device_flags"] == 0 and h1.query()["device_flags"] == 0


def test_node_data_after_rebuild(hq):
    """Centroids and T22 are refreshed by hq_rebuild only for handles built
    with keep_node_data; otherwise hq_node_data refuses them."""
    w, rot, trans, _ = _workload()
    moved = w.pos.copy()
    for j in range(w.m):
        sl = slice(w.offsets[j], w.offsets[j + 1])
        c = moved[sl].mean(axis=0)
        moved[sl] = (moved[sl] - c) @ rot[2, j].T + c + trans[2, j]
    pos2 = torch.from_numpy(moved).cuda()
    fresh = hq.build(pos2, w.offsets).node_data()
    h = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets)
    h.rebuild(pos2)
    with pytest.raises(hq.HQError):
        h.node_data()
    hk = hq.build(torch.from_numpy(w.pos).cuda(), w.offsets, keep_node_data=1)
    hk.rebuild(pos2)
    got = hk.node_data()
    assert np.array_equal(got["centroid"], fresh["centroid"])
    assert np.array_equal(got["T22"], fresh["T22"])
    assert hk.query()["device_flags"] == 0


def test_apply_timed_and_node_phase(hq):
    """hq_apply_timed computes what hq_apply computes and times every tile
    phase; hq_node_phase names a phase for every node."""
    w, _, _, f = _workload()
    pos = torch.from_numpy(w.pos).cuda()
    h = hq.build(pos, w.offsets, tile_units=16)
    fd = torch.from_numpy(f).float().cuda()
    ref = h.apply(fd)
    got, ms = h.apply(fd, timed=True)
    assert torch.equal(got, ref)
    q = h.query()
    assert len(ms) >= q["phases"] and all(x >= 0.0 for x in ms)
    back, ms2 = h.apply(ref, transpose=True, timed=True)
    assert torch.equal(back, h.apply(ref, transpose=True)) and len(ms2) == len(ms)
    ph = h.node_phase()
    assert ph.min() >= 1 and ph.max() == q["phases"]
