"""Benchmark: the Brownian-dynamics step of many rigid bodies on one MI355X.

Workload (seeded, synthetic): m = 4096 bodies with lognormal sizes (median 500
beads, sigma 0.6, clipped to [50, 20000]) on random ellipsoids in a 500^3 box,
32 force vectors per body.  One step = rigid motion of every body (Haar
rotation about its centroid + translation in [-1,1]^3), rebuild of the tree and
FP64 transforms, then Q~^T (Q~ f) in FP32 for the 32 right-hand sides.  K steps
are captured in one hipGraph and replayed; the timed region is bracketed by
synchronisations.  By default consecutive steps alternate between two handles
of the same bodies on four streams and position buffers (--pipeline), so a
step's rebuild and sweeps overlap those of the steps before it (--no-pipeline:
one handle, one stream, positions moved in place).  Force vectors are held as [bead][system][xyz] (the
library's triples layout) unless --layout rows is given.

value = bead-vectors per second = N * R / (time per step).  The roofline row
is the upward sweep Q~ v (FP32): algorithmic bytes (input vectors, residue
output, compact reflectors, links, permutation) over its measured duration.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bead-vectors/s for batched Q̃v+Q̃ᵀv; % HBM peak; FP32 err vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
PROBE_SWEEPS = 3  # must match traffic.PROBE_SWEEPS
TRAFFIC_GLOB = "traffic_up_sweep_bd_m4096_R32*.json"  # one counter summary per launch configuration


def phase_bytes(h, nrhs, elem=4):
    """The same bytes split by the tile phase of the node that moves them (a
    bead's vector rows and permutation entry go with its parent node)."""
    nd = h.node_data(with_G=False, with_geometry=False)
    ph = h.node_phase()
    k = nd["k"].astype(np.int64)
    beads = (nd["x"] < 0).astype(np.int64) + (nd["y"] < 0).astype(np.int64)
    w = np.where(k == 9, 24, np.where(k == 6, 15, 5))
    per = elem * nrhs * 3 * beads + elem * nrhs * (k - 3) + elem * w + 16 + 4 * beads
    return {int(p): int(per[ph == p].sum()) for p in np.unique(ph)}


def algorithmic_bytes(h, nrhs, elem=4):
    """Bytes one sweep must move: vectors in and out, the compact reflectors
    of every node (5, 15 or 24 values for k = 3, 6, 9), 16 bytes of links and
    weights per node, and 4 bytes of permutation per bead."""
    nd = h.node_data(with_G=False, with_geometry=False)
    k = nd["k"]
    w = np.where(k == 9, 24, np.where(k == 6, 15, 5)).sum()
    return (elem * 3 * h.N * nrhs + elem * h.rows * nrhs + elem * int(w) + 16 * (h.N - h.m) + 4 * h.N)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_workers():
    """Host threads this process may use (its CPU affinity, at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


_CPU_WL = None  # the workload, inherited by the forked oracle workers


def _oracle_body(j):
    """The oracle's rebuild + Q~ f + Q~^T (Q~ f) for body j (all R right-hand
    sides, f drawn from a per-body seed): (beads, seconds)."""
    from oracle import hier
    wl = _CPU_WL
    p = wl.pos[wl.offsets[j]:wl.offsets[j + 1]]
    f = np.random.default_rng(1000 + int(j)).standard_normal((3 * len(p), wl.nrhs))
    ts = time.perf_counter()
    b = hier.Body(p)
    y = b.apply(f)
    b.apply(y, transpose=True)
    return len(p), time.perf_counter() - ts


def cpu_baseline(wl, rng_seed, budget_s=8.0):
    """The FP64 oracle as it stands (plain C recursion, one body per call) on
    bounded samples of the same bodies: one thread, then every host core (a
    process pool over bodies).  Runs before the GPU is touched, so the pool's
    processes are forked from a process without GPU state."""
    import multiprocessing as mp
    global _CPU_WL
    _CPU_WL = wl
    R = wl.nrhs
    order = np.random.default_rng(rng_seed).permutation(wl.m)
    beads1, t1, n1 = 0, 0.0, 0
    for j in order:
        b, t = _oracle_body(j)
        beads1, t1, n1 = beads1 + b, t1 + t, n1 + 1
        if t1 > budget_s:
            break
    workers = host_workers()
    # the all-core sample: about budget_s of wall time on every worker
    sample = order[:min(wl.m, n1 * workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_body, [int(j) for j in sample], chunksize=4)
    wall = time.perf_counter() - t0
    beads = sum(b for b, _ in res)
    return {"value": beads * R / wall, "unit": "bead-vectors/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(sample)} of {wl.m} bodies ({beads} beads, R={R}) over {workers} processes, "
                      f"FP64 plain C recursion, rebuild + Q~f + Q~^T(Q~f) per body, {wall:.1f} s wall",
            "one_core": {"value": beads1 * R / t1, "unit": "bead-vectors/s", "cores": 1,
                         "sample": f"{n1} bodies ({beads1} beads), {t1:.1f} s"}}


def sweep_kernel(nrhs, layout, dtype, transpose=False, phase=1):
    """The kernel the library launches for a tile phase of a sweep with this
    many right-hand sides, when its buffers fit the wide sweeps' 2 GiB range
    and the tiles hold 32 units (its dispatch: runs of 32 or 64 lanes above 16
    right-hand sides, 32-lane ones specialised for exactly 32; for 8 to 16,
    16-lane runs in FP32 and 32-lane runs in FP64; below 8, a lane group per
    tile in the first phase and node-parallel sweeps in the later ones)."""
    lpt = 1
    while lpt < nrhs and lpt < 64:
        lpt *= 2
    if nrhs < 8:
        # first phase: a lane group per tile with exact wait counts; later
        # phases node-parallel
        if phase == 1:
            return f"k_{'down' if transpose else 'up'}_lane<{dtype}, {lpt}>"
        return f"k_{'down' if transpose else 'up'}_np<{dtype}, 256, {lpt}, 32, false>"
    if lpt < 32:
        lpt = 16 if dtype == "float" else 32
    rt = 32 if nrhs == 32 else 0
    tri = str(layout == "triples").lower()
    if transpose:
        return f"k_down_wide<{dtype}, {lpt}, {rt}, 6, 3, {str(phase > 1).lower()}, 1, {tri}, false>"
    return f"k_up_wide<{dtype}, {lpt}, {rt}, 6, 3, {3 if phase == 1 else 6}, 1, {tri}, false>"


def stream_ceiling(hq, torch, read_bytes, write_bytes, stream, reps=10):
    """The library's streaming kernel (hq_stream_ceiling: non-temporal 16-byte
    accesses, the sweeps' cache policy) with a given read:write mix; the best
    median over a few grid sizes, in GB/s of bytes moved."""
    import ctypes
    from paper_1708_08427_amd import _lib
    lib = _lib.load()
    rb = (int(read_bytes) // 4096) * 4096
    wb = min(rb, (int(write_bytes) // 4096) * 4096)
    src = torch.ones(rb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty(wb // 4, dtype=torch.float32, device="cuda")
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    sp = ctypes.c_void_p(stream.cuda_stream)
    best = None
    for blocks in (256, 512, 1024, 2048, 4096, 8192):
        def run():
            st = lib.hq_stream_ceiling(ctypes.c_void_p(src.data_ptr()), rb, ctypes.c_void_p(dst.data_ptr()), wb,
                                       blocks, ctypes.c_void_p(sink.data_ptr()), sp)
            if st != 0:
                raise RuntimeError(lib.hq_last_error().decode())
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        run()
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            run()
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
        gbs = (rb + wb) / (ms * 1e-3) / 1e9
        if best is None or gbs > best["achieved"]:
            best = {"achieved": gbs, "unit": "GB/s", "ms": ms, "read_bytes": rb, "write_bytes": wb,
                    "blocks": blocks}
    del src, dst
    best["frac"] = best["achieved"] / HBM_PEAK_GBS
    best["what"] = ("hq_stream_ceiling: one launch reading and writing the dominant launch's HBM traffic mix "
                    "(non-temporal 16-byte accesses, 256 threads per block, best of 256-8192 blocks)")
    return best


def to_layout(a, layout):
    """(3T, R) rows -> the layout's host array ((T, R, 3) for triples)."""
    if layout == "rows":
        return np.ascontiguousarray(a)
    return np.ascontiguousarray(a.reshape(a.shape[0] // 3, 3, a.shape[1]).transpose(0, 2, 1))


def from_layout(a, layout):
    if layout == "rows":
        return a
    return np.ascontiguousarray(a.transpose(0, 2, 1).reshape(3 * a.shape[0], a.shape[1]))


def vec_shape(nrows, R, layout):
    return (nrows, R) if layout == "rows" else (nrows // 3, R, 3)


def probe(hq, torch, wl, f, args):
    """The counter run: one 512 MiB device copy (calibrates FETCH_SIZE and
    WRITE_SIZE against known bytes), then PROBE_SWEEPS upward and downward FP32
    sweeps of the bench workload."""
    dev = torch.device("cuda:0")
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    pos = torch.from_numpy(wl.pos).to(dev)
    lay = args.layout
    f32 = torch.from_numpy(to_layout(f, lay)).float().to(dev)
    tmp = torch.empty(vec_shape(wl.rows, wl.nrhs, lay), dtype=torch.float32, device=dev)
    out = torch.empty(vec_shape(3 * wl.N, wl.nrhs, lay), dtype=torch.float32, device=dev)
    h = hq.build(pos, wl.offsets, store=2, **fixed_options(args))
    for _ in range(PROBE_SWEEPS):
        h.apply(f32, out=tmp, layout=lay)
    for _ in range(PROBE_SWEEPS):
        h.apply(tmp, transpose=True, out=out, layout=lay)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "algorithmic_bytes": algorithmic_bytes(h, wl.nrhs), "phases": h.query()["phases"],
                      "options": options_tag(fixed_options(args), lay)}), flush=True)


def fixed_options(args):
    return {"tile_units": args.tile_units, "run_nodes": args.run_nodes, "waves_per_cu": args.waves_per_cu,
            "later_tile_units": args.later_tile_units, "leaf_size": args.leaf_size}


DEFAULT_OPTIONS = {"tile_units": 32, "run_nodes": 48, "waves_per_cu": 16}  # the library's defaults for 0


def effective(opts):
    e = {k: int(opts.get(k) or v) for k, v in DEFAULT_OPTIONS.items()}
    e["later_tile_units"] = int(opts.get("later_tile_units") or e["tile_units"])
    e["leaf_size"] = max(1, int(opts.get("leaf_size") or 1))
    return e


def options_tag(opts, layout):
    """The configuration of the first-phase launch a counter summary belongs
    to (waves_per_cu only shapes the later phases' grids)."""
    e = effective(opts)
    return ",".join([f"{k}={e[k]}" for k in ("tile_units", "run_nodes")] + [f"layout={layout}"])


def traffic_from_profile(opts, layout):
    """HBM bytes of one first-phase upward launch from the committed counter
    summary, if it was taken on the current sweep sources in the same launch
    configuration (else None)."""
    import glob

    from traffic import sweep_source_hash
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", TRAFFIC_GLOB)))
    if not paths:
        return None, "no counter summary"
    src, tag, seen = sweep_source_hash(), options_tag(opts, layout), []
    for path in paths:
        with open(path) as fh:
            prof = json.load(fh)
        if prof.get("source_sha256") != src:
            seen.append(f"{os.path.basename(path)}: sweep sources changed since the counters were taken")
        elif prof.get("options") != tag:
            seen.append(f"{os.path.basename(path)}: counters taken with {prof.get('options')}")
        else:
            return prof["up_phase1"]["hbm_bytes"], prof["command"]
    return None, f"bench runs {tag}; " + "; ".join(seen)


def timed_ms(torch, stream, fn, reps, before=None):
    """Median over reps of fn's duration (HIP events on ``stream``); ``before``
    runs ahead of each rep, outside the timed interval (e.g. a cache flush)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    fn()
    torch.cuda.synchronize()
    for a, b in evs:
        if before is not None:
            before()
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def first_phase_ms(torch, h, v, out, stream, reps, transpose=False):
    """Median duration of the first tile phase's launch (hq_apply_timed)."""
    ms = []
    for _ in range(reps):
        h.apply(v, out=out, stream=stream, transpose=transpose)
        _, ph = h.apply(v, out=out, stream=stream, timed=True, transpose=transpose)
        ms.append(ph[0])
    torch.cuda.synchronize()
    return float(np.median(ms))


def leg_workload(W, name):
    """(workload, right-hand sides, FP64 timed too) of a configuration leg."""
    if name == "C2":
        return W.ellipsoid_n65536(), 16, True
    if name == "C3":
        return W.batched_m1000(), 1, False
    return W.large_clustered(), 1, False


def leg_options_tag(opts, R):
    """The configuration a leg's first-phase launch depends on: the tile size,
    and the run length for the wide sweeps (8 or more right-hand sides); the
    lane sweeps below 8 take one tile per lane group whatever the run length."""
    e = effective(opts)
    keys = ("tile_units", "run_nodes") if R >= 8 else ("tile_units",)
    return ",".join([f"{k}={e[k]}" for k in keys] + ["layout=rows"])


def leg_traffic(wl, opts, R):
    """HBM bytes of one first-phase upward launch of a leg from its committed
    counter summary (traffic_up_sweep_<workload>.json), if taken on the
    current sweep sources in the same configuration (else None and why)."""
    from traffic import sweep_source_hash
    path = os.path.join(ROOT, "profiles", f"traffic_up_sweep_{wl.name}.json")
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as fh:
        prof = json.load(fh)
    if prof.get("source_sha256") != sweep_source_hash():
        return None, "sweep sources changed since the counters were taken"
    tag = leg_options_tag(opts, R)
    if prof.get("options") != tag:
        return None, f"leg runs {tag}; counters taken with {prof.get('options')}"
    return prof["up_phase1"]["hbm_bytes"], prof["command"]


def probe_leg(hq, torch, W, name, args):
    """The counter run of a leg: the 512 MiB copy, then PROBE_SWEEPS upward and
    downward FP32 sweeps of the leg's workload (rows layout) in the launch
    configuration given on the command line."""
    dev = torch.device("cuda:0")
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    wl, R, _ = leg_workload(W, name)
    v, w = wl.draw_vectors()
    pos = torch.from_numpy(wl.pos).to(dev)
    opts = fixed_options(args)
    h = hq.build(pos, wl.offsets, store=2, **opts)
    vd = torch.from_numpy(v).float().to(dev)
    wd = torch.from_numpy(w).float().to(dev)
    up = torch.empty((wl.rows, R), dtype=torch.float32, device=dev)
    dn = torch.empty((3 * wl.N, R), dtype=torch.float32, device=dev)
    for _ in range(PROBE_SWEEPS):
        h.apply(vd, out=up)
    for _ in range(PROBE_SWEEPS):
        h.apply(wd, transpose=True, out=dn)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "workload": wl.name, "algorithmic_bytes": algorithmic_bytes(h, R),
                      "first_phase_bytes": phase_bytes(h, R)[1], "phases": h.query()["phases"],
                      "options": leg_options_tag(opts, R)}), flush=True)


def config_leg(hq, torch, W, name, stream, reps=10, log=print):
    """One of the other target configurations, timed like the sweeps of the
    BD step: FP32 Q~v and Q~^T w (and FP64 where the configuration asks for
    it), algorithmic bytes and fraction of the HBM peak per direction, the
    first tile phase's launch (with its measured HBM bytes where a counter
    summary of the same configuration is committed), the FP32 error against
    the FP64 oracle and the leak.  Inputs are N(0,1) in the rows layout."""
    from oracle import dense, hier
    dev = torch.device("cuda:0")
    flush = None
    wl, R, fp64 = leg_workload(W, name)
    if name in ("C2", "C3"):
        # the working set fits the 256 MB Infinity Cache: time it after a
        # 1 GiB write evicts it, as well as warm
        fbuf = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        flush = lambda: fbuf.fill_(1.0)
    assert wl.nrhs == R
    v, w = wl.draw_vectors()
    log(f"leg {name}: {wl.name} N={wl.N} m={wl.m} R={R}")
    pos = torch.from_numpy(wl.pos).to(dev)
    # the launch configuration the autotuner picks for this workload's FP32
    # sweeps (these legs time sweeps, not rebuilds), with one-bead leaves: the
    # per-node byte model and the element-wise oracle comparison below hold
    # for the tree of Section 2.1, whose basis leaf boxes change
    t0 = time.perf_counter()
    tuned = hq.autotune(pos, wl.offsets, R, torch.float32, include_rebuild=False, stream=stream, leaf_size=1)
    opts = {k: tuned[k] for k in ("tile_units", "run_nodes", "waves_per_cu", "later_tile_units", "leaf_size")}
    log(f"leg {name}: autotune {1e3 * (time.perf_counter() - t0):.0f} ms: {opts}")
    # C5 also generates its explicit block-sparse Q~, which needs the FP64
    # transforms
    h = hq.build(pos, wl.offsets, store=3 if (fp64 or name == "C5") else 2, stream=stream, **opts)
    res = {"workload": wl.name, "beads": wl.N, "bodies": wl.m, "nrhs": R, "rows": wl.rows,
           "tiles": h.query()["tiles"], "phases": h.query()["phases"], "autotuned": opts}
    precs = [("fp32", torch.float32, 4)] + ([("fp64", torch.float64, 8)] if fp64 else [])
    outs = {}
    for tag, dt, elem in precs:
        vd = torch.from_numpy(v).to(dt).to(dev)
        wd = torch.from_numpy(w).to(dt).to(dev)
        up = torch.empty((wl.rows, R), dtype=dt, device=dev)
        dn = torch.empty((3 * wl.N, R), dtype=dt, device=dev)
        nbytes = algorithmic_bytes(h, R, elem)
        t_up = timed_ms(torch, stream, lambda: h.apply(vd, out=up, stream=stream), reps)
        t_dn = timed_ms(torch, stream, lambda: h.apply(wd, transpose=True, out=dn, stream=stream), reps)
        t_p1 = first_phase_ms(torch, h, vd, up, stream, reps)
        pb = phase_bytes(h, R, elem)
        leg = {"up_ms": t_up, "down_ms": t_dn, "bytes_per_sweep": int(nbytes),
               "bead_vectors_per_s": wl.N * R / ((t_up + t_dn) * 1e-3),
               "frac_up": nbytes / (t_up * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "frac_down": nbytes / (t_dn * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "first_phase": {"kernel": sweep_kernel(R, "rows", "float" if elem == 4 else "double"),
                               "ms": t_p1, "bytes": int(pb[1]),
                               "frac": pb[1] / (t_p1 * 1e-3) / 1e9 / HBM_PEAK_GBS}}
        if tag == "fp32":
            tb, tsrc = leg_traffic(wl, opts, R)
            leg["first_phase"]["traffic"] = tb
            leg["first_phase"]["traffic_source"] = tsrc
        if flush is not None:
            c_up = timed_ms(torch, stream, lambda: h.apply(vd, out=up, stream=stream), reps, before=flush)
            c_dn = timed_ms(torch, stream, lambda: h.apply(wd, transpose=True, out=dn, stream=stream), reps,
                            before=flush)
            leg["after_1gib_flush"] = {"up_ms": c_up, "down_ms": c_dn,
                                       "frac_up": nbytes / (c_up * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                       "frac_down": nbytes / (c_dn * 1e-3) / 1e9 / HBM_PEAK_GBS}
        torch.cuda.synchronize()
        outs[tag] = (up.double().cpu().numpy(), dn.double().cpu().numpy())
        res[tag] = leg
        del vd, wd, up, dn
    assert h.query()["device_flags"] == 0
    up32, dn32 = outs["fp32"]
    # accuracy: FP32 against the FP64 oracle (element-wise where the bodies'
    # nodes are well conditioned), and the leak of Q~^T w
    if name == "C5":
        # one body of 4.2M beads with near-collinear clusters: its basis is
        # fixed only up to rounding, so the comparison is basis-free (the
        # projector and the leak, Z applied in O(n) on the host)
        pr = h.apply(h.apply(torch.from_numpy(v).float().to(dev)), transpose=True).double().cpu().numpy()
        want = dense.project_large(wl.pos, v)
        res["fp32_projector_rel_err"] = float(np.linalg.norm(pr - want) / np.linalg.norm(v))
        res["fp32_leak"] = float(dense.leak_large(wl.pos, dn32).max())
        res["accuracy_note"] = "FP32 Q~^T(Q~ v) against the FP64 dense projector; leak of FP32 Q~^T w"
        # explicit block-sparse Q~ in FP32: generation time and bytes written
        nb, nv = h.explicit_blocks_size(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vals = h.explicit_blocks(0, dtype=torch.float32, stream=stream)[0]
        torch.cuda.synchronize()
        t_ex = (time.perf_counter() - t0) * 1e3
        res["explicit_blocks"] = {"blocks": nb, "values": nv, "bytes_written": 4 * nv, "ms_incl_host": t_ex,
                                  "what": "hq_explicit_blocks (FP32), wall time including its host-side tables"}
        del vals
    else:
        sample = np.arange(wl.m) if wl.m <= 100 else np.random.default_rng(8).choice(wl.m, 100, replace=False)
        err = leak = 0.0
        rows = np.concatenate([[0], np.cumsum(3 * np.diff(wl.offsets) - 6)])
        for j in sample:
            b0, b1 = wl.offsets[j], wl.offsets[j + 1]
            p = wl.pos[b0:b1]
            bo = hier.Body(p)
            r0, r1 = rows[j], rows[j + 1]
            ref_up = bo.apply(v[3 * b0:3 * b1])
            ref_dn = bo.apply(w[r0:r1], transpose=True)
            e1 = np.linalg.norm(up32[r0:r1] - ref_up, axis=0) / np.linalg.norm(v[3 * b0:3 * b1], axis=0)
            e2 = np.linalg.norm(dn32[3 * b0:3 * b1] - ref_dn, axis=0) / np.linalg.norm(w[r0:r1], axis=0)
            err = max(err, float(e1.max()), float(e2.max()))
            leak = max(leak, float(dense.leak_large(p, dn32[3 * b0:3 * b1]).max()))
            if "fp64" in outs:
                u64, d64 = outs["fp64"]
                res.setdefault("fp64_rel_err_vs_oracle", 0.0)
                e64 = max(float((np.linalg.norm(u64[r0:r1] - ref_up, axis=0) /
                                 np.linalg.norm(ref_up, axis=0)).max()),
                          float((np.linalg.norm(d64[3 * b0:3 * b1] - ref_dn, axis=0) /
                                 np.linalg.norm(ref_dn, axis=0)).max()))
                res["fp64_rel_err_vs_oracle"] = max(res["fp64_rel_err_vs_oracle"], e64)
        res["fp32_rel_err_vs_fp64_oracle"] = err
        res["fp32_leak"] = leak
        res["accuracy_bodies"] = int(len(sample))
    h.destroy()
    if flush is not None:
        del fbuf
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile-units", type=int, default=0, help="0: autotuned (with run length and waves per CU)")
    ap.add_argument("--run-nodes", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--later-tile-units", type=int, default=0, help="0: tile size of the first phase")
    ap.add_argument("--leaf-size", type=int, default=0, help="leaf boxes of up to this many beads (0: autotuned "
                    "with the tile sizes, or 1 bead without the autotuner)")
    ap.add_argument("--no-autotune", action="store_true", help="library defaults for options left at 0")
    ap.add_argument("--layout", choices=("triples", "rows"), default="triples",
                    help="vector layout of the force and residue vectors (hq_layout)")
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--bodies", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--first-waves-per-cu", type=int, default=0,
                    help="cap of the first tile phase's sweep grid (waves per CU; 0: uncapped)")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="one handle and one stream: step i+1's rebuild waits for step i's sweeps")
    ap.add_argument("--pipeline", type=int, default=4,
                    help="handles, streams and position buffers that consecutive steps rotate through")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--probe", action="store_true",
                    help="only build, copy 512 MiB once and run 3 sweeps per direction (for rocprofv3 --pmc)")
    ap.add_argument("--no-legs", action="store_true", help="skip the other configurations (C2, C3, C5)")
    ap.add_argument("--legs-only", action="store_true", help="only the other configurations (for rocprofv3)")
    ap.add_argument("--probe-leg", choices=("C2", "C3", "C5"),
                    help="the counter run of one configuration leg (launch options from the command line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the bodies of this workload "
              "would shard across GPUs with no communication, but the library runs one GPU per process and "
              "the benchmark drives one.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1708_08427_amd as hq
    import workloads as W

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.probe_leg:
        probe_leg(hq, torch, W, args.probe_leg, args)
        return
    if args.legs_only:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            for name in ("C2", "C3", "C5"):
                log(json.dumps({name: config_leg(hq, torch, W, name, stream, log=log)}))
        return
    # the CPU baseline first: its process pool forks before the GPU is touched
    cpu = None
    if not args.no_cpu and not args.probe:
        t0 = time.perf_counter()
        cpu = cpu_baseline(W.bd_m4096(m=args.bodies, nrhs=args.nrhs), 5)
        log(f"cpu baseline {time.perf_counter() - t0:.1f} s: {cpu}")

    wl = W.bd_m4096(m=args.bodies, nrhs=args.nrhs)
    N, m, R = wl.N, wl.m, wl.nrhs
    rng = np.random.default_rng(33)
    f = rng.standard_normal((3 * N, R))
    if args.probe:
        probe(hq, torch, wl, f, args)
        return
    total_steps = args.steps + args.warmup
    rot, trans = W.rigid_motions(rng, total_steps, m)
    log(f"workload {wl.name}: N={N} m={m} R={R} rows={wl.rows}")

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pos = torch.from_numpy(wl.pos).to(dev)
        pos0 = pos.clone()
        lay = args.layout
        f32 = torch.from_numpy(to_layout(f, lay)).float().to(dev)
        tmp = torch.empty(vec_shape(wl.rows, R, lay), dtype=torch.float32, device=dev)
        out = torch.empty(vec_shape(3 * N, R, lay), dtype=torch.float32, device=dev)
        rot_d = torch.from_numpy(rot.reshape(total_steps, m, 9)).to(dev)
        trans_d = torch.from_numpy(trans).to(dev)
        # launch configuration: given, or picked by the autotuner for this
        # workload (rebuild + both sweeps, FP32, R right-hand sides)
        opts = fixed_options(args)
        autotuned = False
        if not args.no_autotune and args.tile_units == 0:
            t0 = time.perf_counter()
            tuned = hq.autotune(pos, wl.offsets, R, torch.float32, include_rebuild=True, stream=stream, layout=lay)
            opts = {k: tuned[k] for k in opts}
            autotuned = True
            log(f"autotune {1e3 * (time.perf_counter() - t0):.0f} ms: {opts}, {tuned['ms']:.3f} ms per round")
        t0 = time.perf_counter()
        # the step applies in FP32, so only the FP32 copy of the FP64-generated
        # transforms is kept; the FP64 sweep is timed on its own handle below
        h = hq.build(pos, wl.offsets, store=2, stream=stream, first_waves_per_cu=args.first_waves_per_cu, **opts)
        torch.cuda.synchronize()
        log(f"first build {1e3 * (time.perf_counter() - t0):.1f} ms; {h.query()}")
        h.reserve(R, torch.float32)
        # software pipeline over P handles of the same bodies (--pipeline,
        # default 4), each with its own stream, vectors and position buffer:
        # step i runs on handle i % P and moves the bodies of buffer
        # (i - 1) % P into buffer i % P, turning each body about c_i, its
        # centroid (c_0 from the first positions, c_{i+1} = c_i + t_i: a turn
        # about the centroid keeps it in place).  So a step's motion waits
        # only for the previous step's motion, and the rebuilds and sweeps of
        # consecutive steps run concurrently on the P streams; a handle's
        # next motion follows its previous sweeps on its own stream.
        # Measured on the bench workload: 1.59, 1.51 and 1.50 ms per step
        # with 2, 3 and 4 handles.  Positions and products are those of the
        # plain one-handle sequence, bit for bit.
        npipe = 1 if args.no_pipeline else max(1, args.pipeline)
        sizes = np.diff(np.asarray(wl.offsets))
        c0 = np.add.reduceat(wl.pos, np.asarray(wl.offsets[:-1]), axis=0) / sizes[:, None]
        tr3 = trans.reshape(total_steps, m, 3)
        cen = c0[None] + np.concatenate([np.zeros((1, m, 3)), np.cumsum(tr3, axis=0)[:-1]], axis=0)
        cen_d = torch.from_numpy(np.ascontiguousarray(cen)).to(dev)
        posb = [pos] + [pos.clone() for _ in range(1, npipe)]
        hs, ss, tmps, outs = [h], [stream], [tmp], [out]
        for _ in range(1, npipe):
            hs.append(hq.build(pos, wl.offsets, store=2, stream=stream, first_waves_per_cu=args.first_waves_per_cu,
                               **opts))
            hs[-1].reserve(R, torch.float32)
            ss.append(torch.cuda.Stream())
            tmps.append(torch.empty_like(tmp))
            outs.append(torch.empty_like(out))
        torch.cuda.synchronize()
        events = []  # kept alive while the graphs are captured

        def event(s):
            e = torch.cuda.Event()
            e.record(s)
            events.append(e)
            return e

        def steps(i0, i1):
            fork = event(stream)
            for s in ss[1:]:
                s.wait_event(fork)
            moved = None
            for i in range(i0, i1):
                x = i % npipe
                hx, sx = hs[x], ss[x]
                if moved is not None and npipe > 1:
                    sx.wait_event(moved)
                hx.rigid_motion(posb[(i - 1) % npipe], posb[x], rot_d[i], trans_d[i], cen_d[i], stream=sx)
                moved = event(sx)
                hx.rebuild(posb[x], stream=sx)
                hx.apply(f32, out=tmps[x], stream=sx, layout=lay)
                hx.apply(tmps[x], transpose=True, out=outs[x], stream=sx, layout=lay)
            for s in ss[1:]:
                stream.wait_event(event(s))

        # graphs: warmup steps, then exactly K timed steps
        hq.capture_begin(stream)
        steps(0, args.warmup)
        g_warm = hq.capture_end(stream)
        hq.capture_begin(stream)
        steps(args.warmup, total_steps)
        g_timed = hq.capture_end(stream)
        log("graphs captured")

        g_warm.launch(stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        g_timed.launch(stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_step = ev0.elapsed_time(ev1) / args.steps
        for hx in hs:
            q = hx.query()
            log(f"timed {args.steps} steps: {ms_step:.3f} ms/step; flags {q['device_flags']}")
            if q["device_flags"] != 0:
                raise RuntimeError(f"device flags raised: {q}")
        out_last = outs[(total_steps - 1) % npipe]
        pos = posb[(total_steps - 1) % npipe]  # the final positions

        # accuracy on the final positions: FP32 sweep pair against the FP64 oracle
        pos_host = pos.cpu().numpy()
        out_host = from_layout(out_last.cpu().numpy(), lay).astype(np.float64)
        from oracle import dense, hier
        sample = np.random.default_rng(7).choice(m, 16, replace=False)
        err, leak = 0.0, 0.0
        for j in sample:
            b0, b1 = wl.offsets[j], wl.offsets[j + 1]
            bo = hier.Body(pos_host[b0:b1])
            ref = bo.apply(bo.apply(f[3 * b0:3 * b1]), transpose=True)
            got = out_host[3 * b0:3 * b1]
            e = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(f[3 * b0:3 * b1], axis=0)
            err = max(err, float(e.max()))
            leak = max(leak, float(dense.leak(pos_host[b0:b1], got).max()))
        log(f"FP32 vs FP64 oracle on 16 bodies: rel err {err:.2e}, leak {leak:.2e}")

        # per-sweep durations (eager launches on the same stream)
        def timed(fn, reps):
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            fn()
            torch.cuda.synchronize()
            for a, b in evs:
                a.record(stream)
                fn()
                b.record(stream)
            torch.cuda.synchronize()
            return float(np.median([a.elapsed_time(b) for a, b in evs]))

        t_up = timed(lambda: h.apply(f32, out=tmp, stream=stream, layout=lay), args.apply_reps)
        t_dn = timed(lambda: h.apply(tmp, transpose=True, out=out, stream=stream, layout=lay), args.apply_reps)
        t_rb = timed(lambda: h.rebuild(pos, stream=stream), 5)
        # transform reuse across rigid motions: the products of the moved
        # bodies from the handle's transforms and each body's accumulated
        # rotation since the last rebuild (here that of the timed steps)
        acc = np.tile(np.eye(3), (m, 1, 1))
        for i in range(total_steps):
            acc = np.einsum("jab,jbc->jac", rot[i].reshape(m, 3, 3), acc)
        rot_acc = torch.from_numpy(np.ascontiguousarray(acc.reshape(m, 9))).to(dev)
        rwork = torch.empty_like(f32)
        t_rup = timed(lambda: h.apply_rotated(rot_acc, f32, out=tmp, work=rwork, stream=stream, layout=lay),
                      args.apply_reps)
        t_rdn = timed(lambda: h.apply_rotated(rot_acc, tmp, transpose=True, out=out, stream=stream, layout=lay),
                      args.apply_reps)
        # the full Q = [Q_Z; Q~]: the same sweeps keeping the root Info-sets
        root_buf = torch.empty(vec_shape(6 * m, R, lay), dtype=torch.float32, device=dev)
        t_fup = timed(lambda: h.apply_full(f32, out=tmp, root=root_buf, stream=stream, layout=lay), args.apply_reps)
        t_fdn = timed(lambda: h.apply_full(tmp, transpose=True, root=root_buf, out=out, stream=stream, layout=lay),
                      args.apply_reps)
        # the Krylov harness of Eqs. 1.5-1.6 (hq_constrained_solve) with a
        # per-bead 3x3 SPD mobility applied by a torch callback
        kg = torch.Generator(device=dev)
        kg.manual_seed(17)
        Ak = torch.randn((N, 3, 3), device=dev, generator=kg)
        Dk = torch.eye(3, device=dev).expand(N, 3, 3) + 0.2 * torch.bmm(Ak, Ak.transpose(1, 2).contiguous()) / 9.0
        # y_k = D_k x_k per bead and right-hand side, as three broadcast FMAs
        Dc = [Dk[:, :, c].contiguous() for c in range(3)]  # column c of every D_k, (N, 3)

        def dapply(x, y):
            if lay == "triples":  # x, y: (N, R, 3)
                torch.mul(x[:, :, 0:1], Dc[0][:, None, :], out=y)
                y.addcmul_(x[:, :, 1:2], Dc[1][:, None, :])
                y.addcmul_(x[:, :, 2:3], Dc[2][:, None, :])
            else:  # (3N, R) viewed as (N, 3, R)
                xv, yv = x.view(N, 3, R), y.view(N, 3, R)
                torch.mul(xv[:, 0:1, :], Dc[0][:, :, None], out=yv)
                yv.addcmul_(xv[:, 1:2, :], Dc[1][:, :, None])
                yv.addcmul_(xv[:, 2:3, :], Dc[2][:, :, None])

        Fk = torch.randn(vec_shape(6 * m, R, lay), device=dev, generator=kg)

        def ksolve(iters, rtol):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = hq.constrained_solve(h, dapply, Fk, layout=lay, rtol=rtol, max_iter=iters, stream=stream)
            torch.cuda.synchronize()
            return res[2], (time.perf_counter() - t0) * 1e3

        ksolve(2, 1e-5)  # warm-up
        _, t_k1 = ksolve(1, 1e-30)
        kinfo, t_k = ksolve(200, 1e-5)
        # the host checks convergence every 4 iterations, so the loop runs to
        # the next multiple of 4 past the last column's convergence
        k_launched = min(200, -(-kinfo["iters"] // 4) * 4)
        k_iter = (t_k - t_k1) / max(k_launched - 1, 1)
        xk = torch.randn(vec_shape(3 * N, R, lay), device=dev, generator=kg)
        yk = torch.empty_like(xk)
        def cb_once():  # on the timed stream, as the solve runs it
            with torch.cuda.stream(stream):
                dapply(xk, yk)
        t_cb = timed(cb_once, 5)
        del xk, yk
        log(f"Krylov solve: {kinfo['iters']} CG iterations to {kinfo['max_rel_residual']:.1e} in {t_k:.1f} ms "
            f"({k_iter:.2f} ms per iteration)")
        # the FP64 path beside it: the same workload at the final positions,
        # FP64 transforms and FP64 vectors (a handle keeping only FP64)
        f64 = f32.double()
        tmp64 = torch.empty(vec_shape(wl.rows, R, lay), dtype=torch.float64, device=dev)
        out64 = torch.empty(vec_shape(3 * N, R, lay), dtype=torch.float64, device=dev)
        h64 = hq.build(pos, wl.offsets, store=1, stream=stream, **opts)
        t_up64 = timed(lambda: h64.apply(f64, out=tmp64, stream=stream, layout=lay), 10)
        t_dn64 = timed(lambda: h64.apply(tmp64, transpose=True, out=out64, stream=stream, layout=lay), 10)
        t_rb64 = timed(lambda: h64.rebuild(pos, stream=stream), 5)

        def step64():
            h64.rebuild(pos, stream=stream)
            h64.apply(f64, out=tmp64, stream=stream, layout=lay)
            h64.apply(tmp64, transpose=True, out=out64, stream=stream, layout=lay)

        t_step64 = timed(step64, 5)
        p1_64 = []
        for _ in range(5):
            h64.apply(f64, out=tmp64, stream=stream, layout=lay)
            _, ms_ph = h64.apply(f64, out=tmp64, stream=stream, timed=True, layout=lay)
            p1_64.append(ms_ph[0])
        t_p1_64 = float(np.median(p1_64))
        pb64 = phase_bytes(h64, R, 8)
        nbytes64 = algorithmic_bytes(h64, R, 8)
        assert h64.query()["device_flags"] == 0
        h64.destroy()
        # the FP64 step pipelined like the FP32 one, the paper's precision
        # throughout: its own handles, vectors and position buffers on the
        # same streams, from the first positions with the same motions
        k64, w64 = min(20, args.steps), min(5, args.warmup)
        posb64 = [pos0.clone() for _ in range(npipe)]
        hs64, tmps64, outs64 = [], [], []
        for _ in range(npipe):
            hs64.append(hq.build(posb64[0], wl.offsets, store=1, stream=stream, **opts))
            hs64[-1].reserve(R, torch.float64)
            tmps64.append(torch.empty_like(tmp64))
            outs64.append(torch.empty_like(out64))
        torch.cuda.synchronize()

        def steps64(i0, i1):
            fork = event(stream)
            for s_ in ss[1:]:
                s_.wait_event(fork)
            moved = None
            for i in range(i0, i1):
                x = i % npipe
                hx, sx = hs64[x], ss[x]
                if moved is not None and npipe > 1:
                    sx.wait_event(moved)
                hx.rigid_motion(posb64[(i - 1) % npipe], posb64[x], rot_d[i], trans_d[i], cen_d[i], stream=sx)
                moved = event(sx)
                hx.rebuild(posb64[x], stream=sx)
                hx.apply(f64, out=tmps64[x], stream=sx, layout=lay)
                hx.apply(tmps64[x], transpose=True, out=outs64[x], stream=sx, layout=lay)
            for s_ in ss[1:]:
                stream.wait_event(event(s_))

        hq.capture_begin(stream)
        steps64(0, w64)
        g64_warm = hq.capture_end(stream)
        hq.capture_begin(stream)
        steps64(w64, w64 + k64)
        g64_timed = hq.capture_end(stream)
        g64_warm.launch(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g64_timed.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t_step64p = e0.elapsed_time(e1) / k64
        for hx in hs64:
            if hx.query()["device_flags"] != 0:
                raise RuntimeError(f"device flags raised (FP64 pipeline): {hx.query()}")
            hx.destroy()
        g64_warm.destroy()
        g64_timed.destroy()
        del f64, tmp64, out64, tmps64, outs64, posb64
        fp64 = {"up_ms": t_up64, "down_ms": t_dn64, "rebuild_ms": t_rb64, "step_ms": t_step64,
                "bead_vectors_per_s": N * R / (t_step64 * 1e-3),
                "pipelined": {"step_ms": t_step64p, "bead_vectors_per_s": N * R / (t_step64p * 1e-3),
                              "steps": k64, "warmup": w64,
                              "what": f"the FP64 BD step (FP64 rebuild, FP64 records and vectors) on {npipe} "
                                      "handles, streams and position buffers, hipGraph, as the FP32 step"},
                "apply_only_bead_vectors_per_s": N * R / ((t_up64 + t_dn64) * 1e-3),
                "roofline": {"bound": "hbm", "kernel": sweep_kernel(R, lay, "double"), "bytes": int(pb64[1]),
                             "ms": t_p1_64, "achieved": pb64[1] / (t_p1_64 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": pb64[1] / (t_p1_64 * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "whole_sweep_up": {"bytes": int(nbytes64), "ms": t_up64,
                                                "frac": nbytes64 / (t_up64 * 1e-3) / 1e9 / HBM_PEAK_GBS}},
                "what": "FP64 transforms and vectors on the same workload (final positions): rebuild + Q~f + "
                        "Q~^T(Q~f) per step, eager launches on one stream (step_ms), and the pipelined graph "
                        "of whole steps (pipelined)"}
        log(f"sweeps: up {t_up:.3f} ms, down {t_dn:.3f} ms, rebuild {t_rb:.3f} ms; FP64 up {t_up64:.3f} "
            f"down {t_dn64:.3f} step {t_step64:.3f} ms (pipelined {t_step64p:.3f} ms)")
        nbytes = algorithmic_bytes(h, R)
        # the dominant kernel: the first tile phase's upward launch, timed with
        # HIP events around that launch on the stream it runs on
        pbytes = phase_bytes(h, R)
        assert sum(pbytes.values()) == nbytes
        p1 = []
        for _ in range(args.apply_reps):
            # a sweep queued just before keeps the GPU busy (no idle gap
            # before the timed launch, as in the step's graph)
            h.apply(f32, out=tmp, stream=stream, layout=lay)
            _, ms_ph = h.apply(f32, out=tmp, stream=stream, timed=True, layout=lay)
            p1.append(ms_ph[0])
        t_p1 = float(np.median(p1))
        achieved = pbytes[1] / (t_p1 * 1e-3) / 1e9
        log(f"first-phase upward launch: {t_p1:.3f} ms, {pbytes[1] / 1e9:.3f} GB -> {achieved:.0f} GB/s; "
            f"whole sweep {nbytes / (t_up * 1e-3) / 1e9:.0f} GB/s")
        # the measured streaming ceiling beside the published peak: the
        # library's streaming kernel with the dominant launch's read:write mix
        # (its algorithmic reads: vectors in, records, permutation; writes:
        # residue rows), the sweeps' non-temporal policy
        nd_k = h.node_data(with_G=False, with_geometry=False)
        ph1 = h.node_phase() == 1
        wbytes = 4 * R * int((nd_k["k"][ph1].astype(np.int64) - 3).sum())
        ceiling = stream_ceiling(hq, torch, pbytes[1] - wbytes, wbytes, stream)
        log(f"streaming ceiling {ceiling['achieved']:.0f} GB/s ({ceiling['read_bytes'] / 1e9:.2f} GB read, "
            f"{ceiling['write_bytes'] / 1e9:.2f} GB written in {ceiling['ms']:.3f} ms)")
        traffic, traffic_src = traffic_from_profile(opts, lay)
        log(f"traffic: {traffic} ({traffic_src})")
        q = h.query()
        legs = {}
        if not args.no_legs:
            for name in ("C2", "C3", "C5"):
                legs[name] = config_leg(hq, torch, W, name, stream, log=log)
                log(f"{name}: {json.dumps(legs[name])}")

    result = {
        "metric": METRIC,
        "value": N * R / (ms_step * 1e-3),
        "unit": "bead-vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"bd_step_m{m}_lognormal500_R{R}", "bodies": m, "beads": N, "nrhs": R,
                   "rows": wl.rows, **effective(opts), "autotuned": autotuned, "layout": lay,
                   "first_waves_per_cu": args.first_waves_per_cu,
                   "step": "rigid motion + FP64 rebuild + FP32 Q~f + FP32 Q~^T(Q~f), hipGraph of K steps",
                   "pipeline": (f"{npipe} handles on {npipe} streams and position buffers: consecutive steps' rebuilds and sweeps overlap"
                                if npipe > 1 else "one handle, one stream")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{sweep_kernel(R, lay, 'float')}: first tile phase of the upward FP32 sweep",
                     "bytes": int(pbytes[1]), "ms": t_p1,
                     "stream_ceiling": dict(ceiling, kernel_frac_of_ceiling=achieved / ceiling["achieved"]),
                     "whole_sweep": {"bytes": int(nbytes), "ms": t_up,
                                     "achieved": nbytes / (t_up * 1e-3) / 1e9}},
        "sweeps_ms": {"up_fp32": t_up, "down_fp32": t_dn, "rebuild_fp64": t_rb, "up_fp64": t_up64,
                      "down_fp64": t_dn64},
        "fp64": fp64,
        "apply_only_bead_vectors_per_s": N * R / ((t_up + t_dn) * 1e-3),
        "krylov": {"iters": kinfo["iters"], "iterations_run": k_launched,
                   "max_rel_residual": kinfo["max_rel_residual"], "ms_total": t_k,
                   "ms_per_iter": k_iter, "callback_ms": t_cb, "sweep_pair_ms": t_up + t_dn,
                   "per_iter_over_sweeps_and_callback": k_iter / (t_up + t_dn + t_cb),
                   "what": "hq_constrained_solve (Eqs. 1.5-1.6), FP32, CG to 1e-5, per-bead 3x3 SPD mobility "
                           "(torch callback), same workload and layout; per iteration = (total - one-iteration "
                           "solve) / (iterations run - 1); CG scalars on the device, convergence read every "
                           "4 iterations"},
        "transform_reuse": {"up_ms": t_rup, "down_ms": t_rdn, "step_ms": t_rup + t_rdn, "rebuild_ms": t_rb,
                            "bead_vectors_per_s": N * R / ((t_rup + t_rdn) * 1e-3),
                            "what": "hq_apply_rotated: Q~(Rot r) v = Q~(r) (Rot^T v) per body, no rebuild; "
                                    "a step of Q~^T(Q~ f) after rigid rotations, FP32, same workload"},
        "full_q": {"up_ms": t_fup, "down_ms": t_fdn, "bead_vectors_per_s": N * R / ((t_fup + t_fdn) * 1e-3),
                   "what": "hq_apply_full: Q v = [Q_Z v; Q~ v] and Q^T [r; w], FP32, same workload"},
        "fp32_rel_err_vs_fp64_oracle": err,
        "fp32_leak": leak,
        "tiles": q["tiles"], "phases": q["phases"],
    }
    if legs:
        result["configs"] = legs
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
