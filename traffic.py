"""HBM traffic of the sweeps from hardware counters.

Two rocprofv3 counter runs of ``bench.py --probe`` (or ``--probe-leg C2|C3|C5``;
one with FETCH_SIZE, one with WRITE_SIZE; both in KiB per dispatch) are turned
into the bytes one upward and one downward FP32 sweep move to and from HBM, in
total and for the launch of the first tile phase (the dominant kernel: the
wide sweep at 8 or more right-hand sides, the lane sweep below).  Each counter
is scaled by what it reads for the probe's device copy of 512 MiB (bytes it
must read and write), and the summary records a hash of the sweep sources so
that a reader can tell whether it still describes the current kernels.

    python traffic.py FETCH_DIR WRITE_DIR OUT.json --command "..." --options "..."
        [--first-up k_up_lane --first-down k_down_lane --workload NAME]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1708_08427_amd")
COPY_BYTES = 128 * 1024 * 1024 * 4  # the probe's float32 copy
PROBE_SWEEPS = 3


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("hq_apply.hip", "hq_common.h", "hq_buffer.h"):
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _read(dirname, counter):
    files = glob.glob(os.path.join(dirname, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise FileNotFoundError(f"expected one counter_collection.csv under {dirname}, found {files}")
    per = {}
    for fn in files:
        with open(fn) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                key = (fn, int(r["Dispatch_Id"]))
                e = per.setdefault(key, {"name": r["Kernel_Name"], "value": 0.0})
                e["value"] += float(r["Counter_Value"])
    return list(per.values())


def first_phase(rows, kernel):
    """The first tile phase's launches: the instantiation of ``kernel`` that
    carries the most counted bytes (later phases use another one); returns
    its name and the mean per launch."""
    groups = {}
    for r in rows:
        if kernel in r["name"]:
            groups.setdefault(r["name"], []).append(r["value"])
    if not groups:
        raise ValueError(f"no {kernel} launches")
    name = max(groups, key=lambda n: sum(groups[n]))
    return name, sum(groups[name]) / len(groups[name])


def is_sweep(name, direction):
    """A launch of one of the sweep kernels of a direction ("up" or "down"):
    wide, lane-group, node-parallel or narrow, any tile phase."""
    return re.search(rf"hq::(\(anonymous namespace\)::)?k_{direction}(_wide|_lane|_np)?[<(]", name) is not None


def summarise(rows, first_up="k_up_wide", first_down="k_down_wide"):
    copies = [r for r in rows if "copy" in r["name"].lower() and "hq::" not in r["name"]]
    if not copies:
        raise ValueError("the probe's copy kernel is missing")
    copy_kib = max(r["value"] for r in copies)
    up = sum(r["value"] for r in rows if is_sweep(r["name"], "up")) / PROBE_SWEEPS
    down = sum(r["value"] for r in rows if is_sweep(r["name"], "down")) / PROBE_SWEEPS
    return copy_kib, up, down, first_phase(rows, first_up), first_phase(rows, first_down)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("out")
    ap.add_argument("--command", required=True)
    ap.add_argument("--options", required=True, help="launch configuration of the probe (its 'options' field)")
    ap.add_argument("--first-up", default="k_up_wide", help="kernel of the first phase's upward launch")
    ap.add_argument("--first-down", default="k_down_wide", help="kernel of the first phase's downward launch")
    ap.add_argument("--workload", default="bd_m4096_lognormal500_R32")
    a = ap.parse_args()
    cf, uf, df, (n_up, u1f), (n_dn, d1f) = summarise(_read(a.fetch_dir, "FETCH_SIZE"), a.first_up, a.first_down)
    cw, uw, dw, (_, u1w), (_, d1w) = summarise(_read(a.write_dir, "WRITE_SIZE"), a.first_up, a.first_down)
    ff = COPY_BYTES / (cf * 1024.0)
    fw = COPY_BYTES / (cw * 1024.0)
    res = {
        "command": a.command,
        "workload": a.workload,
        "source_sha256": sweep_source_hash(),
        "options": a.options,
        "copy": {"bytes_each_way": COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
                 "fetch_factor": ff, "write_factor": fw},
        "up_sweep": {"fetch_kib": uf, "write_kib": uw,
                     "hbm_bytes": uf * 1024.0 * ff + uw * 1024.0 * fw},
        "down_sweep": {"fetch_kib": df, "write_kib": dw,
                       "hbm_bytes": df * 1024.0 * ff + dw * 1024.0 * fw},
        "up_phase1": {"kernel": n_up, "fetch_kib": u1f, "write_kib": u1w,
                      "hbm_bytes": u1f * 1024.0 * ff + u1w * 1024.0 * fw},
        "down_phase1": {"kernel": n_dn, "fetch_kib": d1f, "write_kib": d1w,
                        "hbm_bytes": d1f * 1024.0 * ff + d1w * 1024.0 * fw},
    }
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
