"""The counter tooling on the CPU: traffic.py turns two rocprofv3 counter
runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch) into calibrated HBM bytes
per sweep and per first-phase launch, and bench.py reports a summary only
while it matches the sweep sources and the launch configuration.

Synthetic counter files with known values stand in for rocprofv3 output.
"""
import csv
import json
import os

import pytest

import bench
import traffic

MiB = 1024 * 1024


def _write_counters(dirname, counter, rows):
    os.makedirs(dirname, exist_ok=True)
    with open(os.path.join(dirname, "probe_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            # two partial values per dispatch (as per-XCD rows are), summed by the reader
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib / 2})
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib / 2})


UP1 = "void hq::(anonymous namespace)::k_up_lane<float, 1>(int const*)"
UPL = "void hq::k_up_np<float, 256, 1, 32, false>(int const*)"
DN1 = "void hq::(anonymous namespace)::k_down_lane<float, 1>(int const*)"
DNL = "void hq::k_down_np<float, 256, 1, 32, false>(int const*)"
COPY = "void at::native::vectorized_elementwise_kernel<4, copy>(float*)"


def _probe_rows(scale):
    """A copy, then three upward sweeps (first phase 1000 KiB, later 10) and
    three downward ones (first 800, later 20), times ``scale``; build kernels
    in between that the summary must ignore."""
    rows = [(COPY, 512 * 1024 * scale), ("hq::k_codes(int)", 5000.0), ("hq::k_units_walk(int)", 7.0)]
    for _ in range(traffic.PROBE_SWEEPS):
        rows += [(UP1, 1000.0 * scale), (UPL, 10.0 * scale)]
    for _ in range(traffic.PROBE_SWEEPS):
        rows += [(DN1, 800.0 * scale), (DNL, 20.0 * scale)]
    return rows


def test_is_sweep():
    for name in (UP1, UPL, "void hq::k_up_wide<float, 32, 32, 6, 3, 3, 1, true, false>(x)", "hq::k_up(int)"):
        assert traffic.is_sweep(name, "up") and not traffic.is_sweep(name, "down")
    for name in (DN1, DNL, "void hq::k_down_wide<double, 32>(x)"):
        assert traffic.is_sweep(name, "down") and not traffic.is_sweep(name, "up")
    for name in ("hq::k_units_walk(int)", "hq::k_upsweep(int)", "hq::k_bucket<float>(x)", COPY):
        assert not traffic.is_sweep(name, "up") and not traffic.is_sweep(name, "down")


def test_summarise_picks_first_phase_and_averages_sweeps():
    rows = [{"name": n, "value": v} for n, v in _probe_rows(1.0)]
    copy_kib, up, down, (n_up, u1), (n_dn, d1) = traffic.summarise(rows, "k_up_lane", "k_down_lane")
    assert copy_kib == 512 * 1024
    assert up == pytest.approx(1010.0) and down == pytest.approx(820.0)
    assert n_up == UP1 and u1 == pytest.approx(1000.0)
    assert n_dn == DN1 and d1 == pytest.approx(800.0)
    with pytest.raises(ValueError):
        traffic.summarise([r for r in rows if r["name"] != COPY], "k_up_lane", "k_down_lane")
    with pytest.raises(ValueError):
        traffic.summarise(rows, "k_up_wide", "k_down_lane")


def test_main_calibrates_both_counters(tmp_path, monkeypatch):
    # FETCH_SIZE reads half of the copied bytes, WRITE_SIZE all of them: the
    # calibrated bytes are 2 x fetch + 1 x write
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", _probe_rows(0.5))
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", _probe_rows(1.0))
    out = tmp_path / "t.json"
    monkeypatch.setattr("sys.argv", ["traffic.py", str(tmp_path / "f"), str(tmp_path / "w"), str(out),
                                     "--command", "cmd", "--options", "tile_units=64,layout=rows",
                                     "--first-up", "k_up_lane", "--first-down", "k_down_lane",
                                     "--workload", "w1"])
    traffic.main()
    d = json.loads(out.read_text())
    assert d["copy"]["fetch_factor"] == pytest.approx(2.0) and d["copy"]["write_factor"] == pytest.approx(1.0)
    assert d["up_phase1"]["kernel"] == UP1
    # fetch 500 KiB x 2 + write 1000 KiB x 1 per first-phase upward launch
    assert d["up_phase1"]["hbm_bytes"] == pytest.approx((500 * 2 + 1000) * 1024)
    assert d["down_sweep"]["hbm_bytes"] == pytest.approx((410 * 2 + 820) * 1024)
    assert d["workload"] == "w1" and d["source_sha256"] == traffic.sweep_source_hash()


def test_leg_traffic_only_for_matching_sources_and_options(tmp_path, monkeypatch):
    class Wl:
        name = "w1"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    opts = {"tile_units": 64, "run_nodes": 48, "waves_per_cu": 8, "later_tile_units": 0, "leaf_size": 1}
    assert bench.leg_traffic(Wl, opts, 1) == (None, "no counter summary")
    (tmp_path / "profiles").mkdir()
    prof = {"command": "cmd", "source_sha256": traffic.sweep_source_hash(), "options": "tile_units=64,layout=rows",
            "up_phase1": {"hbm_bytes": 123.0}}
    path = tmp_path / "profiles" / "traffic_up_sweep_w1.json"
    path.write_text(json.dumps(prof))
    # below 8 RHS the run length does not shape the first-phase launch
    assert bench.leg_traffic(Wl, opts, 1) == (123.0, "cmd")
    assert bench.leg_traffic(Wl, dict(opts, run_nodes=32), 1) == (123.0, "cmd")
    b, why = bench.leg_traffic(Wl, dict(opts, tile_units=32), 1)
    assert b is None and "tile_units=32" in why
    # at 8 or more it does
    b, why = bench.leg_traffic(Wl, opts, 16)
    assert b is None and "run_nodes=48" in why
    path.write_text(json.dumps(dict(prof, source_sha256="0" * 64)))
    b, why = bench.leg_traffic(Wl, opts, 1)
    assert b is None and "changed" in why
