"""The copy-calibrated traffic record (paper_2606_26547_amd.traffic): the
per-dispatch counter means are taken over the matching kernel and grid only,
scaled by the factor that makes the copy read its own size, and the record
carries the hash of the kernel's sources; bench.py drops the figure once
those sources, the batch or the tile differ."""
import csv
import json
import os

from paper_2606_26547_amd import traffic


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], r)))


def test_counter_mean_filters_kernel_and_grid(tmp_path):
    d = str(tmp_path / "k")
    _write(d, [("k_encode<a>", 256, "FETCH_SIZE", 100.0), ("k_encode<a>", 256, "FETCH_SIZE", 300.0),
               ("k_encode<a>", 512, "FETCH_SIZE", 9999.0), ("other", 256, "FETCH_SIZE", 7.0),
               ("k_encode<a>", 256, "WRITE_SIZE", 5.0)])
    assert traffic.counter_mean(d, "FETCH_SIZE", r"k_encode<a>", 256) == (200.0, 2)
    assert traffic.counter_mean(d, "FETCH_SIZE", r"k_encode") == ((100 + 300 + 9999) / 3, 3)


def test_record_scales_by_the_copy_and_hashes_sources(tmp_path, monkeypatch):
    kib = 1 << 20                                     # a 1 GiB copy
    _write(str(tmp_path / "cf"), [("copyBuffer", 1, "FETCH_SIZE", kib / 2)])   # the counter reads half
    _write(str(tmp_path / "cw"), [("copyBuffer", 1, "WRITE_SIZE", kib)])
    _write(str(tmp_path / "kf"), [("k_x", 64, "FETCH_SIZE", 1000.0)])
    _write(str(tmp_path / "kw"), [("k_x", 64, "WRITE_SIZE", 10.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(traffic, "TRAFFIC", str(out))
    traffic.main(["--key", "w", "--kernel", "k_x", "--grid", "64", "--fetch", str(tmp_path / "kf"),
                  "--write", str(tmp_path / "kw"), "--copy-fetch", str(tmp_path / "cf"),
                  "--copy-write", str(tmp_path / "cw"), "--copy-bytes", str(1 << 30), "--batch", "8",
                  "--tile", "dma_2x2", "--sources", "bench.py"])
    rec = json.load(open(out))
    e = rec["w"]
    assert rec["calibration"]["fetch_factor"] == 2.0 and rec["calibration"]["write_factor"] == 1.0
    assert e["fetch_bytes"] == 1000 * 1024 * 2 and e["write_bytes"] == 10 * 1024
    assert e["bytes_per_launch"] == e["fetch_bytes"] + e["write_bytes"]
    assert e["sha256"] == traffic.sources_hash(["bench.py"]) and e["batch"] == 8 and e["tile"] == "dma_2x2"


def test_bench_uses_the_record_only_while_it_matches():
    """The committed record gives its figure for its own batch and tile
    while the kernel's sources still hash to it, and nothing otherwise."""
    import bench
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", "traffic.json")))
    key = bench.traffic_key("dma_2x3", "int8shift")
    assert key == "k_encode_classify_speech_b262144_dma_2x3_shift"
    e = rec[key]
    current = traffic.sources_hash(e["sources"]) == e["sha256"]
    v = bench.measured_traffic(key, e["batch"], e["tile"])
    assert v == (e["bytes_per_launch"] if current else None)
    assert bench.measured_traffic(key, e["batch"] + 1, e["tile"]) is None
    assert bench.measured_traffic(key, e["batch"], "reg_qt1") is None
    assert bench.measured_traffic("no such key", e["batch"], e["tile"]) is None
