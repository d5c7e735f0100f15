"""The benchmark's last stdout line is a compact summary of its full record
(the full record goes to a file): it keeps the contract fields and stays
short enough to survive a truncated capture of the output."""
import json

import bench


def _full_record():
    rl = {"bound": "mfma", "kernel": "k_encode<int8, classify>", "achieved": 2498.123456, "peak": 5000.0,
          "unit": "TOP/s", "frac": 0.4996246, "traffic": 389512345.0, "tile": "dma_2x2",
          "traffic_unit": "bytes per launch (HBM read + write, profiles/traffic.json)", "ms_per_launch": 1.3256,
          "ops_per_launch": 3.31e12}
    ladder_row = {"flip_rate": 0.0089, "accuracy": 0.914, "ms_batch": 2.2, "queries_per_s": 1.2e8}
    rec = {
        "metric": "queries/s (encode+Hamming argmin) plain vs tuned at <=1% acc loss; p99 ms",
        "value": 196812345.678, "unit": "queries/s", "n_gpus": 1, "steps": 20, "warmup": 3,
        "ms_per_step": 1.331987, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic (seeded c2 Gaussian-mixture generator; ISOLET-shaped, no real dataset)",
        "config": {"workload": "x" * 200, "F": 617, "K": 26, "D": 10240, "batch": 262144,
                   "parallelism": "none (1 GPU)"},
        "accuracy_plain": 0.9141, "tiles": [{"big": "y" * 2000}], "roofline": rl,
        "train": {"ms": 0.5, "n_train": 6238},
        "sweep": {"slots": 256, "ms": 1.9, "roofline": dict(rl, frac=0.14)},
        "bundle": {"ms": 0.3, "GB_s": 4000.0, "roofline": dict(rl, bound="hbm", frac=0.5)},
        "plain_fp32": {"queries_per_s": 1e8, "accuracy": 0.99, "roofline": dict(rl, frac=0.2)},
        "tuned": {"config": {"d_trunc": 8192, "stride": 2, "start": 0, "dtype": "int8"}, "value": 4.7e8,
                  "ms_per_step": 0.56, "accuracy": 0.906, "speedup_vs_plain": 2.4, "sweep_accuracy": 0.9,
                  "sweep_accuracy_plain": 0.91, "rule": "z" * 100},
        "latency": {"plain": {"p50_ms": 0.27, "p99_ms": 0.4, "queries_per_call": 1559},
                    "tuned": {"p50_ms": 0.2, "p99_ms": 0.3, "queries_per_call": 1559}},
        "p50_ms": 0.27, "p99_ms": 0.4,
        "hamming_unfused": {n: {"queries": 1 << 20, "mfma": {"ms": 0.3, "GB_s": 4400.0},
                                "popcount": {"ms": 1.0, "GB_s": 1250.0}, "agree": True}
                            for n in ("speech K=26 D=10240", "image K=10 D=8192", "K=100 D=10240")},
        "adc": {"roofline": dict(rl, frac=0.3), "big": ["w" * 500]},
        "cosine": {"roofline": dict(rl, frac=0.4), "big": ["w" * 500]},
        "retrain": {"roofline": dict(rl, frac=0.2), "test_accuracy_by_epoch": [0.9] * 7},
        "encode_side": {"big": "v" * 3000},
        "ladder": {wl: {t: dict(ladder_row) for t in ("int8", "bf16", "fp8", "fp8split")} | {"grid": [1] * 300}
                   for wl in ("speech", "image")},
        "serving": {m: {"p50_ms": 0.5, "p99_ms": 1.5, "queries_per_s": 870000.0, "requests": 6000}
                    for m in ("plain", "tuned")} | {"models": ["u" * 300] * 8},
        "cpu_baseline": {"value": 7300.0, "unit": "queries/s", "cores": 16, "kind": "oracle",
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor", "host_cpus": 256,
                         "sample": "first 98304 queries of the batch, plain config (exact int encode + "
                                   "bit-by-bit Hamming + argmin), 13.4s",
                         "labels_agree_with_gpu": 1.0, "tuned_value": 20000.0, "single_thread_value": 460.0,
                         "rows": {"r%d" % i: {"sample": "s" * 200} for i in range(6)}},
        "full_record": "gpurun_out/bench_full.json",
    }
    return rec


def test_summary_line_is_short_and_keeps_the_contract_fields():
    rec = _full_record()
    line = json.dumps(bench.compact(rec))
    assert len(line) < 4096, len(line)
    c = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in c, k
    assert c["config"]["workload"] == rec["config"]["workload"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in c["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample", "cpu_model"):
        assert k in c["cpu_baseline"], k
    assert c["tuned"]["config"]["d_trunc"] == 8192
    assert c["extras"]["ladder"]["speech"]["fp8split"]["flip_rate"] == 0.0089
    assert abs(c["value"] - rec["value"]) / rec["value"] < 1e-3


def test_summary_of_a_minimal_record():
    rec = {k: v for k, v in _full_record().items()
           if k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "config", "roofline")}
    c = bench.compact(rec)
    assert c["value"] > 0 and "extras" not in c
