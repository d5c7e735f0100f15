"""Per-launch HBM traffic of a kernel from rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one counter per run) are read
from the counter CSVs of the kernel's run and scaled by what the same
counters read for a plain device-to-device copy of known size (the copy
reads and writes exactly its size).  The result goes into
profiles/traffic.json under a workload key, with a SHA-256 of the kernel's
sources and build script: bench.py reports the figure only while those
still hash to it, the batch is the same and the tile variant matches.

    python -m paper_2606_26547_amd.traffic --key NAME --kernel REGEX \\
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \\
        --copy-bytes N --batch B --tile T --sources FILE...

Each DIR is a rocprofv3 output directory holding *counter_collection.csv.
The copy the counters are calibrated on is this module's own:

    python -m paper_2606_26547_amd.traffic --copy-run BYTES

copies BYTES (a multiple of 4) from one device buffer to another six times.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")


def counter_mean(directory: str, counter: str, kernel: str, grid: int | None = None) -> tuple[float, int]:
    """Mean value of `counter` over the dispatches of kernels matching the
    regex `kernel` (and of grid size `grid` when given), and their count."""
    vals = []
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter or not re.search(kernel, r["Kernel_Name"]):
                    continue
                if grid is not None and int(r["Grid_Size"]) != grid:
                    continue
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise ValueError("no %s rows for %r in %s" % (counter, kernel, directory))
    return sum(vals) / len(vals), len(vals)


def sources_hash(sources: list[str]) -> str:
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in sources)).hexdigest()


def copy_run(nbytes: int, reps: int = 6):
    """The calibration copy: device to device, `reps` times."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()


def main(argv=None):
    import sys
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "--copy-run":
        copy_run(int(argv[1]))
        return
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--key", required=True)
    ap.add_argument("--kernel", required=True, help="regex of the kernel name")
    ap.add_argument("--grid", type=int, default=None, help="grid size (threads) of the dispatches to use")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--batch", type=int, required=True)
    ap.add_argument("--tile", default=None)
    ap.add_argument("--sources", nargs="+", required=True)
    a = ap.parse_args(argv)
    cf, _ = counter_mean(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw, _ = counter_mean(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    ff, wf = a.copy_bytes / (cf * 1024.0), a.copy_bytes / (cw * 1024.0)
    kf, nf = counter_mean(a.fetch, "FETCH_SIZE", a.kernel, a.grid)
    kw, nw = counter_mean(a.write, "WRITE_SIZE", a.kernel, a.grid)
    entry = {"sources": a.sources, "sha256": sources_hash(a.sources), "batch": a.batch, "tile": a.tile,
             "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
             "fetch_bytes": kf * 1024.0 * ff, "write_bytes": kw * 1024.0 * wf,
             "bytes_per_launch": kf * 1024.0 * ff + kw * 1024.0 * wf}
    t = json.load(open(TRAFFIC)) if os.path.exists(TRAFFIC) else {}
    t["note"] = ("HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, each scaled by the factor that "
                 "makes the same counter read the size of a device-to-device copy; valid while the kernel "
                 "sources hash to sha256")
    t["calibration"] = {"copy_bytes": a.copy_bytes, "fetch_size_kib": cf, "write_size_kib": cw,
                        "fetch_factor": ff, "write_factor": wf}
    t[a.key] = entry
    with open(TRAFFIC, "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps({a.key: entry, "calibration": t["calibration"]}, indent=1))


if __name__ == "__main__":
    main()
