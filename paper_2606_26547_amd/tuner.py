"""Configuration sweep and tuned-configuration selection.

This stands in for the paper's tuning loop (Sec. 3, Sec. 4.1): there, each
candidate approximation configuration is compiled, run by a user driver
that reports its quality of service (QoS) and time, and the search keeps the
fastest configuration whose QoS stays within a user bound (Sec. 5.2 uses
"baseline QoS minus 0.05").  Here every candidate is evaluated on the device
in one call (``hdc_eval_configs``: a persistent kernel, or the shared path
that ranks all configurations of an encoding type from one encoding), QoS is
classification accuracy on the sweep queries, and the bound is an accuracy
loss of at most ``budget_pts`` points against the plain (unapproximated)
configuration.

A configuration is (d_trunc, stride, start, dtype): the encoding and Hamming
reductions run over dimensions S = {start + j*stride < d_trunc} (reduction
perforation / truncated dimensionality, Sec. 4.2) with the encoding in
``dtype`` (Sec. 4.2 "Element Type Representation").
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import hdc

# relative cost of one encoded dimension per compute type on gfx950 (MFMA
# throughput: int8 and fp8 run at the same dense rate, bf16 at half)
DTYPE_COST = {"int8": 1.0, "fp8": 1.0, "bf16": 2.0}


@dataclasses.dataclass
class Result:
    cfg: tuple            # (d_trunc, stride, start, dtype)
    correct: int
    n: int
    device_us: float      # busy time reported by the sweep kernel (summed over work items)
    qps: float = 0.0      # standalone queries/s, filled for candidates that are re-timed

    @property
    def accuracy(self) -> float:
        return self.correct / max(1, self.n)

    @property
    def n_dims(self) -> int:
        d, k, s, _ = self.cfg
        return hdc.dims_count(s, d, k)

    @property
    def cost(self) -> float:
        return self.n_dims * DTYPE_COST[self.cfg[3]]


def sweep(X: torch.Tensor, F: int, truth: torch.Tensor, P: torch.Tensor, D: int, Cw: torch.Tensor,
          cfgs, tile: int = 0) -> list[Result]:
    """Evaluate every configuration in one hdc_eval_configs call, every
    configuration with the sweep tile variant `tile` (0 = the built-in
    per-configuration items; 4 = the shared path)."""
    cfgs = [tuple(c) for c in cfgs]
    res = hdc.eval_configs(X, F, truth, P, D, Cw, cfgs, tile=tile)
    return [Result(cfg, int(res["correct"][i]), int(res["n"][i]), float(res["device_us"][i]))
            for i, cfg in enumerate(cfgs)]


def sweep_loop(X: torch.Tensor, F: int, truth: torch.Tensor, P: torch.Tensor, D: int, Cw: torch.Tensor,
               cfgs) -> list[Result]:
    """The same evaluation with one hdc_classify call per configuration."""
    out = []
    for cfg in cfgs:
        d, k, s, t = cfg
        lab = hdc.classify(X, F, P, D, Cw, t, s, d, k)
        out.append(Result(tuple(cfg), int((lab == truth).sum().item()), X.shape[0], 0.0))
    return out


def time_config(cfg, X: torch.Tensor, F: int, P: torch.Tensor, D: int, Cw: torch.Tensor, reps: int = 5,
                tile: int = 0, shifted: dict | None = None) -> float:
    """Standalone queries/s of one configuration on batch X (median of
    reps).  ``shifted`` maps a compute type ("int8", "fp8") to the model's
    projection in the shifted form hdc.shift_projection writes for it; such
    configurations run on it as "int8shift" / "fp8shift".  ``tile`` is the
    int8 configurations' kernel shape."""
    d, k, s, t = cfg
    plain_t = t
    if shifted and t in shifted:
        t, P = hdc.SHIFTED[t], shifted[t]
    prep = hdc.Prepared(Cw, D, t, s, d, k, tile=tile if plain_t == "int8" else 0)
    labels = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    prep(X, F, P, labels)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        prep(X, F, P, labels)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    return X.shape[0] / float(np.median(ts))


def select_tuned(results: list[Result], plain_cfg, budget_pts: float = 1.0, timer=None, max_timed: int = 12):
    """Fastest configuration whose accuracy is within ``budget_pts`` points of
    the plain configuration's.  Candidates are ranked by encoded work
    (dimensions x dtype cost); the cheapest ones are re-timed standalone with
    ``timer(cfg) -> queries/s`` when a timer is given."""
    by_cfg = {r.cfg: r for r in results}
    plain = by_cfg[tuple(plain_cfg)]
    floor = plain.accuracy - budget_pts / 100.0
    ok = [r for r in {r.cfg: r for r in results}.values() if r.accuracy >= floor - 1e-12]
    ok.sort(key=lambda r: (r.cost, -r.accuracy))
    if timer is None:
        return ok[0], plain
    cand = ok[:max_timed]
    if plain not in cand:
        cand.append(plain)
    for r in cand:
        r.qps = timer(r.cfg)
    best = max(cand, key=lambda r: r.qps)
    return best, plain


def wall(fn):
    t = time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t
