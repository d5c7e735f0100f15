"""Tile autotuner: times every compiled tile variant of the kernels a
workload launches, on the device, and keeps the fastest per bucket.

A bucket is what one set of compiled variants covers: (kind, feature type,
compute type, compiled feature width, class tiles).  For each
shape, ``tune`` builds seeded synthetic operands of that shape (features,
+-1 projection rows, class hypervectors, for the sweep a configuration
list), runs every variant after a warm-up, checks that its result equals
the built-in variant's (every variant computes the same labels, encodings
or counts; a variant that differs is an error, not a candidate) and takes
the mean device time over ``reps`` launches.  A variant replaces the
built-in one only when it is faster by more than ``margin``.  ``autotune``
tunes a list of shapes; a ``TileTable`` holds the choices (read-only once
built) and the caller passes the chosen variant with each launch (the
library keeps no tile state).  ``save`` / ``load`` keep the table as JSON
together with the device name, and ``load`` refuses a table measured on
another device.
"""
from __future__ import annotations

import json
from dataclasses import asdict, dataclass, field

import numpy as np
import torch

from . import hdc


@dataclass
class Shape:
    kind: str                 # "encode", "classify" or "sweep"
    F: int
    K: int
    D: int
    n: int                    # queries per timed launch
    x_type: str = "int8"
    compute: str = "int8"
    cfgs: list | None = None  # sweep: the configuration list


@dataclass
class Choice:
    shape: Shape
    variants: dict = field(default_factory=dict)   # name -> mean ms
    chosen: int = 0
    chosen_name: str = ""
    default_name: str = ""


def _events(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def _operands(sh: Shape, seed: int):
    g = torch.Generator(device="cuda").manual_seed(seed)
    ld = max(64, (sh.F + 63) // 64 * 64)
    if sh.x_type == "fp32":
        X = torch.zeros((sh.n, ld), dtype=torch.float32, device="cuda")
        X[:, :sh.F] = torch.randn((sh.n, sh.F), device="cuda", generator=g)
    else:
        lo, hi = (-127, 128) if sh.x_type == "int8" else (0, 256)
        dt = torch.int8 if sh.x_type == "int8" else torch.uint8
        X = torch.zeros((sh.n, ld), dtype=dt, device="cuda")
        X[:, :sh.F] = torch.randint(lo, hi, (sh.n, sh.F), dtype=torch.int16, device="cuda", generator=g).to(dt)
    P = torch.zeros((sh.D, ld), dtype=torch.int8, device="cuda")
    P[:, :sh.F] = (torch.randint(0, 2, (sh.D, sh.F), dtype=torch.int8, device="cuda", generator=g) * 2 - 1)
    if sh.compute in ("int8shift", "fp8shift"):
        P = hdc.shift_projection(P, sh.F, compute=sh.compute)
    C = torch.randint(-(1 << 62), 1 << 62, (sh.K, (sh.D + 63) // 64), dtype=torch.int64, device="cuda",
                      generator=g)
    if sh.D % 64:
        C[:, -1] &= (1 << (sh.D % 64)) - 1
    return X, P, C


def tune(sh: Shape, reps: int = 5, margin: float = 0.03, seed: int = 1) -> Choice:
    """Time every variant of the bucket of ``sh``; the choice is returned."""
    variants = hdc.tile_variants(sh.kind, sh.x_type, sh.compute, sh.F, sh.K)
    names = hdc.TILE_NAMES[sh.kind]
    X, P, C = _operands(sh, seed)
    if sh.kind == "classify":
        prep = hdc.Prepared(C, sh.D, sh.compute)
        lab = torch.empty(sh.n, dtype=torch.int32, device="cuda")

        def run(v):
            prep.tile = v
            prep(X, sh.F, P, lab)
        result = lambda: lab.clone()                                             # noqa: E731
    elif sh.kind == "encode":
        H = torch.empty((sh.n, (sh.D + 63) // 64), dtype=torch.int64, device="cuda")
        run = lambda v: hdc.encode(X, sh.F, P, sh.D, sh.compute, out=H, tile=v)  # noqa: E731
        result = lambda: H.clone()                                               # noqa: E731
    else:
        truth = torch.randint(0, sh.K, (sh.n,), dtype=torch.int32, device="cuda")
        ws = torch.empty(int(hdc.lib().hdc_eval_configs_workspace_bytes(len(sh.cfgs), sh.F, sh.D, sh.K)),
                         dtype=torch.uint8, device="cuda")
        out = torch.empty(16 * len(sh.cfgs), dtype=torch.uint8, pin_memory=True)
        cfgs = [tuple(c[:4]) for c in sh.cfgs]
        arrs = {v: hdc.config_array(cfgs, v) for v in variants}      # built once, outside the timing

        def run(v):
            hdc.eval_configs(X, sh.F, truth, P, sh.D, C, arrs[v], ws=ws, out=out)
        result = lambda: torch.as_tensor(hdc.result_view(out, len(cfgs))["correct"].copy())  # noqa: E731
    ch = Choice(shape=sh)
    ref = None
    times = {}
    for v in variants:
        run(v)
        torch.cuda.synchronize()
        res = result()
        if ref is None:
            ref = res
        elif not torch.equal(res, ref):
            raise RuntimeError("tile variant %s of %s gives a different result" % (names[v], sh))
        times[v] = _events(lambda: run(v), reps)
    best = min(times, key=times.get)
    default = variants[0]
    if times[best] > times[default] * (1 - margin):
        best = default
    ch.variants = {names[v]: times[v] for v in variants}
    ch.chosen, ch.chosen_name, ch.default_name = best, names[best], names[default]
    return ch


def autotune(shapes: list[Shape], reps: int = 5, margin: float = 0.03) -> list[Choice]:
    return [tune(sh, reps, margin) for sh in shapes]


class TileTable:
    """Chosen variants keyed by (kind, x_type, compute, F, K); 0 (the
    built-in rule) for a shape that was not tuned.  Built once, then only
    read: the caller passes ``get(...)`` with each launch."""

    def __init__(self, entries: dict | None = None):
        self._t = dict(entries or {})

    @classmethod
    def from_choices(cls, choices: list[Choice]) -> "TileTable":
        return cls({(c.shape.kind, c.shape.x_type, c.shape.compute, c.shape.F, c.shape.K): c.chosen
                    for c in choices})

    def get(self, kind: str, x_type: str, compute: str, F: int, K: int) -> int:
        return self._t.get((kind, x_type, compute, F, K), 0)

    def __len__(self):
        return len(self._t)


def to_json(choices: list[Choice]) -> dict:
    return {"device": torch.cuda.get_device_name(0),
            "entries": [dict(asdict(c.shape), variants_ms=c.variants, variant=c.chosen, name=c.chosen_name,
                             default=c.default_name) for c in choices]}


def save(choices: list[Choice], path: str):
    with open(path, "w") as f:
        json.dump(to_json(choices), f, indent=1)


def load(path: str) -> TileTable:
    """A saved table (refused when it was measured on another device)."""
    with open(path) as f:
        t = json.load(f)
    if t.get("device") != torch.cuda.get_device_name(0):
        raise ValueError("tile table measured on %r, this device is %r" % (t.get("device"),
                                                                             torch.cuda.get_device_name(0)))
    return TileTable({(e["kind"], e["x_type"], e["compute"], e["F"], e["K"]): e["variant"] for e in t["entries"]})
