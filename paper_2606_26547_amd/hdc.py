"""Thin Python binding of libhdc.so (include/hdc.h).

Argument marshalling only: torch supplies device memory and the current
stream; every step of the hot path runs in the library's HIP kernels.  The
library is loaded from the package directory; if it is missing this module
raises at import time, so no call can silently fall back to another
implementation.

Layout helpers pad features and projections to the leading dimensions the
kernels require (a multiple of 64 elements); the pad columns are ignored by
the kernels.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhdc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhdc.so is not built (%s); run __graft_entry__.build() or "
                      "python paper_2606_26547_amd/build.py" % LIB_PATH)

_lib = C.CDLL(LIB_PATH)

INT8, UINT8, BF16, FP8_E4M3, FP32, FP8_SPLIT, INT8_SHIFTED, FP8_SHIFTED = 0, 1, 2, 3, 4, 5, 6, 7
DTYPE = {"int8": INT8, "uint8": UINT8, "bf16": BF16, "fp8": FP8_E4M3, "fp32": FP32, "fp8split": FP8_SPLIT,
         "int8shift": INT8_SHIFTED, "fp8shift": FP8_SHIFTED}
# the shifted compute type of each plain one (hdc_shift_projection)
SHIFTED = {"int8": "int8shift", "fp8": "fp8shift"}
STATUS = {0: "HDC_OK", 1: "HDC_ERR_INVALID", 2: "HDC_ERR_UNSUPPORTED", 3: "HDC_ERR_WORKSPACE",
          4: "HDC_ERR_DEVICE"}
EXPORTS = ["hdc_status_string", "hdc_dims_count", "hdc_encode", "hdc_encode_tiled", "hdc_bundle_workspace_bytes",
           "hdc_bundle", "hdc_bundle_noalloc_limit_bytes", "hdc_bundle_noalloc", "hdc_hamming_argmin", "hdc_hamming_workspace_bytes", "hdc_hamming_prepare",
           "hdc_hamming_argmin_prepared", "hdc_classify_workspace_bytes", "hdc_classify_scratch_bytes", "hdc_classify",
           "hdc_classify_prepare", "hdc_classify_prepared",
           "hdc_eval_configs_workspace_bytes", "hdc_eval_configs", "hdc_device_clock_hz",
           "hdc_convert_features", "hdc_retrain_workspace_bytes", "hdc_class_acc", "hdc_retrain_epoch",
           "hdc_adc_argmax",
           "hdc_cosine_workspace_bytes", "hdc_cosine_prepare", "hdc_cosine_argmax_prepared",
           "hdc_feature_perforate", "hdc_level_quantize", "hdc_level_id_encode",
           "hdc_tile_variants", "hdc_shift_projection",
           "hdc_adc_workspace_bytes", "hdc_adc_prepare", "hdc_adc_argmax_prepared"]


class Dims(C.Structure):
    _fields_ = [("start", C.c_int32), ("end", C.c_int32), ("stride", C.c_int32)]


class Adc(C.Structure):
    _fields_ = [("res_bits", C.c_int32), ("step", C.c_int32), ("floor", C.c_int32), ("ceil", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("d_trunc", C.c_int32), ("stride", C.c_int32), ("start", C.c_int32), ("dtype", C.c_int32),
                ("tile_id", C.c_int32)]


class ConfigResult(C.Structure):
    _fields_ = [("correct", C.c_int32), ("n", C.c_int32), ("device_us", C.c_double)]


# host layout of hdc_config_result as a numpy record
RESULT_DTYPE = np.dtype([("correct", np.int32), ("n", np.int32), ("device_us", np.float64)])


class HDCError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s: %s" % (where, _lib.hdc_status_string(code).decode()))
        self.code = code


_p, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_lib.hdc_status_string.restype = C.c_char_p
_lib.hdc_status_string.argtypes = [C.c_int]
_lib.hdc_dims_count.restype = _i32
_lib.hdc_dims_count.argtypes = [Dims]
_lib.hdc_encode.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, _p, _i32, _i64, C.c_int, Dims, _p, _i64]
_lib.hdc_encode_tiled.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, _p, _i32, _i64, C.c_int, Dims, _p, _i64, _i32]
_lib.hdc_bundle_workspace_bytes.restype = _sz
_lib.hdc_bundle_workspace_bytes.argtypes = [_i64, _i32, _i32]
_lib.hdc_bundle.argtypes = [_p, _p, _i64, _i32, _i64, _p, _i32, _p, _i64, _p, _p, _sz]
_lib.hdc_bundle_noalloc_limit_bytes.restype = _sz
_lib.hdc_bundle_noalloc_limit_bytes.argtypes = []
_lib.hdc_bundle_noalloc.argtypes = [_p, _p, _i64, _i32, _i64, _p, _i32, _p, _i64, _p]
_lib.hdc_hamming_argmin.argtypes = [_p, _p, _i64, _i64, _p, _i32, _i64, _i32, Dims, _p, _p, _p]
_lib.hdc_hamming_workspace_bytes.restype = _sz
_lib.hdc_hamming_workspace_bytes.argtypes = [Dims, _i32]
_lib.hdc_hamming_prepare.argtypes = [_p, _p, _i32, _i64, Dims, _p, _sz]
_lib.hdc_hamming_argmin_prepared.argtypes = [_p, _p, _i64, _i64, _i32, Dims, _p, _p, _p, _p, _sz]
_lib.hdc_classify_workspace_bytes.restype = _sz
_lib.hdc_classify_workspace_bytes.argtypes = [_i32, _i32]
_lib.hdc_classify_scratch_bytes.restype = _sz
_lib.hdc_classify_scratch_bytes.argtypes = [_i64, _i32, _i32]
_lib.hdc_classify.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, _p, _i32, _i64, C.c_int, Dims, _p, _i32,
                              _i64, _p, _p, _p, _sz, _p, _sz, _i32]
_lib.hdc_classify_prepare.argtypes = [_p, _p, _i32, _i64, Dims, _p, _sz]
_lib.hdc_classify_prepared.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, _p, _i32, _i64, C.c_int, Dims, _i32,
                                       _p, _p, _p, _sz, _p, _sz, _i32]
_lib.hdc_eval_configs_workspace_bytes.restype = _sz
_lib.hdc_eval_configs_workspace_bytes.argtypes = [_i32, _i32, _i32, _i32]
_lib.hdc_eval_configs.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, _p, _p, _i32, _i64, _p, _i32, _i64,
                                  _p, _i32, _p, _p, _sz, _i32]
_lib.hdc_device_clock_hz.restype = C.c_double
_lib.hdc_device_clock_hz.argtypes = []
_lib.hdc_convert_features.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, C.c_int, _p]
_lib.hdc_adc_argmax.argtypes = [_p, _p, _i64, _i64, _p, _i32, _i64, Dims, Adc, _p, _p, _p]
_lib.hdc_retrain_workspace_bytes.restype = _sz
_lib.hdc_retrain_workspace_bytes.argtypes = [_i64, _i32, _i32]
_lib.hdc_class_acc.argtypes = [_p, _p, _i64, _i32, _i64, _p, _i32, _p, _p, _i64, _p, _sz]
_lib.hdc_retrain_epoch.argtypes = [_p, _p, _i64, _i32, _i64, _p, _p, _i32, _p, _p, _i64, _p, _p, _sz]
_lib.hdc_adc_workspace_bytes.restype = _sz
_lib.hdc_adc_workspace_bytes.argtypes = [Dims, _i32]
_lib.hdc_adc_prepare.argtypes = [_p, _p, _i32, _i64, Dims, _p, _sz]
_lib.hdc_adc_argmax_prepared.argtypes = [_p, _p, _i64, _i64, _i32, Dims, Adc, _p, _p, _p, _p, _sz]
_lib.hdc_tile_variants.restype = _i32
_lib.hdc_tile_variants.argtypes = [C.c_int, C.c_int, C.c_int, _i32, _i32, _p, _i32]
_lib.hdc_shift_projection.argtypes = [_p, _p, _i32, _i32, _i64, C.c_int, _p, _i64]
_lib.hdc_feature_perforate.argtypes = [_p, _p, C.c_int, _i64, _i32, _i64, Dims, _p, _i64]
_lib.hdc_level_quantize.argtypes = [_p, _p, _i64, _i32, _i64, _p, _p, _i32, _p, _i64]
_lib.hdc_level_id_encode.argtypes = [_p, _p, _i64, _i32, _i64, _p, _i64, _p, _i32, _i64, _i32, _p, _i64]
_lib.hdc_cosine_workspace_bytes.restype = _sz
_lib.hdc_cosine_workspace_bytes.argtypes = [Dims, _i32]
_lib.hdc_cosine_prepare.argtypes = [_p, _p, _i32, _i64, Dims, _p, _sz]
_lib.hdc_cosine_argmax_prepared.argtypes = [_p, _p, _i64, _i64, _i32, Dims, _p, _p, _p, _p, _sz]
for _name in EXPORTS:
    assert hasattr(_lib, _name)


def lib():
    return _lib


def _check(code: int, where: str):
    if code != 0:
        raise HDCError(code, where)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _xtype(t: torch.Tensor) -> int:
    return {torch.int8: INT8, torch.uint8: UINT8, torch.float32: FP32}[t.dtype]


def dims_count(start: int, end: int, stride: int) -> int:
    return int(_lib.hdc_dims_count(Dims(start, end, stride)))


def words(nbits: int) -> int:
    return max(1, (nbits + 63) // 64)


def pad_cols(a, device="cuda", mult: int = 64) -> torch.Tensor:
    """Copy a 2-D array into a zero-padded device tensor whose row pitch is a
    multiple of ``mult`` elements (the layout the kernels read)."""
    t = torch.as_tensor(np.ascontiguousarray(a)) if isinstance(a, np.ndarray) else a
    n, F = t.shape
    ld = max(mult, (F + mult - 1) // mult * mult)
    out = torch.zeros((n, ld), dtype=t.dtype, device=device)
    out[:, :F] = t.to(device)
    return out


class Model:
    """Device-resident projection (and, once trained, class hypervectors)."""

    def __init__(self, P, K: int, device="cuda"):
        P = np.asarray(P) if not isinstance(P, torch.Tensor) else P
        self.D, self.F = int(P.shape[0]), int(P.shape[1])
        self.K = int(K)
        self.P = pad_cols(P, device)
        self.C = None
        self.counts = None


def encode(X: torch.Tensor, F: int, P: torch.Tensor, D: int, compute="int8", start=0, end=None, stride=1,
           out: torch.Tensor | None = None, tile: int = 0) -> torch.Tensor:
    """hdc_encode_tiled (hdc_encode for tile 0): packed sign bits
    [n][words(|S|)] (uint64 viewed as int64)."""
    end = D if end is None else end
    nd = dims_count(start, end, stride)
    n = X.shape[0]
    if out is None:
        out = torch.zeros((n, words(nd)), dtype=torch.int64, device=X.device)
    _check(_lib.hdc_encode_tiled(_stream(), _ptr(X), _xtype(X), n, F, X.shape[1], _ptr(P), D, P.shape[1],
                                 DTYPE[compute], Dims(start, end, stride), _ptr(out), out.shape[1], int(tile)),
           "hdc_encode")
    return out


def shift_supported(kind: str, F: int, K: int, compute: str = "int8shift", x_type: str = "int8") -> bool:
    """Whether a shifted compute type ("int8shift", "fp8shift") has kernels
    for the (kind, x_type, F, K) bucket."""
    buf = (C.c_int32 * 8)()
    return _lib.hdc_tile_variants(KERNEL[kind], DTYPE[x_type], DTYPE[compute], F, K, buf, 8) > 0


def shift_projection(P: torch.Tensor, F: int, out: torch.Tensor | None = None,
                     compute: str = "int8shift") -> torch.Tensor:
    """hdc_shift_projection: the projection as the shifted compute type
    reads it (p + 1 in the F feature columns, as int8 for "int8shift" or
    E4M3 bytes for "fp8shift"; 0 in the pad columns), same layout."""
    if out is None:
        out = torch.empty_like(P)
    _check(_lib.hdc_shift_projection(_stream(), _ptr(P), P.shape[0], F, P.shape[1], DTYPE[compute], _ptr(out),
                                     out.shape[1]), "hdc_shift_projection")
    return out


def bundle(H: torch.Tensor, nbits: int, labels: torch.Tensor, K: int, ws: torch.Tensor | None = None):
    """hdc_bundle: class hypervectors [K][words(nbits)] and class sizes."""
    W = words(nbits)
    # every word of every class, and every class size, is written by the call
    Cw = torch.empty((K, W), dtype=torch.int64, device=H.device)
    counts = torch.empty(K, dtype=torch.int32, device=H.device)
    need = int(_lib.hdc_bundle_workspace_bytes(H.shape[0], nbits, K))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=H.device)
    _check(_lib.hdc_bundle(_stream(), _ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), K, _ptr(Cw),
                           Cw.shape[1], _ptr(counts), _ptr(ws), ws.numel()), "hdc_bundle")
    return Cw, counts


def bundle_noalloc(H: torch.Tensor, nbits: int, labels: torch.Tensor, K: int, Cw: torch.Tensor | None = None,
                   counts: torch.Tensor | None = None):
    """hdc_bundle_noalloc: hdc_bundle on the library's own per-device
    scratch (no workspace); fills Cw [K][words(nbits)] and counts [K] (the
    tensors are allocated here when not given)."""
    if Cw is None:
        Cw = torch.empty((K, words(nbits)), dtype=torch.int64, device=H.device)
    if counts is None:
        counts = torch.empty(K, dtype=torch.int32, device=H.device)
    _check(_lib.hdc_bundle_noalloc(_stream(), _ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), K, _ptr(Cw),
                                   Cw.shape[1], _ptr(counts)), "hdc_bundle_noalloc")
    return Cw, counts


def hamming_argmin(Q: torch.Tensor, Cw: torch.Tensor, start: int, end: int, stride: int = 1,
                   with_min=False, with_dists=False, nbits: int | None = None):
    """hdc_hamming_argmin; nbits (the hypervector length) defaults to the
    longest the row pitches of Q and Cw hold."""
    n, K = Q.shape[0], Cw.shape[0]
    if nbits is None:
        nbits = 64 * min(Q.shape[1], Cw.shape[1])
    lab = torch.empty(n, dtype=torch.int32, device=Q.device)
    mn = torch.empty(n, dtype=torch.int32, device=Q.device) if with_min else None
    dists = torch.empty((n, K), dtype=torch.int32, device=Q.device) if with_dists else None
    _check(_lib.hdc_hamming_argmin(_stream(), _ptr(Q), n, Q.shape[1], _ptr(Cw), K, Cw.shape[1], nbits,
                                   Dims(start, end, stride), _ptr(lab), _ptr(mn), _ptr(dists)),
           "hdc_hamming_argmin")
    return lab, mn, dists


def hamming_workspace_bytes(start: int, end: int, stride: int, K: int) -> int:
    return int(_lib.hdc_hamming_workspace_bytes(Dims(start, end, stride), K))


class HammingPrepared:
    """Class hypervectors of one (classes, perforation) turned into the
    matrix-core operand once; each call searches a batch of query
    hypervectors against them (hdc_hamming_argmin_prepared)."""

    def __init__(self, Cw: torch.Tensor, start: int, end: int, stride: int = 1):
        self.K, self.perf = Cw.shape[0], Dims(start, end, stride)
        need = hamming_workspace_bytes(start, end, stride, self.K)
        self.ws = torch.empty(max(need, 16), dtype=torch.uint8, device=Cw.device)
        _check(_lib.hdc_hamming_prepare(_stream(), _ptr(Cw), self.K, Cw.shape[1], self.perf, _ptr(self.ws),
                                        self.ws.numel()), "hdc_hamming_prepare")

    def __call__(self, Q: torch.Tensor, with_min=False, with_dists=False, out: torch.Tensor | None = None):
        n = Q.shape[0]
        if Q.shape[1] % 2:                      # the search wants an even row pitch
            Q = torch.nn.functional.pad(Q, (0, 1))
        lab = out if out is not None else torch.empty(n, dtype=torch.int32, device=Q.device)
        mn = torch.empty(n, dtype=torch.int32, device=Q.device) if with_min else None
        dists = torch.empty((n, self.K), dtype=torch.int32, device=Q.device) if with_dists else None
        _check(_lib.hdc_hamming_argmin_prepared(_stream(), _ptr(Q), n, Q.shape[1], self.K, self.perf, _ptr(lab),
                                                _ptr(mn), _ptr(dists), _ptr(self.ws), self.ws.numel()),
               "hdc_hamming_argmin_prepared")
        return lab, mn, dists


def feature_perforate(X: torch.Tensor, F: int, start: int, end: int, stride: int = 1,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """hdc_feature_perforate: the feature columns {start + j*stride < end}
    of X (int8 / uint8 / float32 rows, or projection rows P) as a dense
    matrix whose pitch (a multiple of 64 elements) the encoder accepts."""
    nf = dims_count(start, end, stride)
    ldy = max(64, (nf + 63) // 64 * 64)
    if out is None:
        out = torch.empty((X.shape[0], ldy), dtype=X.dtype, device=X.device)
    _check(_lib.hdc_feature_perforate(_stream(), _ptr(X), _xtype(X), X.shape[0], F, X.shape[1],
                                      Dims(start, end, stride), _ptr(out), out.shape[1]), "hdc_feature_perforate")
    return out


def level_quantize(X: torch.Tensor, lo: torch.Tensor, hi: torch.Tensor, L: int,
                   out: torch.Tensor | None = None) -> torch.Tensor:
    """hdc_level_quantize: levels [n][F] (uint16 values in an int16 tensor),
    row pitch rounded up to 8 (as hdc_level_id_encode reads them); the
    returned tensor is the [n][F] view."""
    n, F = X.shape
    if out is None:
        out = torch.zeros((n, (F + 7) // 8 * 8), dtype=torch.int16, device=X.device)[:, :F]
    _check(_lib.hdc_level_quantize(_stream(), _ptr(X), n, F, X.stride(0), _ptr(lo), _ptr(hi), L, _ptr(out),
                                   out.stride(0)), "hdc_level_quantize")
    return out


def level_id_encode(lev: torch.Tensor, ID: torch.Tensor, LV: torch.Tensor, D: int,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """hdc_level_id_encode: packed Level-ID hypervectors [n][ceil(D/64)].
    lev may be a column view of a row-major tensor whose pitch is a
    multiple of 8; other layouts are copied into one."""
    n, F = lev.shape
    if lev.stride(1) != 1 or lev.stride(0) % 8 or lev.stride(0) < F or lev.data_ptr() % 16:
        ld = (F + 7) // 8 * 8
        buf = torch.zeros((n, ld), dtype=lev.dtype, device=lev.device)
        buf[:, :F] = lev
        lev = buf[:, :F]
    W = (D + 63) // 64
    if out is None:
        out = torch.empty((n, W), dtype=torch.int64, device=lev.device)
    _check(_lib.hdc_level_id_encode(_stream(), _ptr(lev), n, F, lev.stride(0), _ptr(ID), ID.shape[1], _ptr(LV),
                                    LV.shape[0], LV.shape[1], D, _ptr(out), out.shape[1]), "hdc_level_id_encode")
    return out


KERNEL = {"encode": 0, "classify": 1, "sweep": 2}
TILE_NAMES = {"encode": {1: "dma_2x2", 2: "dma_1x1", 3: "reg_qt1", 4: "reg_qt2"},
              "classify": {1: "dma_2x2", 2: "dma_1x1", 3: "reg_qt1", 4: "reg_qt2", 5: "dma_2x3"},
              "sweep": {1: "items_128", 2: "items_256", 3: "items_256_dma", 4: "shared"}}


def tile_variants(kind: str, x_type: str, compute: str, F: int, K: int) -> list[int]:
    """hdc_tile_variants: the variant ids of a bucket, the built-in one first."""
    buf = (C.c_int32 * 8)()
    n = _lib.hdc_tile_variants(KERNEL[kind], DTYPE[x_type], DTYPE[compute], F, K, buf, 8)
    if n < 0:
        raise HDCError(1, "hdc_tile_variants")
    return list(buf[:n])


class AdcPrepared:
    """Class hypervectors of one (classes, perforation) as the matrix-core
    operand of the ADC-chunked similarity; each call searches a batch of
    query hypervectors under an ADC setting (hdc_adc_argmax_prepared)."""

    def __init__(self, Cw: torch.Tensor, start: int, end: int, stride: int = 1):
        self.K, self.perf = Cw.shape[0], Dims(start, end, stride)
        need = int(_lib.hdc_adc_workspace_bytes(self.perf, self.K))
        self.ws = torch.empty(max(need, 16), dtype=torch.uint8, device=Cw.device)
        _check(_lib.hdc_adc_prepare(_stream(), _ptr(Cw), self.K, Cw.shape[1], self.perf, _ptr(self.ws),
                                    self.ws.numel()), "hdc_adc_prepare")

    def __call__(self, Q: torch.Tensor, adc, with_max=False, with_scores=False, out: torch.Tensor | None = None):
        n = Q.shape[0]
        if Q.shape[1] % 2:                      # the search wants an even row pitch
            Q = torch.nn.functional.pad(Q, (0, 1))
        lab = out if out is not None else torch.empty(n, dtype=torch.int32, device=Q.device)
        mx = torch.empty(n, dtype=torch.int32, device=Q.device) if with_max else None
        sc = torch.empty((n, self.K), dtype=torch.int32, device=Q.device) if with_scores else None
        _check(_lib.hdc_adc_argmax_prepared(_stream(), _ptr(Q), n, Q.shape[1], self.K, self.perf, Adc(*adc),
                                            _ptr(lab), _ptr(mx), _ptr(sc), _ptr(self.ws), self.ws.numel()),
               "hdc_adc_argmax_prepared")
        return lab, mx, sc


def cosine_workspace_bytes(start: int, end: int, stride: int, K: int) -> int:
    return int(_lib.hdc_cosine_workspace_bytes(Dims(start, end, stride), K))


class CosinePrepared:
    """Integer class accumulators of one (classes, perforation) turned into
    the matrix-core operand, sums and norms once; each call ranks a batch of
    query hypervectors by cosine similarity (hdc_cosine_argmax_prepared).
    Labels are -1 if an accumulator entry over the set lies outside
    [-32639, 32639]."""

    def __init__(self, acc: torch.Tensor, start: int, end: int, stride: int = 1):
        self.K, self.perf = acc.shape[0], Dims(start, end, stride)
        need = cosine_workspace_bytes(start, end, stride, self.K)
        self.ws = torch.empty(max(need, 16), dtype=torch.uint8, device=acc.device)
        _check(_lib.hdc_cosine_prepare(_stream(), _ptr(acc), self.K, acc.shape[1], self.perf, _ptr(self.ws),
                                       self.ws.numel()), "hdc_cosine_prepare")

    def __call__(self, Q: torch.Tensor, with_max=False, with_scores=False, out: torch.Tensor | None = None):
        n = Q.shape[0]
        if Q.shape[1] % 2:                      # the search wants an even row pitch
            Q = torch.nn.functional.pad(Q, (0, 1))
        lab = out if out is not None else torch.empty(n, dtype=torch.int32, device=Q.device)
        mx = torch.empty(n, dtype=torch.float64, device=Q.device) if with_max else None
        sc = torch.empty((n, self.K), dtype=torch.float64, device=Q.device) if with_scores else None
        _check(_lib.hdc_cosine_argmax_prepared(_stream(), _ptr(Q), n, Q.shape[1], self.K, self.perf, _ptr(lab),
                                               _ptr(mx), _ptr(sc), _ptr(self.ws), self.ws.numel()),
               "hdc_cosine_argmax_prepared")
        return lab, mx, sc


def classify_workspace_bytes(n_dims: int, K: int) -> int:
    return int(_lib.hdc_classify_workspace_bytes(n_dims, K))


def classify_scratch(n: int, nd: int, K: int, device, have: torch.Tensor | None = None):
    """Scratch for the dimension-split classify of n queries (None when the
    batch fills the device by itself); `have` is reused when large enough."""
    need = int(_lib.hdc_classify_scratch_bytes(n, nd, K))
    if need == 0:
        return None
    if have is not None and have.numel() >= need:
        return have
    return torch.empty(need, dtype=torch.uint8, device=device)


def classify(X: torch.Tensor, F: int, P: torch.Tensor, D: int, Cw: torch.Tensor, compute="int8", start=0,
             d_trunc=None, stride=1, with_dists=False, ws: torch.Tensor | None = None,
             labels: torch.Tensor | None = None, split: bool = True, tile: int = 0):
    """hdc_classify: fused encode + Hamming + argmin under one configuration
    (split=False: no dimension splits for small batches; tile: the kernel
    shape, 0 = built-in)."""
    d_trunc = D if d_trunc is None else d_trunc
    n, K = X.shape[0], Cw.shape[0]
    nd = dims_count(start, d_trunc, stride)
    need = classify_workspace_bytes(nd, K)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=X.device)
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    dists = torch.empty((n, K), dtype=torch.int32, device=X.device) if with_dists else None
    sc = classify_scratch(n, nd, K, X.device) if split else None
    _check(_lib.hdc_classify(_stream(), _ptr(X), _xtype(X), n, F, X.shape[1], _ptr(P), D, P.shape[1],
                             DTYPE[compute], Dims(start, d_trunc, stride), _ptr(Cw), K, Cw.shape[1],
                             _ptr(labels), _ptr(dists), _ptr(ws), ws.numel(), _ptr(sc),
                             sc.numel() if sc is not None else 0, int(tile)), "hdc_classify")
    return (labels, dists) if with_dists else labels


class Prepared:
    """Class operand of one (model, configuration) kept on the device, so that
    repeated classification launches only the fused kernel.  Holds the
    dimension-split scratch of the largest small batch seen (calls through
    one Prepared object are ordered on the stream they are issued on)."""

    def __init__(self, Cw: torch.Tensor, D: int, compute="int8", start=0, d_trunc=None, stride=1, tile: int = 0):
        self.D, self.K = D, Cw.shape[0]
        self.tile = tile          # kernel shape of every call (0: built-in)
        self.compute, self.start = compute, start
        self.d_trunc = D if d_trunc is None else d_trunc
        self.stride = stride
        self.nd = dims_count(start, self.d_trunc, stride)
        need = classify_workspace_bytes(self.nd, self.K)
        self.ws = torch.empty(max(need, 16), dtype=torch.uint8, device=Cw.device)
        self.scratch = None
        _check(_lib.hdc_classify_prepare(_stream(), _ptr(Cw), self.K, Cw.shape[1],
                                         Dims(start, self.d_trunc, stride), _ptr(self.ws), self.ws.numel()),
               "hdc_classify_prepare")

    def __call__(self, X: torch.Tensor, F: int, P: torch.Tensor, labels: torch.Tensor | None = None,
                 with_dists=False, split: bool = True):
        n = X.shape[0]
        if labels is None:
            labels = torch.empty(n, dtype=torch.int32, device=X.device)
        dists = torch.empty((n, self.K), dtype=torch.int32, device=X.device) if with_dists else None
        sc = None
        if split:
            sc = classify_scratch(n, self.nd, self.K, X.device, self.scratch)
            if sc is not None:
                self.scratch = sc
        _check(_lib.hdc_classify_prepared(_stream(), _ptr(X), _xtype(X), n, F, X.shape[1], _ptr(P), self.D,
                                          P.shape[1], DTYPE[self.compute],
                                          Dims(self.start, self.d_trunc, self.stride), self.K, _ptr(labels),
                                          _ptr(dists), _ptr(self.ws), self.ws.numel(), _ptr(sc),
                                          sc.numel() if sc is not None else 0, int(self.tile)),
               "hdc_classify_prepared")
        return (labels, dists) if with_dists else labels


def adc_argmax(Q: torch.Tensor, Cw: torch.Tensor, start: int, end: int, stride: int, adc, with_max=False,
               with_scores=False):
    """hdc_adc_argmax: adc = (res_bits, step, floor, ceil)."""
    n, K = Q.shape[0], Cw.shape[0]
    lab = torch.empty(n, dtype=torch.int32, device=Q.device)
    mx = torch.empty(n, dtype=torch.int32, device=Q.device) if with_max else None
    sc = torch.empty((n, K), dtype=torch.int32, device=Q.device) if with_scores else None
    _check(_lib.hdc_adc_argmax(_stream(), _ptr(Q), n, Q.shape[1], _ptr(Cw), K, Cw.shape[1], Dims(start, end, stride),
                               Adc(*adc), _ptr(lab), _ptr(mx), _ptr(sc)), "hdc_adc_argmax")
    return lab, mx, sc


def retrain_workspace(n: int, nbits: int, K: int, device) -> torch.Tensor:
    """A workspace for hdc_class_acc / hdc_retrain_epoch on n rows."""
    need = int(_lib.hdc_retrain_workspace_bytes(n, nbits, K))
    return torch.empty(max(need, 16), dtype=torch.uint8, device=device)


def class_acc(H: torch.Tensor, nbits: int, labels: torch.Tensor, K: int, ws: torch.Tensor | None = None):
    """hdc_class_acc: (acc[K][nbits] int32, C[K][words] int64) from training rows."""
    acc = torch.empty((K, nbits), dtype=torch.int32, device=H.device)
    Cw = torch.empty((K, words(nbits)), dtype=torch.int64, device=H.device)
    if ws is None or ws.numel() < int(_lib.hdc_retrain_workspace_bytes(H.shape[0], nbits, K)):
        ws = retrain_workspace(H.shape[0], nbits, K, H.device)
    _check(_lib.hdc_class_acc(_stream(), _ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), K, _ptr(acc),
                              _ptr(Cw), Cw.shape[1], _ptr(ws), ws.numel()), "hdc_class_acc")
    return acc, Cw


def retrain_epoch(H: torch.Tensor, nbits: int, labels: torch.Tensor, pred: torch.Tensor, acc: torch.Tensor,
                  Cw: torch.Tensor, n_wrong: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """hdc_retrain_epoch: updates acc and Cw in place; n_wrong (device int32[1]) if given."""
    K = acc.shape[0]
    if ws is None or ws.numel() < int(_lib.hdc_retrain_workspace_bytes(H.shape[0], nbits, K)):
        ws = retrain_workspace(H.shape[0], nbits, K, H.device)
    _check(_lib.hdc_retrain_epoch(_stream(), _ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), _ptr(pred),
                                  K, _ptr(acc), _ptr(Cw), Cw.shape[1], _ptr(n_wrong), _ptr(ws), ws.numel()),
           "hdc_retrain_epoch")


def convert_features(X: torch.Tensor, F: int, compute: str) -> torch.Tensor:
    out = torch.empty((X.shape[0], F), dtype=torch.float32, device=X.device)
    _check(_lib.hdc_convert_features(_stream(), _ptr(X), _xtype(X), X.shape[0], F, X.shape[1],
                                     DTYPE[compute], _ptr(out)), "hdc_convert_features")
    return out


def config_array(cfgs, tile: int = 0) -> np.ndarray:
    """Host hdc_config array ([n][5] int32: d_trunc, stride, start, dtype,
    tile_id) from (d_trunc, stride, start, dtype[, tile_id]) tuples (dtype a
    name or an hdc_dtype value; tile_id defaults to `tile`).  An array
    already in that form is returned as it is, so a caller that evaluates
    the same configurations repeatedly builds it once."""
    if isinstance(cfgs, np.ndarray):
        assert cfgs.dtype == np.int32 and cfgs.ndim == 2 and cfgs.shape[1] == 5 and cfgs.flags.c_contiguous
        return cfgs
    rows = [(c[0], c[1], c[2], DTYPE[c[3]] if isinstance(c[3], str) else c[3], c[4] if len(c) > 4 else tile)
            for c in cfgs]
    return np.array(rows, dtype=np.int32).reshape(-1, 5)


def result_view(out: torch.Tensor, ncfg: int) -> np.ndarray:
    """The hdc_config_result records held in a host uint8 tensor."""
    return out.numpy()[:ncfg * RESULT_DTYPE.itemsize].view(RESULT_DTYPE)


def eval_configs(X: torch.Tensor, F: int, truth: torch.Tensor, P: torch.Tensor, D: int, Cw: torch.Tensor,
                 cfgs, ws: torch.Tensor | None = None, max_workgroups: int = 0, tile: int = 0,
                 out: torch.Tensor | None = None):
    """hdc_eval_configs: cfgs = [(d_trunc, stride, start, dtype[, tile_id])]
    or a config_array of them.  Without `out` the call waits for the stream and
    returns the result records (numpy: correct, n, device_us); with `out`, a
    page-locked host uint8 tensor of at least 16 * len(cfgs) bytes, nothing
    waits and the records are read later with result_view(out, ncfg) once
    the stream has passed the call."""
    arr = config_array(cfgs, tile)
    K = Cw.shape[0]
    need = int(_lib.hdc_eval_configs_workspace_bytes(len(arr), F, D, K))
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device=X.device)
    wait = out is None
    if wait:
        out = torch.empty(len(arr) * RESULT_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True)
    assert out.numel() >= len(arr) * RESULT_DTYPE.itemsize and out.device.type == "cpu"
    _check(_lib.hdc_eval_configs(_stream(), _ptr(X), _xtype(X), X.shape[0], F, X.shape[1], _ptr(truth),
                                 _ptr(P), D, P.shape[1], _ptr(Cw), K, Cw.shape[1], arr.ctypes.data, len(arr),
                                 _ptr(out), _ptr(ws), ws.numel(), int(max_workgroups)), "hdc_eval_configs")
    if wait:
        torch.cuda.current_stream().synchronize()
        return result_view(out, len(arr)).copy()
    return out


def device_clock_hz() -> float:
    return float(_lib.hdc_device_clock_hz())


def to_u64(t: torch.Tensor) -> np.ndarray:
    """Device int64 word tensor -> host uint64 numpy array."""
    return t.cpu().numpy().view(np.uint64)
