"""ctypes binding of the plain CPU oracle (``oracle/hdc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  This is the correctness reference for the GPU
path.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product package never does, and the
oracle imports nothing from the product package.

Every function takes and returns numpy arrays; see ``hdc_oracle.h`` for the
definitions, the paper passages they follow and the conventions used where
the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hdc_oracle.c")
LIB = os.path.join(HERE, "libhdc_oracle.so")

INT8, UINT8, BF16, FP8_E4M3, FP32, FP8_SPLIT = 0, 1, 2, 3, 4, 5
DTYPE = {"int8": INT8, "uint8": UINT8, "bf16": BF16, "fp8": FP8_E4M3, "fp32": FP32, "fp8split": FP8_SPLIT}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over queries, portable x86-64-v3)."""
    cmd = ["gcc", "-std=c11", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        p, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.or_round_bf16.argtypes = [dbl]; L.or_round_bf16.restype = dbl
        L.or_round_e4m3.argtypes = [dbl]; L.or_round_e4m3.restype = dbl
        L.or_dims_count.argtypes = [i32, i32, i32]; L.or_dims_count.restype = i32
        L.or_threads.argtypes = [C.c_int]; L.or_threads.restype = C.c_int
        L.or_class_acc.argtypes = [p, i64, i32, i64, p, i32, p]
        L.or_retrain_epoch.argtypes = [p, i64, i32, i64, p, p, i32, p]; L.or_retrain_epoch.restype = i64
        L.or_binarize.argtypes = [p, i32, i32, p, i64]
        L.or_adc_quantize.argtypes = [i32, i32, i32, i32, i32]; L.or_adc_quantize.restype = i32
        L.or_adc_scores.argtypes = [p, i64, i64, p, i32, i64, i32, i32, i32, i32, i32, i32, i32, p, C.c_int]
        L.or_argmax.argtypes = [p, i64, i32, p, p]
        L.or_cosine_scores.argtypes = [p, i64, i64, p, i32, i64, i32, i32, i32, p, C.c_int]
        L.or_argmax_f64.argtypes = [p, i64, i32, p, p]
        L.or_encode_fperf.argtypes = [p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, i32, i32, i32, i32, i32,
                                      i32, p, i64, C.c_int]
        L.or_level_quantize.argtypes = [p, i64, i32, i64, p, p, i32, p, i64]
        L.or_level_id_encode.argtypes = [p, i64, i32, i64, p, i64, p, i32, i64, i32, p, i64, C.c_int]
        L.or_encode.argtypes = [p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, i32, i32, i32, p, i64, C.c_int]
        L.or_project.argtypes = [p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, i32, i32, i32, p, p, C.c_int]
        L.or_bundle.argtypes = [p, i64, i32, i64, p, i32, p, i64, p]
        L.or_bundle_bipolar.argtypes = [p, i64, i32, i64, p, i32, p, i64]
        L.or_hamming.argtypes = [p, i64, i64, p, i32, i64, i32, i32, i32, p, C.c_int]
        L.or_hamming_popcount.argtypes = [p, i64, i64, p, i32, i64, i32, i32, i32, p, C.c_int]
        L.or_argmin.argtypes = [p, i64, i32, p, p]
        L.or_classify.argtypes = [p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, i32, i32, i32,
                                  p, i32, i64, p, p, C.c_int]
        L.or_eval_configs.argtypes = [p, C.c_int, i64, i32, i64, p, p, i32, i64, p, i32, i64,
                                      p, i32, p, C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _xtype(X: np.ndarray) -> int:
    return {np.dtype(np.int8): INT8, np.dtype(np.uint8): UINT8, np.dtype(np.float32): FP32}[X.dtype]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def threads(t: int = 0) -> int:
    return lib().or_threads(t)


def round_bf16(v: float) -> float:
    return lib().or_round_bf16(float(v))


def round_e4m3(v: float) -> float:
    return lib().or_round_e4m3(float(v))


def dims_count(start: int, end: int, stride: int) -> int:
    return lib().or_dims_count(start, end, stride)


def words(nbits: int) -> int:
    return max(1, (nbits + 63) // 64)


def encode(X, P, compute="int8", start=0, end=None, stride=1, threads=0) -> np.ndarray:
    """Packed sign bits of X @ P[S].T, shape [n][ceil(|S|/64)] uint64."""
    X = np.ascontiguousarray(X)
    P = _c(P, np.int8)
    end = P.shape[0] if end is None else end
    ns = dims_count(start, end, stride)
    H = np.zeros((X.shape[0], words(ns)), dtype=np.uint64)
    lib().or_encode(_ptr(X), _xtype(X), X.shape[0], X.shape[1], X.shape[1], _ptr(P), P.shape[0],
                    P.shape[1], DTYPE.get(compute, compute), start, end, stride, _ptr(H), H.shape[1],
                    threads)
    return H


def project(X, P, compute="int8", start=0, end=None, stride=1, threads=0):
    """Exact projections y[n][|S|] (double) and sum_f |x'_f| per row."""
    X = np.ascontiguousarray(X)
    P = _c(P, np.int8)
    end = P.shape[0] if end is None else end
    ns = dims_count(start, end, stride)
    Y = np.zeros((X.shape[0], ns), dtype=np.float64)
    ab = np.zeros(X.shape[0], dtype=np.float64)
    lib().or_project(_ptr(X), _xtype(X), X.shape[0], X.shape[1], X.shape[1], _ptr(P), P.shape[0],
                     P.shape[1], DTYPE.get(compute, compute), start, end, stride, _ptr(Y), _ptr(ab),
                     threads)
    return Y, ab


def bundle(H, labels, K, nbits):
    H = _c(H, np.uint64)
    labels = _c(labels, np.int32)
    Cw = np.zeros((K, words(nbits)), dtype=np.uint64)
    counts = np.zeros(K, dtype=np.int32)
    lib().or_bundle(_ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), K, _ptr(Cw), Cw.shape[1],
                    _ptr(counts))
    return Cw, counts


def bundle_bipolar(H, labels, K, nbits):
    H = _c(H, np.uint64)
    labels = _c(labels, np.int32)
    Cw = np.zeros((K, words(nbits)), dtype=np.uint64)
    lib().or_bundle_bipolar(_ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), K, _ptr(Cw),
                            Cw.shape[1])
    return Cw


def hamming(Q, Cw, start, end, stride=1, threads=0):
    Q = _c(Q, np.uint64)
    Cw = _c(Cw, np.uint64)
    dist = np.zeros((Q.shape[0], Cw.shape[0]), dtype=np.int32)
    lib().or_hamming(_ptr(Q), Q.shape[0], Q.shape[1], _ptr(Cw), Cw.shape[0], Cw.shape[1], start,
                     end, stride, _ptr(dist), threads)
    return dist


def hamming_popcount(Q, Cw, start, end, stride=1, threads=0):
    Q = _c(Q, np.uint64)
    Cw = _c(Cw, np.uint64)
    dist = np.zeros((Q.shape[0], Cw.shape[0]), dtype=np.int32)
    lib().or_hamming_popcount(_ptr(Q), Q.shape[0], Q.shape[1], _ptr(Cw), Cw.shape[0], Cw.shape[1],
                              start, end, stride, _ptr(dist), threads)
    return dist


def argmin(dist):
    dist = _c(dist, np.int32)
    lab = np.zeros(dist.shape[0], dtype=np.int32)
    mn = np.zeros(dist.shape[0], dtype=np.int32)
    lib().or_argmin(_ptr(dist), dist.shape[0], dist.shape[1], _ptr(lab), _ptr(mn))
    return lab, mn


def classify(X, P, Cw, compute="int8", start=0, d_trunc=None, stride=1, with_dists=False,
             threads=0):
    X = np.ascontiguousarray(X)
    P = _c(P, np.int8)
    Cw = _c(Cw, np.uint64)
    d_trunc = P.shape[0] if d_trunc is None else d_trunc
    K = Cw.shape[0]
    lab = np.zeros(X.shape[0], dtype=np.int32)
    dists = np.zeros((X.shape[0], K), dtype=np.int32) if with_dists else None
    lib().or_classify(_ptr(X), _xtype(X), X.shape[0], X.shape[1], X.shape[1], _ptr(P), P.shape[0],
                      P.shape[1], DTYPE.get(compute, compute), start, d_trunc, stride, _ptr(Cw), K,
                      Cw.shape[1], _ptr(lab), _ptr(dists), threads)
    return (lab, dists) if with_dists else lab


def eval_configs(X, truth, P, Cw, cfgs, threads=0):
    """cfgs: iterable of (d_trunc, stride, start, compute)."""
    X = np.ascontiguousarray(X)
    P = _c(P, np.int8)
    Cw = _c(Cw, np.uint64)
    truth = _c(truth, np.int32)
    arr = np.array([[d, k, s, DTYPE.get(t, t)] for (d, k, s, t) in cfgs], dtype=np.int32).reshape(-1, 4)
    correct = np.zeros(arr.shape[0], dtype=np.int32)
    lib().or_eval_configs(_ptr(X), _xtype(X), X.shape[0], X.shape[1], X.shape[1], _ptr(truth),
                          _ptr(P), P.shape[0], P.shape[1], _ptr(Cw), Cw.shape[0], Cw.shape[1],
                          _ptr(arr), arr.shape[0], _ptr(correct), threads)
    return correct


def train(X, y, P, K, compute="int8", threads=0):
    """Class hypervectors of a training set: encode (exact) then bundle."""
    H = encode(X, P, compute, threads=threads)
    return bundle(H, y, K, P.shape[0])


def class_acc(H, labels, K, nbits):
    """Integer class accumulators acc[K][nbits] (bipolar sums per class)."""
    H = _c(H, np.uint64)
    labels = _c(labels, np.int32)
    acc = np.zeros((K, nbits), dtype=np.int32)
    lib().or_class_acc(_ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), K, _ptr(acc))
    return acc


def retrain_epoch(H, labels, pred, acc, nbits):
    """One retraining epoch in place on acc; returns the number of mispredicted rows."""
    H = _c(H, np.uint64)
    labels = _c(labels, np.int32)
    pred = _c(pred, np.int32)
    assert acc.dtype == np.int32 and acc.flags.c_contiguous
    return int(lib().or_retrain_epoch(_ptr(H), H.shape[0], nbits, H.shape[1], _ptr(labels), _ptr(pred),
                                      acc.shape[0], _ptr(acc)))


def binarize(acc, nbits):
    acc = _c(acc, np.int32)
    Cw = np.zeros((acc.shape[0], words(nbits)), dtype=np.uint64)
    lib().or_binarize(_ptr(acc), acc.shape[0], nbits, _ptr(Cw), Cw.shape[1])
    return Cw


def retrain(H, labels, K, nbits, epochs):
    """Bundle, then `epochs` retraining epochs, each predicting every row with
    the model at the start of the epoch (exact Hamming over all nbits).
    Returns (C, acc, wrong-per-epoch)."""
    acc = class_acc(H, labels, K, nbits)
    hist = []
    for _ in range(epochs):
        Cw = binarize(acc, nbits)
        pred, _ = argmin(hamming_popcount(H, Cw, 0, nbits, 1))
        hist.append(retrain_epoch(H, labels, pred, acc, nbits))
    return binarize(acc, nbits), acc, hist


def adc_quantize(s, res, step, floor_, ceil_):
    return int(lib().or_adc_quantize(int(s), res, step, floor_, ceil_))


def adc_scores(Q, Cw, start, end, stride, res, step, floor_, ceil_, threads=0):
    """ADC-chunked dot-product scores [n][K] (128-dimension chunks)."""
    Q = _c(Q, np.uint64)
    Cw = _c(Cw, np.uint64)
    sc = np.zeros((Q.shape[0], Cw.shape[0]), dtype=np.int32)
    lib().or_adc_scores(_ptr(Q), Q.shape[0], Q.shape[1], _ptr(Cw), Cw.shape[0], Cw.shape[1], start, end, stride,
                        res, step, floor_, ceil_, _ptr(sc), threads)
    return sc


def argmax(scores):
    scores = _c(scores, np.int32)
    lab = np.zeros(scores.shape[0], dtype=np.int32)
    mx = np.zeros(scores.shape[0], dtype=np.int32)
    lib().or_argmax(_ptr(scores), scores.shape[0], scores.shape[1], _ptr(lab), _ptr(mx))
    return lab, mx


def cosine_scores(Q, acc, start, end, stride=1, threads=0):
    """Cosine scores [n][K] (float64) of bipolar queries against integer class accumulators."""
    Q = _c(Q, np.uint64)
    acc = _c(acc, np.int32)
    sc = np.zeros((Q.shape[0], acc.shape[0]), dtype=np.float64)
    lib().or_cosine_scores(_ptr(Q), Q.shape[0], Q.shape[1], _ptr(acc), acc.shape[0], acc.shape[1], start, end,
                           stride, _ptr(sc), threads)
    return sc


def argmax_f64(scores):
    scores = _c(scores, np.float64)
    lab = np.zeros(scores.shape[0], dtype=np.int32)
    mx = np.zeros(scores.shape[0], dtype=np.float64)
    lib().or_argmax_f64(_ptr(scores), scores.shape[0], scores.shape[1], _ptr(lab), _ptr(mx))
    return lab, mx


def encode_fperf(X, P, fstart, fend, fstride, compute="int8", start=0, end=None, stride=1, threads=0):
    """Packed sign bits of the rescaled feature-perforated projection."""
    X = np.ascontiguousarray(X)
    P = _c(P, np.int8)
    end = P.shape[0] if end is None else end
    ns = dims_count(start, end, stride)
    H = np.zeros((X.shape[0], words(ns)), dtype=np.uint64)
    lib().or_encode_fperf(_ptr(X), _xtype(X), X.shape[0], X.shape[1], X.shape[1], _ptr(P), P.shape[0],
                          P.shape[1], DTYPE.get(compute, compute), fstart, fend, fstride, start, end, stride,
                          _ptr(H), H.shape[1], threads)
    return H


def level_quantize(X, lo, hi, L):
    """Levels [n][F] uint16 of float32 features under per-feature ranges."""
    X = _c(X, np.float32)
    lo = _c(lo, np.float32)
    hi = _c(hi, np.float32)
    lev = np.zeros(X.shape, dtype=np.uint16)
    lib().or_level_quantize(_ptr(X), X.shape[0], X.shape[1], X.shape[1], _ptr(lo), _ptr(hi), L, _ptr(lev),
                            lev.shape[1])
    return lev


def level_id_encode(lev, ID, LV, D, threads=0):
    """Packed Level-ID hypervectors [n][ceil(D/64)] of level rows lev [n][F]."""
    lev = _c(lev, np.uint16)
    ID = _c(ID, np.uint64)
    LV = _c(LV, np.uint64)
    H = np.zeros((lev.shape[0], words(D)), dtype=np.uint64)
    lib().or_level_id_encode(_ptr(lev), lev.shape[0], lev.shape[1], lev.shape[1], _ptr(ID), ID.shape[1],
                             _ptr(LV), LV.shape[0], LV.shape[1], D, _ptr(H), H.shape[1], threads)
    return H
