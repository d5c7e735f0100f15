"""The C ABI library loads and exports every entry point include/hdc.h
declares; argument validation (which runs before any device work) rejects
bad calls.  No compute call is made here, so no GPU is needed."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdc.h")
LIB = os.path.join(ROOT, "paper_2606_26547_amd", "libhdc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2606_26547_amd.build import build
        build()
    return C.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared()
    for n in ["hdc_encode", "hdc_bundle", "hdc_hamming_argmin", "hdc_eval_configs", "hdc_classify"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


class Dims(C.Structure):
    _fields_ = [("start", C.c_int32), ("end", C.c_int32), ("stride", C.c_int32)]


def test_validation_without_device(lib):
    lib.hdc_status_string.restype = C.c_char_p
    assert lib.hdc_status_string(0) == b"HDC_OK"
    lib.hdc_dims_count.argtypes = [Dims]
    assert lib.hdc_dims_count(Dims(0, 10240, 1)) == 10240
    assert lib.hdc_dims_count(Dims(3, 100, 7)) == 14
    assert lib.hdc_dims_count(Dims(5, 5, 1)) == 0
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.hdc_encode.argtypes = [p, p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, Dims, p, i64]
    fake = C.c_void_p(1 << 20)       # never dereferenced: validation fails first
    # negative n, F <= 0, end > D, stride < 1, unsupported pair, unaligned ld
    assert lib.hdc_encode(None, fake, 0, -1, 8, 64, fake, 64, 64, 0, Dims(0, 64, 1), fake, 1) == 1
    assert lib.hdc_encode(None, fake, 0, 1, 0, 64, fake, 64, 64, 0, Dims(0, 64, 1), fake, 1) == 1
    assert lib.hdc_encode(None, fake, 0, 1, 8, 64, fake, 64, 64, 0, Dims(0, 65, 1), fake, 1) == 1
    assert lib.hdc_encode(None, fake, 0, 1, 8, 64, fake, 64, 64, 0, Dims(0, 64, 0), fake, 1) == 1
    assert lib.hdc_encode(None, fake, 4, 1, 8, 64, fake, 64, 64, 0, Dims(0, 64, 1), fake, 1) == 2
    assert lib.hdc_encode(None, fake, 0, 1, 8, 40, fake, 64, 64, 0, Dims(0, 64, 1), fake, 1) == 1
    assert lib.hdc_encode(None, fake, 0, 1, 2000, 2048, fake, 64, 2048, 0, Dims(0, 64, 1), fake, 1) == 2
    # n == 0 is a no-op
    assert lib.hdc_encode(None, None, 0, 0, 8, 64, fake, 64, 64, 0, Dims(0, 64, 1), None, 1) == 0
    # the split E4M3 compute type (5) takes integer features only
    assert lib.hdc_encode(None, None, 0, 0, 8, 64, fake, 64, 64, 5, Dims(0, 64, 1), None, 1) == 0
    assert lib.hdc_encode(None, None, 1, 0, 8, 64, fake, 64, 64, 5, Dims(0, 64, 1), None, 1) == 0
    assert lib.hdc_encode(None, fake, 4, 1, 8, 64, fake, 64, 64, 5, Dims(0, 64, 1), fake, 1) == 2
    assert lib.hdc_encode(None, fake, 5, 1, 8, 64, fake, 64, 64, 5, Dims(0, 64, 1), fake, 1) == 1
    # a projection of 2^32 bytes or more is refused (32-bit row offsets):
    # encode, classify and the configuration sweep share the check
    big_d = (1 << 32) // 1024
    assert lib.hdc_encode(None, fake, 0, 1, 1000, 1024, fake, big_d, 1024, 0, Dims(0, 64, 1), fake, 1) == 2
    assert lib.hdc_encode(None, fake, 0, 1, 1000, 1024, fake, big_d - 2, 1024, 0, Dims(0, 64, 1), None, 1) == 1
    lib.hdc_classify.argtypes = [p, p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, Dims, p, i32, i64, p, p, p,
                                 C.c_size_t, p, C.c_size_t]
    assert lib.hdc_classify(None, fake, 0, 1, 1000, 1024, fake, big_d, 1024, 0, Dims(0, 64, 1), fake, 3, 1, fake,
                            None, fake, 1 << 20, None, 0) == 2
    # a misaligned dimension-split scratch is refused
    lib.hdc_classify_prepared.argtypes = [p, p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, Dims, i32, p, p, p,
                                          C.c_size_t, p, C.c_size_t]
    assert lib.hdc_classify_prepared(None, fake, 0, 1, 64, 64, fake, 64, 64, 0, Dims(0, 64, 1), 3, fake, None,
                                     fake, 1 << 20, C.c_void_p((1 << 20) + 2), 1 << 20) == 3
    # scratch sizes: a batch that fills the device by its query blocks alone
    # needs none; 1559 queries of 10240 dimensions split the dimensions into
    # 40 parts of four words (the most the words allow), each holding K
    # partial sums per query
    lib.hdc_classify_scratch_bytes.restype = C.c_size_t
    lib.hdc_classify_scratch_bytes.argtypes = [i64, i32, i32]
    assert lib.hdc_classify_scratch_bytes(1 << 18, 10240, 26) == 0
    assert lib.hdc_classify_scratch_bytes(1559, 10240, 26) == 4 * 40 * 26 * 1559
    assert lib.hdc_classify_scratch_bytes(1559, 448, 26) == 0          # too few words to split
    lib.hdc_eval_configs.argtypes = [p, p, C.c_int, i64, i32, i64, p, p, i32, i64, p, i32, i64, p, i32, p, p,
                                     C.c_size_t, i32]
    assert lib.hdc_eval_configs(None, fake, 0, 1, 1000, 1024, fake, fake, big_d, 1024, fake, 3, big_d // 64, fake,
                                1, fake, fake, 1 << 30, 0) == 2
    # hdc_hamming_argmin: nbits bounds the perforation set and the pitches
    lib.hdc_hamming_argmin.argtypes = [p, p, i64, i64, p, i32, i64, i32, Dims, p, p, p]
    assert lib.hdc_hamming_argmin(None, fake, 4, 2, fake, 3, 2, 0, Dims(0, 64, 1), fake, None, None) == 1
    assert lib.hdc_hamming_argmin(None, fake, 4, 2, fake, 3, 2, 100, Dims(0, 101, 1), fake, None, None) == 1
    assert lib.hdc_hamming_argmin(None, fake, 4, 1, fake, 3, 2, 100, Dims(0, 64, 1), fake, None, None) == 1
    assert lib.hdc_hamming_argmin(None, fake, 4, 2, fake, 3, 1, 100, Dims(0, 64, 1), fake, None, None) == 1
    assert lib.hdc_hamming_argmin(None, None, 0, 2, fake, 3, 2, 100, Dims(0, 64, 1), None, None, None) == 0
    lib.hdc_classify_workspace_bytes.restype = C.c_size_t
    assert lib.hdc_classify_workspace_bytes(10240, 26) == 324 * 1024 + 512   # 320 tiles, padded to 6
    assert lib.hdc_classify_workspace_bytes(10240, 200) == 0
    lib.hdc_hamming_workspace_bytes.restype = C.c_size_t
    lib.hdc_hamming_workspace_bytes.argtypes = [Dims, i32]
    assert lib.hdc_hamming_workspace_bytes(Dims(0, 10240, 1), 26) == 160 * 1024 + 512
    # words from the even word at or below start, whole windows of 4 words
    assert lib.hdc_hamming_workspace_bytes(Dims(64, 4096, 2), 100) == 64 * 4 * 1024 + 512
    assert lib.hdc_hamming_workspace_bytes(Dims(200, 1000, 1), 5) == 16 * 1024 + 512
    assert lib.hdc_hamming_workspace_bytes(Dims(0, 10240, 1), 129) == 0
    assert lib.hdc_hamming_workspace_bytes(Dims(0, 70000, 1), 26) == 0
    lib.hdc_bundle_workspace_bytes.restype = C.c_size_t
    lib.hdc_bundle_workspace_bytes.argtypes = [C.c_int64, i32, i32]
    # class sums [K][nbits], per-block group sizes (one block up to 8192
    # rows, then one per 4096), group cursors, group and segment offsets, the
    # row list: each part padded to 256 bytes
    pad = lambda b: (b + 255) // 256 * 256
    assert lib.hdc_bundle_workspace_bytes(6238, 10240, 26) == \
        pad(4 * 26 * 10240) + pad(4 * 26) + pad(4 * 26) + 2 * pad(4 * 27) + pad(4 * 6238)
    assert lib.hdc_bundle_workspace_bytes(20000, 10240, 26) == \
        pad(4 * 26 * 10240) + pad(4 * 5 * 26) + pad(4 * 26) + 2 * pad(4 * 27) + pad(4 * 20000)
    assert lib.hdc_bundle_workspace_bytes(6238, 10240, 129) == 0
    assert lib.hdc_bundle_workspace_bytes(1 << 30, 10240, 26) == 0
    lib.hdc_retrain_workspace_bytes.restype = C.c_size_t
    lib.hdc_retrain_workspace_bytes.argtypes = [C.c_int64, i32, i32]
    # (class, sign) groups and up to two list entries per row; no class sums
    assert lib.hdc_retrain_workspace_bytes(6238, 10240, 26) == 2 * pad(4 * 52) + 2 * pad(4 * 53) + pad(4 * 2 * 6238)


def test_bundle_validation_without_device(lib):
    p, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.hdc_bundle.argtypes = [p, p, i64, i32, i64, p, i32, p, i64, p, p, sz]
    fake, ws, big = C.c_void_p(1 << 20), C.c_void_p(1 << 24), 1 << 30
    assert lib.hdc_bundle(None, fake, 4, 0, 1, fake, 3, fake, 1, None, ws, big) == 1          # nbits <= 0
    assert lib.hdc_bundle(None, fake, 4, 64, 1, fake, 200, fake, 1, None, ws, big) == 2       # K > 128
    assert lib.hdc_bundle(None, fake, 4, 130, 2, fake, 3, fake, 3, None, ws, big) == 1        # ldh < words
    assert lib.hdc_bundle(None, fake, 4, 130, 3, fake, 3, fake, 2, None, ws, big) == 1        # ldc < words
    assert lib.hdc_bundle(None, None, 4, 64, 1, fake, 3, fake, 1, None, ws, big) == 1         # no H
    assert lib.hdc_bundle(None, fake, 4, 64, 1, fake, 3, fake, 1, None, ws, 16) == 3          # workspace
    assert lib.hdc_bundle(None, fake, 4, 64, 1, fake, 3, fake, 1, None, C.c_void_p((1 << 24) + 8), big) == 3
    assert lib.hdc_bundle(None, fake, 1 << 30, 64, 1, fake, 3, fake, 1, None, ws, big) == 2   # n >= 2^30
    # the no-allocation form: the same checks, and a size beyond its fixed
    # scratch is refused before any device work
    lib.hdc_bundle_noalloc.argtypes = [p, p, i64, i32, i64, p, i32, p, i64, p]
    lib.hdc_bundle_noalloc_limit_bytes.restype = sz
    assert lib.hdc_bundle_noalloc_limit_bytes() == 32 << 20
    assert lib.hdc_bundle_noalloc(None, fake, 4, 0, 1, fake, 3, fake, 1, None) == 1           # nbits <= 0
    assert lib.hdc_bundle_noalloc(None, fake, 4, 64, 1, fake, 200, fake, 1, None) == 2        # K > 128
    assert lib.hdc_bundle_noalloc(None, None, 4, 64, 1, fake, 3, fake, 1, None) == 1          # no H
    assert lib.hdc_bundle_noalloc(None, fake, 1 << 24, 64, 1, fake, 3, fake, 1, None) == 2    # beyond 32 MiB
    assert lib.hdc_bundle_noalloc(None, fake, 4, 65536, 1024, fake, 128, fake, 1024, None) == 2  # class sums


def test_retrain_validation_without_device(lib):
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sz = C.c_size_t
    lib.hdc_class_acc.argtypes = [p, p, i64, i32, i64, p, i32, p, p, i64, p, sz]
    lib.hdc_retrain_epoch.argtypes = [p, p, i64, i32, i64, p, p, i32, p, p, i64, p, p, sz]
    fake = C.c_void_p(1 << 20)
    ws, big = C.c_void_p(1 << 24), 1 << 30
    assert lib.hdc_class_acc(None, fake, 4, 0, 1, fake, 3, fake, fake, 1, ws, big) == 1        # nbits <= 0
    assert lib.hdc_class_acc(None, fake, 4, 64, 1, fake, 200, fake, fake, 1, ws, big) == 2     # K > 128
    assert lib.hdc_class_acc(None, fake, 4, 130, 2, fake, 3, fake, fake, 3, ws, big) == 1      # ldh < words
    assert lib.hdc_class_acc(None, fake, 4, 64, 1, fake, 3, None, fake, 1, ws, big) == 1       # no acc
    assert lib.hdc_class_acc(None, fake, 4, 64, 1, fake, 3, fake, fake, 1, ws, 64) == 3        # workspace
    assert lib.hdc_class_acc(None, fake, 4, 64, 1, fake, 3, fake, fake, 1, C.c_void_p((1 << 24) + 4), big) == 3
    assert lib.hdc_class_acc(None, fake, 1 << 30, 64, 1, fake, 3, fake, fake, 1, ws, big) == 2  # n >= 2^30
    assert lib.hdc_retrain_epoch(None, fake, 4, 64, 1, fake, None, 3, fake, fake, 1, None, ws, big) == 1  # pred


class Adc(C.Structure):
    _fields_ = [("res_bits", C.c_int32), ("step", C.c_int32), ("floor", C.c_int32), ("ceil", C.c_int32)]


def test_adc_validation_without_device(lib):
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.hdc_adc_argmax.argtypes = [p, p, i64, i64, p, i32, i64, Dims, Adc, p, p, p]
    fake = C.c_void_p(1 << 20)
    ok = Adc(8, 1, -127, 128)
    assert lib.hdc_adc_argmax(None, fake, 4, 2, fake, 3, 2, Dims(0, 128, 1), Adc(0, 1, -1, 1), fake, None, None) == 1
    assert lib.hdc_adc_argmax(None, fake, 4, 2, fake, 3, 2, Dims(0, 128, 1), Adc(8, 0, -1, 1), fake, None, None) == 1
    assert lib.hdc_adc_argmax(None, fake, 4, 2, fake, 3, 2, Dims(0, 128, 1), Adc(8, 1, 5, 1), fake, None, None) == 1
    assert lib.hdc_adc_argmax(None, fake, 4, 2, fake, 300, 2, Dims(0, 128, 1), ok, fake, None, None) == 2
    assert lib.hdc_adc_argmax(None, fake, 4, 1, fake, 3, 2, Dims(0, 128, 1), ok, fake, None, None) == 1   # ldq
    assert lib.hdc_adc_argmax(None, None, 0, 2, fake, 3, 2, Dims(0, 128, 1), ok, None, None, None) == 0   # n == 0


def test_cosine_validation_without_device(lib):
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.hdc_cosine_workspace_bytes.restype = C.c_size_t
    lib.hdc_cosine_workspace_bytes.argtypes = [Dims, i32]
    lib.hdc_cosine_prepare.argtypes = [p, p, i32, i64, Dims, p, C.c_size_t]
    lib.hdc_cosine_argmax_prepared.argtypes = [p, p, i64, i64, i32, Dims, p, p, p, p, C.c_size_t]
    tail = 128 * 8 * 2 + 128 * 4 + 16           # class sums, reciprocal norms, maxima, range flag
    assert lib.hdc_cosine_workspace_bytes(Dims(0, 10240, 1), 26) == 20 * 8 * 4 * 1024 + tail
    assert lib.hdc_cosine_workspace_bytes(Dims(64, 4096, 2), 100) == 8 * 8 * 4 * 4 * 1024 + tail
    assert lib.hdc_cosine_workspace_bytes(Dims(200, 1000, 1), 5) == 2 * 8 * 4 * 1024 + tail
    assert lib.hdc_cosine_workspace_bytes(Dims(0, 10240, 1), 129) == 0
    assert lib.hdc_cosine_workspace_bytes(Dims(0, 70000, 1), 26) == 0
    fake = C.c_void_p(1 << 20)
    need = lib.hdc_cosine_workspace_bytes(Dims(0, 128, 1), 3)
    assert lib.hdc_cosine_prepare(None, fake, 3, 100, Dims(0, 128, 1), fake, need) == 1        # lda < end
    assert lib.hdc_cosine_prepare(None, None, 3, 128, Dims(0, 128, 1), fake, need) == 1        # no acc
    assert lib.hdc_cosine_prepare(None, fake, 3, 128, Dims(0, 128, 1), fake, need - 1) == 3    # small ws
    assert lib.hdc_cosine_prepare(None, fake, 200, 128, Dims(0, 128, 1), fake, 1 << 30) == 2   # K > 128
    assert lib.hdc_cosine_argmax_prepared(None, fake, 4, 3, 3, Dims(0, 128, 1), fake, None, None, fake,
                                          need) == 1                                            # odd ldq
    assert lib.hdc_cosine_argmax_prepared(None, C.c_void_p((1 << 20) + 8), 4, 2, 3, Dims(0, 128, 1), fake, None,
                                          None, fake, need) == 1                                # Q misaligned
    assert lib.hdc_cosine_argmax_prepared(None, fake, 4, 2, 3, Dims(0, 128, 1), None, None, None, fake,
                                          need) == 1                                            # no label
    assert lib.hdc_cosine_argmax_prepared(None, None, 0, 2, 3, Dims(0, 128, 1), None, None, None, fake,
                                          need) == 0                                            # n == 0
    assert lib.hdc_cosine_argmax_prepared(None, fake, 4, (1 << 20) + 2, 3, Dims(0, 128, 1), fake, None, None, fake,
                                          need) == 2                                            # ldq too large


def test_f3_validation_without_device(lib):
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.hdc_feature_perforate.argtypes = [p, p, C.c_int, i64, i32, i64, Dims, p, i64]
    lib.hdc_level_quantize.argtypes = [p, p, i64, i32, i64, p, p, i32, p, i64]
    lib.hdc_level_id_encode.argtypes = [p, p, i64, i32, i64, p, i64, p, i32, i64, i32, p, i64]
    fake = C.c_void_p(1 << 20)
    assert lib.hdc_feature_perforate(None, fake, 0, 4, 100, 128, Dims(0, 101, 1), fake, 128) == 1   # end > F
    assert lib.hdc_feature_perforate(None, fake, 2, 4, 100, 128, Dims(0, 100, 1), fake, 128) == 2   # bf16 storage
    assert lib.hdc_feature_perforate(None, fake, 4, 4, 100, 128, Dims(0, 100, 2), fake, 50) == 1    # ldy*4 % 16
    assert lib.hdc_feature_perforate(None, fake, 0, 4, 100, 128, Dims(0, 100, 2), fake, 49) == 1    # ldy < nf
    assert lib.hdc_level_quantize(None, fake, 4, 10, 10, fake, fake, 0, fake, 10) == 1               # L < 1
    assert lib.hdc_level_quantize(None, fake, 4, 10, 9, fake, fake, 4, fake, 10) == 1                # ldx < F
    assert lib.hdc_level_id_encode(None, fake, 4, 1025, 1025, fake, 2, fake, 4, 2, 128, fake, 2) == 2  # F > 1024
    assert lib.hdc_level_id_encode(None, fake, 4, 10, 16, fake, 2, fake, 1025, 2, 128, fake, 2) == 2   # L > 1024
    assert lib.hdc_level_id_encode(None, fake, 4, 10, 10, fake, 2, fake, 4, 2, 128, fake, 2) == 1      # ldl % 8
    assert lib.hdc_level_id_encode(None, fake, 4, 10, 10, fake, 1, fake, 4, 2, 128, fake, 2) == 1      # ldid
    assert lib.hdc_level_id_encode(None, fake, 4, 10, 16, fake, 2, fake, 4, 2, 128, fake, 1) == 1      # ldh
    assert lib.hdc_level_id_encode(None, None, 0, 10, 10, fake, 2, fake, 4, 2, 128, None, 2) == 0      # n == 0


def test_tile_variants_without_device(lib):
    """Variant lists follow the compiled shapes (built-in first); launches
    that name a variant the bucket is not compiled with are refused before
    any device work; the library exports no tile setter."""
    p, i32 = C.c_void_p, C.c_int32
    lib.hdc_tile_variants.restype = i32
    lib.hdc_tile_variants.argtypes = [C.c_int, C.c_int, C.c_int, i32, i32, p, i32]
    ENC, CLS, SWP = 0, 1, 2
    INT8, UINT8, BF16, FP8, FP32 = 0, 1, 2, 3, 4

    def variants(*a):
        buf = (C.c_int32 * 8)()
        n = lib.hdc_tile_variants(*a, buf, 8)
        return None if n < 0 else list(buf[:n])
    # 617 features -> 640-wide int8 kernels: 20 K steps, no two-tile register staging
    assert variants(CLS, INT8, INT8, 617, 26) == [1, 2, 5, 3]
    assert variants(CLS, INT8, INT8, 617, 100) == [2, 3]          # four class tiles: one query tile
    assert variants(CLS, UINT8, INT8, 512, 10) == [4, 3]          # uint8 features: register staging
    assert variants(CLS, INT8, BF16, 617, 26) == [3]
    assert variants(ENC, FP32, FP32, 64, 0) == [4, 3]
    assert variants(SWP, INT8, INT8, 617, 26) == [2, 1, 3, 4]     # built-in: items of 256 queries; 4 shared
    assert variants(SWP, UINT8, INT8, 617, 26) == [2, 1, 3, 4]    # (int8 configurations then stage through registers)
    assert variants(SWP, INT8, INT8, 617, 100) == [2, 1, 4]       # and one class tile
    assert variants(SWP, INT8, INT8, 784, 10) == [2, 1, 4]        # and F <= 640
    assert variants(CLS, FP32, INT8, 64, 2) is None               # no fp32-feature int8 kernels
    assert variants(CLS, INT8, INT8, 2000, 26) is None            # beyond the compiled widths
    assert variants(SWP, FP32, FP32, 64, 2) is None
    # the shifted projection: the two-query-tile direct shapes from 10 K steps
    # (F > 256) and up to two class tiles, int8 features only
    SHIFT = 6
    assert variants(CLS, INT8, SHIFT, 617, 26) == [1, 5]
    assert variants(CLS, INT8, SHIFT, 640, 64) == [1]
    assert variants(ENC, INT8, SHIFT, 617, 0) == [1]
    assert variants(ENC, INT8, SHIFT, 300, 0) == [1]
    assert variants(CLS, INT8, SHIFT, 256, 26) is None
    assert variants(CLS, INT8, SHIFT, 617, 100) is None
    assert variants(CLS, INT8, SHIFT, 1024, 10) is None
    assert variants(CLS, UINT8, SHIFT, 617, 26) is None
    assert variants(CLS, FP32, SHIFT, 64, 2) is None
    # E4M3 on the shifted projection: the direct 2x2 shape, 256 < F <= 640,
    # byte features of either kind, up to two class tiles
    SHIFT8 = 7
    assert variants(CLS, INT8, SHIFT8, 617, 26) == [1]
    assert variants(CLS, UINT8, SHIFT8, 300, 64) == [1]
    assert variants(ENC, INT8, SHIFT8, 640, 0) == [1]
    assert variants(CLS, INT8, SHIFT8, 256, 26) is None
    assert variants(CLS, INT8, SHIFT8, 784, 10) is None
    assert variants(CLS, INT8, SHIFT8, 617, 100) is None
    assert variants(CLS, FP32, SHIFT8, 64, 2) is None
    assert not hasattr(lib, "hdc_set_tile") and not hasattr(lib, "hdc_get_tile")
    p, i64, sz = C.c_void_p, C.c_int64, C.c_size_t
    fake = C.c_void_p(1 << 20)
    lib.hdc_encode_tiled.argtypes = [p, p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, Dims, p, i64, i32]
    # (617 features, int8 -> int8) encode bucket: 2x2 and 1x1 direct staging, register QT1
    assert lib.hdc_encode_tiled(None, fake, INT8, 4, 617, 640, fake, 1024, 640, INT8, Dims(0, 1024, 1), fake,
                                16, 4) == 2                       # two-tile register staging: not compiled
    assert lib.hdc_encode_tiled(None, fake, INT8, 4, 617, 640, fake, 1024, 640, INT8, Dims(0, 1024, 1), fake,
                                16, -1) == 2
    assert lib.hdc_encode_tiled(None, None, INT8, 0, 617, 640, fake, 1024, 640, INT8, Dims(0, 1024, 1), None,
                                16, 2) == 0                       # n == 0 with a compiled variant
    lib.hdc_classify_prepared.argtypes = [p, p, C.c_int, i64, i32, i64, p, i32, i64, C.c_int, Dims, i32, p, p, p,
                                          sz, p, sz, i32]
    assert lib.hdc_classify_prepared(None, fake, INT8, 4, 617, 640, fake, 1024, 640, INT8, Dims(0, 1024, 1), 100,
                                     fake, None, fake, 1 << 20, None, 0, 1) == 2   # 2x2 with four class tiles
    assert lib.hdc_classify_prepared(None, fake, INT8, 0, 617, 640, fake, 1024, 640, INT8, Dims(0, 1024, 1), 100,
                                     fake, None, fake, 1 << 20, None, 0, 2) == 0
    # shifted projection: shapes it has no kernel for are refused, tile 0 included
    assert lib.hdc_classify_prepared(None, fake, INT8, 4, 617, 640, fake, 1024, 640, SHIFT, Dims(0, 1024, 1), 100,
                                     fake, None, fake, 1 << 20, None, 0, 0) == 2
    assert lib.hdc_classify_prepared(None, fake, INT8, 4, 617, 640, fake, 1024, 640, SHIFT, Dims(0, 1024, 1), 26,
                                     fake, None, fake, 1 << 20, None, 0, 2) == 2   # 1x1: not taken
    assert lib.hdc_classify_prepared(None, fake, UINT8, 4, 617, 640, fake, 1024, 640, SHIFT, Dims(0, 1024, 1), 26,
                                     fake, None, fake, 1 << 20, None, 0, 0) == 2
    assert lib.hdc_encode_tiled(None, fake, INT8, 4, 200, 256, fake, 1024, 256, SHIFT, Dims(0, 1024, 1), fake,
                                16, 0) == 2
    assert lib.hdc_classify_prepared(None, fake, INT8, 0, 617, 640, fake, 1024, 640, SHIFT, Dims(0, 1024, 1), 26,
                                     fake, None, fake, 1 << 20, None, 0, 5) == 0



def test_adc_prepared_validation_without_device(lib):
    p, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.hdc_adc_workspace_bytes.restype = C.c_size_t
    lib.hdc_adc_workspace_bytes.argtypes = [Dims, i32]
    lib.hdc_adc_argmax_prepared.argtypes = [p, p, i64, i64, i32, Dims, Adc, p, p, p, p, C.c_size_t]
    # class operand windows from the chunk-aligned word, then one int32 per chunk
    assert lib.hdc_adc_workspace_bytes(Dims(0, 10240, 1), 26) == 20 * 8 * 1024 + 20 * 4 * 4
    assert lib.hdc_adc_workspace_bytes(Dims(64, 4096, 2), 100) == 8 * 8 * 4 * 1024 + 8 * 4 * 4
    assert lib.hdc_adc_workspace_bytes(Dims(200, 1000, 1), 5) == 2 * 8 * 1024 + 2 * 4 * 4
    assert lib.hdc_adc_workspace_bytes(Dims(0, 10240, 1), 129) == 0
    fake = C.c_void_p(1 << 20)
    need = lib.hdc_adc_workspace_bytes(Dims(0, 128, 1), 3)
    ok = Adc(8, 1, -127, 128)
    assert lib.hdc_adc_argmax_prepared(None, fake, 4, 2, 3, Dims(0, 128, 1), Adc(8, 0, 0, 1), fake, None, None,
                                       fake, need) == 1                                       # step < 1
    assert lib.hdc_adc_argmax_prepared(None, fake, 4, 3, 3, Dims(0, 128, 1), ok, fake, None, None, fake,
                                       need) == 1                                             # odd ldq
    assert lib.hdc_adc_argmax_prepared(None, fake, 4, 2, 3, Dims(0, 128, 1), ok, fake, None, None, fake,
                                       need - 1) == 3                                         # small ws
    assert lib.hdc_adc_argmax_prepared(None, None, 0, 2, 3, Dims(0, 128, 1), ok, None, None, None, fake,
                                       need) == 0                                             # n == 0


class Config(C.Structure):
    _fields_ = [("d_trunc", C.c_int32), ("stride", C.c_int32), ("start", C.c_int32), ("dtype", C.c_int32),
                ("tile_id", C.c_int32)]


class ConfigResult(C.Structure):
    _fields_ = [("correct", C.c_int32), ("n", C.c_int32), ("device_us", C.c_double)]


def test_eval_configs_host_arrays_without_device(lib):
    """Configurations and results are host arrays; each configuration's tile
    id is checked against the bucket before any device work; n == 0 writes
    empty results on the host."""
    p, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    assert C.sizeof(Config) == 20 and C.sizeof(ConfigResult) == 16
    lib.hdc_eval_configs.argtypes = [p, p, C.c_int, i64, i32, i64, p, p, i32, i64, p, i32, i64, p, i32, p, p, sz,
                                     i32]
    fake, ws = C.c_void_p(1 << 20), C.c_void_p(1 << 24)
    cfgs = (Config * 3)(Config(1024, 1, 0, 0, 0), Config(2048, 2, 0, 2, 1), Config(10240, 1, 0, 3, 3))
    out = (ConfigResult * 3)()
    for r in out:
        r.correct, r.n, r.device_us = 7, 7, 7.0
    call = lambda X, xt, n, F, c, o, w: lib.hdc_eval_configs(None, X, xt, n, F, 704, fake, fake, 10240, 704,  # noqa
                                                            fake, 26, 160, c, 3, o, ws, w, 0)
    bad = (Config * 3)(Config(1024, 1, 0, 0, 0), Config(2048, 2, 0, 2, 5), Config(10240, 1, 0, 3, 0))
    assert call(fake, 0, 2000, 617, bad, out, 1 << 30) == 2                   # tile id 5: no such variant
    dma = (Config * 3)(Config(1024, 1, 0, 0, 3), Config(2048, 2, 0, 2, 0), Config(10240, 1, 0, 3, 0))
    assert call(fake, 0, 2000, 700, dma, out, 1 << 30) == 2                   # direct staging: F <= 640
    assert call(fake, 0, 2000, 617, None, out, 1 << 30) == 1                  # no configurations
    assert call(fake, 0, 2000, 617, cfgs, None, 1 << 30) == 1                 # no results
    assert call(fake, 0, 2000, 617, cfgs, out, 64) == 3                       # workspace
    assert call(None, 0, 0, 617, cfgs, out, 1 << 30) == 0                     # n == 0
    assert [(r.correct, r.n, r.device_us) for r in out] == [(0, 0, 0.0)] * 3


def test_config_array_layout():
    """The binding's configuration table is the C struct layout (five int32:
    d_trunc, stride, start, dtype, tile_id), tile ids default to the call's,
    and an array already in that form passes through unchanged."""
    import numpy as np

    from paper_2606_26547_amd import hdc
    a = hdc.config_array([(1024, 2, 0, "int8"), (2048, 1, 3, "fp8", 4), (512, 4, 1, hdc.DTYPE["bf16"])], tile=2)
    assert a.dtype == np.int32 and a.shape == (3, 5) and a.flags.c_contiguous
    assert a.tolist() == [[1024, 2, 0, hdc.DTYPE["int8"], 2], [2048, 1, 3, hdc.DTYPE["fp8"], 4],
                          [512, 4, 1, hdc.DTYPE["bf16"], 2]]
    assert C.sizeof(Config) == a.itemsize * a.shape[1]
    assert hdc.config_array(a) is a
    assert hdc.TILE_NAMES["sweep"][4] == "shared"
