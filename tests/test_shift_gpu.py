"""GPU parity of the int8 path on the shifted projection (compute
"int8shift": weights p + 1 in {0, 2}, every sum started from minus the
query's feature sum) against the oracle's int8 encoding on the +-1
projection the shifted one is made from.  Integer arithmetic on both sides:
labels, distances and packed words must match bit for bit."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hdc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_26547_amd import hdc as H
    return H


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def class_words(K, D, seed):
    g = np.random.default_rng(seed)
    Cw = g.integers(0, 2 ** 63, size=(K, (D + 63) // 64), dtype=np.int64).view(np.uint64)
    if D % 64:
        Cw[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    return Cw


def test_shift_projection_layout(hdc):
    """out = P + 1 in the feature columns, 0 in the pad columns; in place
    with the same pitch; overlapping buffers of another pitch refused."""
    say("shift layout")
    D, F = 300, 617
    _, P = dg.random_case(1, F, D, "int8", seed=5)
    Pd = hdc.pad_cols(P)
    Pd[:, F:] = 5                                   # pad content must not leak into the output
    S = hdc.shift_projection(Pd, F)
    torch.cuda.synchronize()
    ref = np.zeros(Pd.shape, np.int8)
    ref[:, :F] = P + 1
    assert np.array_equal(S.cpu().numpy(), ref)
    assert set(np.unique(S.cpu().numpy()[:, :F])) <= {0, 2}
    # a wider output pitch
    W = torch.full((D, 1024), 9, dtype=torch.int8, device="cuda")
    hdc.shift_projection(Pd, F, out=W)
    torch.cuda.synchronize()
    refw = np.zeros((D, 1024), np.int8)
    refw[:, :F] = P + 1
    assert np.array_equal(W.cpu().numpy(), refw)
    # in place
    Q = Pd.clone()
    hdc.shift_projection(Q, F, out=Q)
    torch.cuda.synchronize()
    assert np.array_equal(Q.cpu().numpy(), ref)
    # the E4M3 form: 2.0 = 0x40 where p = +1, 0 where p = -1 and in the pad
    E = hdc.shift_projection(Pd, F, compute="fp8shift")
    torch.cuda.synchronize()
    refe = np.zeros(Pd.shape, np.uint8)
    refe[:, :F] = np.where(P > 0, 0x40, 0)
    assert np.array_equal(E.cpu().numpy().view(np.uint8), refe)
    lib = hdc.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    I8S, FP8 = hdc.DTYPE["int8shift"], hdc.DTYPE["fp8"]
    # overlap with another pitch, misaligned pitch, F past the pitch: refused before any launch
    assert lib.hdc_shift_projection(st, C.c_void_p(W.data_ptr()), D // 2, F, 1024, I8S,
                                    C.c_void_p(W.data_ptr() + 64), 640) == 1
    assert lib.hdc_shift_projection(st, C.c_void_p(Pd.data_ptr()), D, F, 640, I8S, C.c_void_p(W.data_ptr()),
                                    648) == 1
    assert lib.hdc_shift_projection(st, C.c_void_p(Pd.data_ptr()), D, 700, 640, I8S, C.c_void_p(W.data_ptr()),
                                    1024) == 1
    assert lib.hdc_shift_projection(st, C.c_void_p(Pd.data_ptr()), D, 1025, 640, I8S, C.c_void_p(W.data_ptr()),
                                    1024) == 2
    assert lib.hdc_shift_projection(st, C.c_void_p(Pd.data_ptr()), D, F, 640, FP8, C.c_void_p(W.data_ptr()),
                                    1024) == 2                # not a shifted type


CLS_SHIFT = [
    # n, F, D, K, (start, d_trunc, stride)
    (1, 617, 1024, 26, None),
    (63, 617, 2048, 26, (0, 1000, 1)),
    (257, 617, 2048, 26, (3, 2048, 2)),
    (700, 617, 4096, 26, None),
    (130, 300, 1536, 40, (1, 1500, 3)),
    (200, 640, 1024, 64, None),
    (129, 512, 2000, 7, (5, 1995, 1)),
    (513, 400, 1100, 33, (0, 1100, 7)),
]


@pytest.mark.parametrize("case", CLS_SHIFT, ids=str)
def test_classify_shifted_bit_exact(hdc, case):
    """Every classify variant of the shifted type, labels and distances
    equal to the oracle's int8 classification on the +-1 projection."""
    n, F, D, K, dims = case
    start, d_trunc, stride = dims or (0, D, 1)
    X, P = dg.random_case(n, F, D, "int8", seed=7 * n + F)
    Cw = class_words(K, D, n + K)
    lref, dref = O.classify(X, P, Cw, "int8", start, d_trunc, stride, with_dists=True)
    Xd, Pd, Cd = hdc.pad_cols(X), hdc.pad_cols(P), dev(Cw.view(np.int64))
    Ps = hdc.shift_projection(Pd, F)
    variants = hdc.tile_variants("classify", "int8", "int8shift", F, K)
    assert variants, "no shifted variant for F=%d K=%d" % (F, K)
    for v in [0] + variants:
        say("classify shifted", case, "variant", v)
        lab, dist = hdc.classify(Xd, F, Ps, D, Cd, "int8shift", start, d_trunc, stride, with_dists=True, tile=v)
        torch.cuda.synchronize()
        assert np.array_equal(dist.cpu().numpy(), dref), v
        assert np.array_equal(lab.cpu().numpy(), lref), v


def test_classify_shifted_without_splits(hdc):
    """A small batch run without dimension splits (one workgroup per query
    block walks every dimension) gives the same results."""
    n, F, D, K = 300, 617, 3000, 26
    say("classify shifted, no splits")
    X, P = dg.random_case(n, F, D, "int8", seed=41)
    Cw = class_words(K, D, 3)
    lref, dref = O.classify(X, P, Cw, "int8", 0, D, 1, with_dists=True)
    Ps = hdc.shift_projection(hdc.pad_cols(P), F)
    lab, dist = hdc.classify(hdc.pad_cols(X), F, Ps, D, dev(Cw.view(np.int64)), "int8shift", with_dists=True,
                             split=False)
    torch.cuda.synchronize()
    assert np.array_equal(dist.cpu().numpy(), dref)
    assert np.array_equal(lab.cpu().numpy(), lref)


ENC_SHIFT = [
    # n, F, D, (start, end, stride)
    (1, 617, 640, None),
    (65, 617, 2048, (0, 1000, 1)),
    (520, 617, 10240, (0, 4000, 3)),
    (257, 300, 2000, (5, 1995, 1)),
    (300, 640, 1100, (3, 1100, 7)),
]


@pytest.mark.parametrize("case", ENC_SHIFT, ids=str)
def test_encode_shifted_bit_exact(hdc, case):
    n, F, D, dims = case
    start, end, stride = dims or (0, D, 1)
    say("encode shifted", case)
    X, P = dg.random_case(n, F, D, "int8", seed=11 * n + F)
    ref = O.encode(X, P, "int8", start, end, stride)
    Ps = hdc.shift_projection(hdc.pad_cols(P), F)
    for v in [0] + hdc.tile_variants("encode", "int8", "int8shift", F, 1):
        H = hdc.encode(hdc.pad_cols(X), F, Ps, D, "int8shift", start, end, stride, tile=v)
        torch.cuda.synchronize()
        assert np.array_equal(H.cpu().numpy().view(np.uint64), ref), v


def test_shifted_features_at_the_int8_extremes(hdc):
    """Features of -128 and 127 everywhere: the largest feature sums the
    start values take (|sum| up to 128 * F), both signs."""
    n, F, D, K = 130, 617, 1024, 26
    say("shifted extremes")
    _, P = dg.random_case(1, F, D, "int8", seed=2)
    X = np.full((n, F), 127, np.int8)
    X[1::2] = -128
    X[::3, ::5] = 0
    Cw = class_words(K, D, 9)
    lref, dref = O.classify(X, P, Cw, "int8", 0, D, 1, with_dists=True)
    Ps = hdc.shift_projection(hdc.pad_cols(P), F)
    lab, dist = hdc.classify(hdc.pad_cols(X), F, Ps, D, dev(Cw.view(np.int64)), "int8shift", with_dists=True)
    torch.cuda.synchronize()
    assert np.array_equal(dist.cpu().numpy(), dref)
    assert np.array_equal(lab.cpu().numpy(), lref)


def test_shifted_refuses_what_it_does_not_run(hdc):
    """uint8 features, F of 256 or less, more than 64 classes and the
    one-query-tile shapes are refused (HDC_ERR_UNSUPPORTED) before any
    launch."""
    say("shifted refusals")
    for xt, F, K in [("uint8", 617, 26), ("int8", 256, 26), ("int8", 617, 100)]:
        with pytest.raises(hdc.HDCError):
            hdc.tile_variants("classify", xt, "int8shift", F, K)
    X, P = dg.random_case(8, 617, 256, "int8", seed=1)
    Ps = hdc.shift_projection(hdc.pad_cols(P), 617)
    Cd = dev(class_words(26, 256, 1).view(np.int64))
    one = {v: k for k, v in hdc.TILE_NAMES["classify"].items()}["dma_1x1"]
    with pytest.raises(hdc.HDCError) as e:
        hdc.classify(hdc.pad_cols(X), 617, Ps, 256, Cd, "int8shift", tile=one)
    assert e.value.code == 2
    Xs, Psm = dg.random_case(8, 200, 256, "int8", seed=1)
    with pytest.raises(hdc.HDCError) as e:
        hdc.classify(hdc.pad_cols(Xs), 200, hdc.shift_projection(hdc.pad_cols(Psm), 200), 256, Cd, "int8shift")
    assert e.value.code == 2


CLS_SHIFT8 = [
    # n, F, D, K, x_type, (start, d_trunc, stride)
    (1, 617, 1024, 26, "int8", None),
    (63, 617, 2048, 26, "int8", (0, 1000, 1)),
    (700, 617, 4096, 26, "int8", (3, 4096, 2)),
    (130, 300, 1536, 40, "int8", (1, 1500, 3)),
    (257, 512, 2000, 64, "uint8", None),
    (90, 640, 1100, 7, "uint8", (0, 1100, 7)),
]


@pytest.mark.parametrize("case", CLS_SHIFT8, ids=str)
def test_classify_fp8_shifted_equals_fp8(hdc, case):
    """E4M3 on the shifted projection: labels and distances equal to the
    oracle's E4M3 classification (features rounded to E4M3, +-1 weights,
    exact sums) on the +-1 projection, split and unsplit launches."""
    n, F, D, K, xt, dims = case
    start, d_trunc, stride = dims or (0, D, 1)
    X, P = dg.random_case(n, F, D, xt, seed=5 * n + F)
    Cw = class_words(K, D, n + 2 * K)
    lref, dref = O.classify(X, P, Cw, "fp8", start, d_trunc, stride, with_dists=True)
    Xd, Cd = hdc.pad_cols(X), dev(Cw.view(np.int64))
    Pe = hdc.shift_projection(hdc.pad_cols(P), F, compute="fp8shift")
    assert hdc.tile_variants("classify", xt, "fp8shift", F, K) == [1]
    for split in (True, False):
        say("classify fp8 shifted", case, "split", split)
        lab, dist = hdc.classify(Xd, F, Pe, D, Cd, "fp8shift", start, d_trunc, stride, with_dists=True,
                                 split=split)
        torch.cuda.synchronize()
        assert np.array_equal(dist.cpu().numpy(), dref), split
        assert np.array_equal(lab.cpu().numpy(), lref), split


@pytest.mark.parametrize("case", [(65, 617, 2048, "int8", (0, 1000, 1)), (300, 640, 1100, "uint8", (3, 1100, 7)),
                                  (520, 617, 10240, "int8", None)], ids=str)
def test_encode_fp8_shifted_equals_fp8(hdc, case):
    n, F, D, xt, dims = case
    start, end, stride = dims or (0, D, 1)
    say("encode fp8 shifted", case)
    X, P = dg.random_case(n, F, D, xt, seed=13 * n + F)
    ref = O.encode(X, P, "fp8", start, end, stride)
    Pe = hdc.shift_projection(hdc.pad_cols(P), F, compute="fp8shift")
    H = hdc.encode(hdc.pad_cols(X), F, Pe, D, "fp8shift", start, end, stride)
    torch.cuda.synchronize()
    assert np.array_equal(H.cpu().numpy().view(np.uint64), ref)
