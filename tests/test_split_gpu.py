"""Dimension-split launches: a batch too small to fill the device spreads
the dimension list over several workgroups per query block (encode: each
writes its own words; classify: integer partial class sums, then an argmin
kernel).  Every tile variant, with and without splits, gives the oracle's
codes, labels and distances bit for bit."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hdc():
    O.build()
    from paper_2606_26547_amd import hdc as H
    return H


def say(*a):
    print("[case]", *a, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def classes(K, D, seed):
    g = np.random.default_rng(seed)
    Cw = g.integers(0, 2 ** 63, size=(K, (D + 63) // 64), dtype=np.int64).view(np.uint64)
    if D % 64:
        Cw[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    return Cw


CASES = [
    # n, F, D, K, x_type, compute, (start, d_trunc, stride)
    (1, 617, 10240, 26, "int8", "int8", None),
    (63, 617, 10240, 26, "int8", "int8", None),
    (1559, 617, 10240, 26, "int8", "int8", None),
    (63, 617, 10240, 26, "int8", "int8", (1, 9001, 2)),
    (200, 617, 10240, 26, "int8", "bf16", (0, 8192, 1)),
    (100, 784, 8192, 10, "uint8", "int8", None),
    (100, 784, 8192, 10, "uint8", "fp8split", (3, 8000, 3)),
    (40, 1024, 16384, 100, "int8", "int8", None),
]


@pytest.mark.parametrize("case", CASES, ids=str)
def test_split_classify_matches_oracle(hdc, case):
    n, F, D, K, xt, ct, dims = case
    start, d_trunc, stride = dims or (0, D, 1)
    nd = hdc.dims_count(start, d_trunc, stride)
    assert int(hdc.lib().hdc_classify_scratch_bytes(n, nd, K)) > 0, "the case must split"
    X, P = dg.random_case(n, F, D, xt, seed=n + F + D)
    Cw = classes(K, D, n + K)
    Cw[min(2, K - 1)] = Cw[0]                     # a duplicate class: the lower index wins ties
    lref, dref = O.classify(X, P, Cw, ct, start, d_trunc, stride, with_dists=True)
    Xd, Pd, Cd = hdc.pad_cols(X), hdc.pad_cols(P), dev(Cw.view(np.int64))
    variants = hdc.tile_variants("classify", xt, ct, F, K)
    for v in variants:
        for split in (True, False):
            say("split classify", case, "variant", v, "split", split)
            lab, dists = hdc.classify(Xd, F, Pd, D, Cd, ct, start, d_trunc, stride, with_dists=True, split=split,
                                      tile=v)
            torch.cuda.synchronize()
            assert np.array_equal(dists.cpu().numpy(), dref), (v, split)
            assert np.array_equal(lab.cpu().numpy(), lref), (v, split)


def test_split_prepared_reuses_scratch(hdc):
    """One prepared model, batches of several sizes in a row (the scratch
    grows, then is reused by smaller batches), each equal to the oracle."""
    F, D, K = 617, 10240, 26
    X, P = dg.random_case(3000, F, D, "int8", seed=4)
    Cw = classes(K, D, 5)
    prep = hdc.Prepared(dev(Cw.view(np.int64)), D, "int8")
    Xd, Pd = hdc.pad_cols(X), hdc.pad_cols(P)
    lref, dref = O.classify(X, P, Cw, "int8", with_dists=True)
    for rows in (slice(0, 700), slice(0, 3000), slice(100, 101), slice(5, 1564)):
        say("prepared split", rows)
        lab, dists = prep(Xd[rows], F, Pd, with_dists=True)
        torch.cuda.synchronize()
        assert np.array_equal(lab.cpu().numpy(), lref[rows])
        assert np.array_equal(dists.cpu().numpy(), dref[rows])


ENC_CASES = [
    # n, F, D, x_type, compute, (start, end, stride)
    (1, 617, 10240, "int8", "int8", None),
    (63, 617, 10240, "int8", "int8", (0, 10000, 1)),
    (1559, 617, 10240, "int8", "int8", None),
    (6238, 617, 10240, "int8", "int8", None),
    (100, 784, 8192, "uint8", "int8", (5, 8192, 3)),
    (300, 617, 10240, "int8", "fp8split", None),
    (64, 64, 2048, "fp32", "fp32", None),
]


@pytest.mark.parametrize("case", ENC_CASES, ids=str)
def test_split_encode_matches_oracle(hdc, case):
    n, F, D, xt, ct, dims = case
    s, e, k = dims or (0, D, 1)
    X, P = dg.random_case(n, F, D, xt, seed=7 * n + D)
    Xd, Pd = hdc.pad_cols(X), hdc.pad_cols(P)
    variants = hdc.tile_variants("encode", xt, ct, F, 1)
    for v in variants:
        say("split encode", case, "variant", v)
        H = hdc.encode(Xd, F, Pd, D, ct, s, e, k, tile=v)
        torch.cuda.synchronize()
        got = H.cpu().numpy().view(np.uint64)
        if xt == "fp32":
            # the sign must be exact wherever |y| exceeds the fp32
            # summation band gamma_F * sum |x'| (2x slack)
            nb = hdc.dims_count(s, e, k)
            Y, absum = O.project(X, P, ct, s, e, k)
            rb = np.unpackbits(O.encode(X, P, ct, s, e, k).view(np.uint8), axis=1, bitorder="little")[:, :nb]
            gb = np.unpackbits(got.view(np.uint8), axis=1, bitorder="little")[:, :nb]
            gamma = 2 * F * 2.0 ** -24 / (1 - F * 2.0 ** -24)
            sure = np.abs(Y) > gamma * absum[:, None]
            assert np.array_equal(gb[sure], rb[sure]), v
        else:
            assert np.array_equal(got, O.encode(X, P, ct, s, e, k)), v
