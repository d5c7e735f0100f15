"""Pins of the oracle's cosine similarity against integer class accumulators
(bipolar query; the query norm, common to all classes, left out)."""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module", autouse=True)
def built():
    O.build()


def rand_case(n, D, K, seed, amp=50):
    g = np.random.default_rng(seed)
    W = (D + 63) // 64
    Q = g.integers(0, 2 ** 63, size=(n, W), dtype=np.int64).view(np.uint64).copy()
    if D % 64:
        Q[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    acc = g.integers(-amp, amp + 1, size=(K, D)).astype(np.int32)
    return Q, acc, g


def test_scores_by_numpy():
    Q, acc, _ = rand_case(20, 300, 6, 1)
    b = 1 - 2 * np.unpackbits(Q.view(np.uint8), axis=1, bitorder="little")[:, :300].astype(np.int64)
    for (s, e, k) in [(0, 300, 1), (7, 290, 3)]:
        idx = np.arange(s, e, k)
        dot = b[:, idx] @ acc[:, idx].T.astype(np.int64)
        nsq = (acc[:, idx].astype(np.int64) ** 2).sum(1)
        ref = dot.astype(np.float64) * (1.0 / np.sqrt(nsq.astype(np.float64)))
        got = O.cosine_scores(Q, acc, s, e, k)
        assert np.array_equal(got, ref)          # same IEEE operations, bit for bit


def test_scaled_bipolar_classes_reduce_to_hamming():
    g = np.random.default_rng(2)
    D, K = 1000, 9
    Q, _, _ = rand_case(50, D, K, 3)
    Cw = g.integers(0, 2 ** 63, size=(K, 16), dtype=np.int64).view(np.uint64)
    Cw[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    bc = 1 - 2 * np.unpackbits(Cw.view(np.uint8), axis=1, bitorder="little")[:, :D].astype(np.int32)
    acc = (bc * 37).astype(np.int32)
    sc = O.cosine_scores(Q, acc, 0, D, 1)
    dist = O.hamming(Q, Cw, 0, D, 1)
    # score = 37 (D - 2 ham) / (37 sqrt(D)) up to rounding; the order is Hamming's
    assert np.allclose(sc, (D - 2.0 * dist) / np.sqrt(D), rtol=0, atol=1e-9)
    lab, _ = O.argmax_f64(sc)
    ref, _ = O.argmin(dist)
    assert np.array_equal(lab, ref)


def test_scale_invariance_and_zero_class():
    Q, acc, _ = rand_case(30, 500, 5, 4)
    lab1, _ = O.argmax_f64(O.cosine_scores(Q, acc, 0, 500))
    lab2, _ = O.argmax_f64(O.cosine_scores(Q, acc * 3, 0, 500))
    assert np.array_equal(lab1, lab2)
    acc[2] = 0
    sc = O.cosine_scores(Q, acc, 0, 500)
    assert (sc[:, 2] == 0).all()


def test_argmax_f64_first_maximum():
    lab, mx = O.argmax_f64(np.array([[0.5, 0.5, 0.1], [-1.0, -2.0, -1.0]]))
    assert lab.tolist() == [0, 0] and mx.tolist() == [0.5, -1.0]
