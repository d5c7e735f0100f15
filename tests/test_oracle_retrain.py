"""Pins of the oracle's retraining (the reading of the unstated update rule:
for each mispredicted row, add its bipolar hypervector to the true class's
integer accumulator and subtract it from the predicted class's, then
re-binarise; a whole epoch is predicted with the model at its start).
Each check is independent of the oracle's own arithmetic: unpacked numpy
bits, pure-Python loops, closed forms and invariants."""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module", autouse=True)
def built():
    O.build()


def bits(H, nbits):
    """Unpacked bits [n][nbits] of packed rows (LSB-first words)."""
    return np.unpackbits(np.ascontiguousarray(H).view(np.uint8), axis=1, bitorder="little")[:, :nbits]


def rand_case(n, nbits, K, seed):
    g = np.random.default_rng(seed)
    W = (nbits + 63) // 64
    H = g.integers(0, 2 ** 63, size=(n, W), dtype=np.int64).view(np.uint64).copy()
    if nbits % 64:
        H[:, -1] &= np.uint64((1 << (nbits % 64)) - 1)
    y = g.integers(0, K, size=n).astype(np.int32)
    return H, y, g


def test_accumulators_are_bipolar_class_sums():
    H, y, _ = rand_case(40, 130, 5, 1)
    acc = O.class_acc(H, y, 5, 130)
    b = 1 - 2 * bits(H, 130).astype(np.int64)
    for k in range(5):
        assert np.array_equal(acc[k], b[y == k].sum(0))


def test_binarised_accumulators_are_the_majority_bundle():
    # even class sizes make ties (sum 0 -> +1) appear
    for seed in range(4):
        H, y, _ = rand_case(64, 200, 4, 10 + seed)
        y = np.repeat(np.arange(4, dtype=np.int32), 16)
        acc = O.class_acc(H, y, 4, 200)
        Cw, _ = O.bundle(H, y, 4, 200)
        assert np.array_equal(O.binarize(acc, 200), Cw)
        assert np.array_equal(O.binarize(acc, 200), O.bundle_bipolar(H, y, 4, 200))
        assert (acc == 0).any()


def test_correct_predictions_change_nothing():
    H, y, _ = rand_case(30, 100, 3, 2)
    acc = O.class_acc(H, y, 3, 100)
    before = acc.copy()
    assert O.retrain_epoch(H, y, y.copy(), acc, 100) == 0
    assert np.array_equal(acc, before)


def test_one_misprediction_moves_two_rows_by_the_hypervector():
    H, y, g = rand_case(30, 100, 3, 3)
    acc = O.class_acc(H, y, 3, 100)
    before = acc.copy()
    pred = y.copy()
    i = 7
    pred[i] = (y[i] + 1) % 3
    assert O.retrain_epoch(H, y, pred, acc, 100) == 1
    b = 1 - 2 * bits(H[i:i + 1], 100)[0].astype(np.int64)
    assert np.array_equal(acc[y[i]] - before[y[i]], b)
    assert np.array_equal(acc[pred[i]] - before[pred[i]], -b)
    other = 3 - y[i] - pred[i]
    assert np.array_equal(acc[other], before[other])


def test_epoch_conserves_column_sums():
    H, y, g = rand_case(80, 190, 6, 4)
    acc = O.class_acc(H, y, 6, 190)
    col = acc.sum(0)
    pred = g.integers(0, 6, size=80).astype(np.int32)
    O.retrain_epoch(H, y, pred, acc, 190)
    assert np.array_equal(acc.sum(0), col)


def test_brute_force_tiny():
    # every label assignment of 4 rows to 2 classes, every prediction vector
    H, _, _ = rand_case(4, 8, 2, 5)
    b = [[1 - 2 * int((int(H[i, 0]) >> d) & 1) for d in range(8)] for i in range(4)]
    for lab in range(16):
        y = np.array([(lab >> i) & 1 for i in range(4)], dtype=np.int32)
        for pr in range(16):
            pred = np.array([(pr >> i) & 1 for i in range(4)], dtype=np.int32)
            ref = [[sum(b[i][d] for i in range(4) if y[i] == k) for d in range(8)] for k in range(2)]
            for i in range(4):
                if pred[i] != y[i]:
                    for d in range(8):
                        ref[y[i]][d] += b[i][d]
                        ref[pred[i]][d] -= b[i][d]
            acc = O.class_acc(H, y, 2, 8)
            O.retrain_epoch(H, y, pred, acc, 8)
            assert acc.tolist() == ref
            words = [sum(1 << d for d in range(8) if ref[k][d] < 0) for k in range(2)]
            assert O.binarize(acc, 8)[:, 0].tolist() == words


def test_retrain_loop_counts_training_errors():
    H, y, _ = rand_case(60, 256, 4, 6)
    Cw, acc, hist = O.retrain(H, y, 4, 256, 3)
    # the first entry is the training error of the bundled model
    C0, _ = O.bundle(H, y, 4, 256)
    lab, _ = O.argmin(O.hamming(H, C0, 0, 256, 1))
    assert hist[0] == int((lab != y).sum())
    assert np.array_equal(Cw, O.binarize(acc, 256))
