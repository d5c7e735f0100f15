"""Cosine similarity against integer class accumulators on the GPU against
the oracle: scores bit for bit (exact dot product, correctly rounded
reciprocal square root and product), labels and maxima."""
import numpy as np
import pytest
import torch

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hdc():
    O.build()
    from paper_2606_26547_amd import hdc as H
    return H


def _acc(g, K, nbits, lim):
    return g.integers(-lim, lim + 1, size=(K, nbits), dtype=np.int32)


CASES = [
    # n, nbits, K, perf, accumulator bound
    (1, 64, 1, (0, 64, 1), 5),
    (300, 2048, 10, (0, 2048, 1), 1000),
    (257, 10240, 26, (0, 10240, 1), 32639),
    (129, 1000, 33, (3, 990, 4), 300),
    (64, 8192, 100, (128, 4096, 2), 50),
    (77, 1100, 128, (70, 1100, 1), 32639),
    (513, 4160, 64, (1, 4097, 3), 7),
]


@pytest.mark.parametrize("case", CASES, ids=str)
def test_cosine_bit_exact(hdc, case):
    n, nbits, K, (s, e, k), lim = case
    print("[case] cosine", case, flush=True)
    g = np.random.default_rng(n + nbits + K)
    W = (nbits + 63) // 64
    Q = g.integers(0, 2 ** 63, size=(n, W), dtype=np.int64).view(np.uint64)
    acc = _acc(g, K, nbits, lim)
    if K >= 3:
        acc[2] = acc[0]                           # equal scores: lower index wins
    if K >= 5:
        acc[4] = 0                                # all-zero class scores 0
    ref = O.cosine_scores(Q, acc, s, e, k)
    lref, mref = O.argmax_f64(ref)
    P = hdc.CosinePrepared(torch.as_tensor(acc).cuda(), s, e, k)
    lab, mx, sc = P(torch.as_tensor(Q.view(np.int64)).cuda(), True, True)
    torch.cuda.synchronize()
    assert np.array_equal(sc.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    assert np.array_equal(lab.cpu().numpy(), lref)
    assert np.array_equal(mx.cpu().numpy().view(np.uint64), mref.view(np.uint64))


def test_cosine_bundled_accumulators(hdc):
    """Accumulators as bundling writes them (oracle class_acc of random
    hypervectors), odd row pitch, labels only."""
    print("[case] cosine bundled", flush=True)
    g = np.random.default_rng(7)
    nbits, K = 4095, 26
    H = g.integers(0, 2 ** 63, size=(2000, 64), dtype=np.int64).view(np.uint64)
    H[:, -1] &= np.uint64((1 << 63) - 1)
    y = g.integers(0, K, size=2000).astype(np.int32)
    acc = O.class_acc(H, y, K, nbits)
    Q = g.integers(0, 2 ** 63, size=(333, 65), dtype=np.int64).view(np.uint64)
    ref = O.cosine_scores(Q, acc, 0, nbits, 1)
    lref, _ = O.argmax_f64(ref)
    lab, mx, sc = hdc.CosinePrepared(torch.as_tensor(acc).cuda(), 0, nbits)(torch.as_tensor(Q.view(np.int64)).cuda())
    torch.cuda.synchronize()
    assert mx is None and sc is None
    assert np.array_equal(lab.cpu().numpy(), lref)


def test_cosine_out_of_range(hdc):
    """An accumulator entry over S beyond the two-byte split marks every label
    -1 and every score NaN; one outside S does not."""
    print("[case] cosine range", flush=True)
    g = np.random.default_rng(11)
    acc = _acc(g, 5, 512, 100)
    Q = torch.as_tensor(g.integers(0, 2 ** 63, size=(40, 8), dtype=np.int64)).cuda()
    acc[3, 301] = 32640
    lab, mx, sc = hdc.CosinePrepared(torch.as_tensor(acc).cuda(), 0, 512)(Q, True, True)
    torch.cuda.synchronize()
    assert (lab.cpu().numpy() == -1).all()
    assert np.isnan(mx.cpu().numpy()).all() and np.isnan(sc.cpu().numpy()).all()
    acc[3, 301] = -32640                          # odd dimension: outside S = {0, 2, 4, ...}
    P = hdc.CosinePrepared(torch.as_tensor(acc).cuda(), 0, 512, 2)
    lab, _, sc = P(Q, False, True)
    torch.cuda.synchronize()
    ref = O.cosine_scores(Q.cpu().numpy().view(np.uint64), acc, 0, 512, 2)
    assert np.array_equal(sc.cpu().numpy().view(np.uint64), ref.view(np.uint64))
    assert np.array_equal(lab.cpu().numpy(), O.argmax_f64(ref)[0])


def test_cosine_empty_batch(hdc):
    acc = torch.ones((3, 128), dtype=torch.int32, device="cuda")
    P = hdc.CosinePrepared(acc, 0, 128)
    lab, _, _ = P(torch.zeros((0, 2), dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    assert lab.numel() == 0


def test_cosine_full_size_sampled(hdc):
    """2^20 query hypervectors of 10240 bits against 26 classes, the launch
    the throughput figure times; 2048 sampled rows checked against the
    oracle bit for bit."""
    print("[case] cosine 2^20 x 10240 x 26", flush=True)
    g = np.random.default_rng(20)
    n, nbits, K = 1 << 20, 10240, 26
    acc = _acc(g, K, nbits, 3000)
    gen = torch.Generator(device="cuda").manual_seed(20)
    Q = torch.randint(-(1 << 62), 1 << 62, (n, nbits // 64), dtype=torch.int64, device="cuda", generator=gen)
    lab, mx, _ = hdc.CosinePrepared(torch.as_tensor(acc).cuda(), 0, nbits)(Q, True)
    torch.cuda.synchronize()
    rows = np.sort(g.choice(n, 2048, replace=False))
    rows[-1] = n - 1
    Qs = Q[torch.as_tensor(rows).cuda()].cpu().numpy().view(np.uint64)
    ref = O.cosine_scores(Qs, acc, 0, nbits, 1)
    lref, mref = O.argmax_f64(ref)
    assert np.array_equal(lab.cpu().numpy()[rows], lref)
    assert np.array_equal(mx.cpu().numpy()[rows].view(np.uint64), mref.view(np.uint64))
