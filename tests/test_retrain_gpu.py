"""Retraining on the GPU against the oracle: integer accumulators, models and
per-epoch error counts must be identical (all-integer arithmetic)."""
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


@pytest.mark.parametrize("case", [(2000, 617, 2048, 26, 3), (6238, 617, 10240, 26, 2), (500, 96, 1000, 100, 2),
                                  (300, 64, 64, 2, 4), (20000, 617, 4096, 26, 2), (9000, 128, 1984, 3, 2)],
                         ids=str)
def test_fit_matches_oracle(hdc, case):
    from paper_2606_26547_amd import train
    n, F, D, K, E = case
    say("fit", case)
    X, P = dg.random_case(n, F, D, "int8", seed=n + D)
    y = (np.arange(n) % K).astype(np.int32)
    np.random.default_rng(n).shuffle(y)
    Xd, Pd = hdc.pad_cols(X), hdc.pad_cols(P)
    H = hdc.encode(Xd, F, Pd, D)
    yd = torch.as_tensor(y).cuda()
    Cw, acc, wrong = train.fit(H, D, yd, K, E)
    torch.cuda.synchronize()
    Hn = H.cpu().numpy().view(np.uint64)
    Cref, accref, hist = O.retrain(Hn, y, K, D, E)
    assert [int(w.item()) for w in wrong] == hist
    assert np.array_equal(acc.cpu().numpy(), accref)
    assert np.array_equal(Cw.cpu().numpy().view(np.uint64), Cref)


def test_class_acc_is_bundle_and_correct_rows_change_nothing(hdc):
    say("class_acc")
    g = np.random.default_rng(9)
    n, D, K = 777, 1000, 7
    W = (D + 63) // 64
    Hn = g.integers(0, 2 ** 63, size=(n, W), dtype=np.int64).view(np.uint64)
    Hn[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    y = g.integers(0, K, size=n).astype(np.int32)
    H = torch.as_tensor(Hn.view(np.int64)).cuda()
    yd = torch.as_tensor(y).cuda()
    acc, Cw = hdc.class_acc(H, D, yd, K)
    Cb, _ = hdc.bundle(H, D, yd, K)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), O.class_acc(Hn, y, K, D))
    assert torch.equal(Cw, Cb)
    before = acc.clone()
    w = torch.zeros(1, dtype=torch.int32, device="cuda")
    hdc.retrain_epoch(H, D, yd, yd.clone(), acc, Cw, w)
    torch.cuda.synchronize()
    assert int(w.item()) == 0 and torch.equal(acc, before)
