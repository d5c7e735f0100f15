"""The precision ladder on the GPU (Sec. 4.2, "Element Type
Representation"): the split E4M3 rung against the oracle bit for bit, and
every rung's sign-flip rate and accuracy change measured against the exact
(int / FP64) encoding on the speech and image test sets.  Bounds: flip rate
<= 1e-3 and |accuracy change| <= 0.5 points.  Direct E4M3 misses the flip
bound (about 0.8% of the signs change, the rate its 4 significant bits
imply); that shortfall is asserted as an expected failure so the suite
notices if it ever changes."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg

pytestmark = pytest.mark.gpu

FLIP_BOUND = 1e-3
ACC_BOUND_PTS = 0.5


@pytest.fixture(scope="module")
def hdc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2606_26547_amd import hdc as H
    return H


def say(*a):
    print("[case]", *a, flush=True)


def bits(H, nbits):
    H = np.ascontiguousarray(H).view(np.uint64)
    return np.unpackbits(H.view(np.uint8).reshape(H.shape[0], -1), axis=1, bitorder="little")[:, :nbits]


SPLIT_CASES = [
    # n, F, D, x_type, (start, end, stride)
    (1, 1, 64, "int8", None),
    (63, 63, 96, "int8", None),
    (300, 617, 2048, "int8", (0, 1000, 1)),
    (257, 784, 1100, "uint8", (3, 1100, 7)),
    (129, 1000, 512, "int8", (1, 512, 2)),
    (70, 130, 700, "uint8", (5, 690, 3)),
    (520, 617, 10240, "int8", (0, 4000, 3)),
]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=str)
def test_split_e4m3_encode_is_the_exact_encoding(hdc, case):
    n, F, D, xt, dims = case
    start, end, stride = dims or (0, D, 1)
    say("fp8split encode", case)
    X, P = dg.random_case(n, F, D, xt, seed=n + F + D + 5)
    if xt == "int8":
        X[0, :min(F, 4)] = [-128, 127, -1, 16][:min(F, 4)]
    else:
        X[0, :min(F, 3)] = [255, 240, 15][:min(F, 3)]
    ref = O.encode(X, P, "fp8split", start, end, stride)
    assert np.array_equal(ref, O.encode(X, P, "int8", start, end, stride))
    H = hdc.encode(hdc.pad_cols(X), F, hdc.pad_cols(P), D, "fp8split", start, end, stride)
    torch.cuda.synchronize()
    assert np.array_equal(H.cpu().numpy().view(np.uint64), ref)


@pytest.mark.parametrize("case", [(300, 617, 2048, 26, "int8", None), (257, 784, 1024, 10, "uint8", (0, 1024, 2)),
                                  (200, 617, 1024, 100, "int8", (2, 1000, 3)), (65, 64, 640, 40, "int8", None)],
                         ids=str)
def test_split_e4m3_classify_bit_exact(hdc, case):
    n, F, D, K, xt, dims = case
    start, end, stride = dims or (0, D, 1)
    say("fp8split classify", case)
    X, P = dg.random_case(n, F, D, xt, seed=n + K)
    g = np.random.default_rng(K + 1)
    Cw = g.integers(0, 2 ** 63, size=(K, D // 64), dtype=np.int64).view(np.uint64)
    if K >= 3:
        Cw[2] = Cw[0]
    lref, dref = O.classify(X, P, Cw, "fp8split", start, end, stride, with_dists=True)
    lab, dists = hdc.classify(hdc.pad_cols(X), F, hdc.pad_cols(P), D, torch.as_tensor(Cw.view(np.int64)).cuda(),
                              "fp8split", start, end, stride, with_dists=True)
    torch.cuda.synchronize()
    assert np.array_equal(dists.cpu().numpy(), dref)
    assert np.array_equal(lab.cpu().numpy(), lref)


def _ladder(hdc, X, y, P, Cw, rung):
    """GPU encoding and fused labels under one rung, against the exact
    encoding and the exact labels from the oracle."""
    F, D = X.shape[1], P.shape[0]
    Xd, Pd = hdc.pad_cols(X), hdc.pad_cols(P)
    H = hdc.encode(Xd, F, Pd, D, rung)
    lab = hdc.classify(Xd, F, Pd, D, torch.as_tensor(Cw.view(np.int64)).cuda(), rung)
    torch.cuda.synchronize()
    exact = O.encode(X, P, "int8")
    flip = float((bits(H.cpu().numpy(), D) != bits(exact, D)).mean())
    lab_exact = O.classify(X, P, Cw, "int8")
    acc = float((lab.cpu().numpy() == y).mean())
    acc_exact = float((lab_exact == y).mean())
    return flip, 100.0 * (acc - acc_exact)


@pytest.fixture(scope="module")
def speech():
    d = dg.SpeechLike(2).dataset()
    Cw, _ = O.train(d.X_train, d.y_train, d.P, d.K)
    return d.X_test, d.y_test, d.P, Cw


@pytest.fixture(scope="module")
def image():
    # model from the first 6000 training images (the oracle encodes them
    # exactly; the whole 60000 would take minutes on the host)
    d = dg.ImageLike(3).dataset()
    Cw, _ = O.train(d.X_train[:6000], d.y_train[:6000], d.P, d.K)
    return d.X_test[:2000], d.y_test[:2000], d.P, Cw


@pytest.mark.parametrize("workload", ["speech", "image"])
@pytest.mark.parametrize("rung", ["bf16", "fp8split"])
def test_ladder_rung_meets_flip_and_accuracy_bounds(hdc, request, workload, rung):
    X, y, P, Cw = request.getfixturevalue(workload)
    say("ladder", workload, rung)
    flip, dacc = _ladder(hdc, X, y, P, Cw, rung)
    print("[ladder] %s %s flip %.2e, accuracy change %+.2f pt" % (workload, rung, flip, dacc), flush=True)
    assert flip <= FLIP_BOUND
    assert abs(dacc) <= ACC_BOUND_PTS
    assert flip == 0.0            # on integer features both rungs are exact


@pytest.mark.parametrize("workload", ["speech", "image"])
def test_direct_e4m3_accuracy_within_bound(hdc, request, workload):
    X, y, P, Cw = request.getfixturevalue(workload)
    say("ladder direct fp8 accuracy", workload)
    flip, dacc = _ladder(hdc, X, y, P, Cw, "fp8")
    print("[ladder] %s fp8 flip %.2e, accuracy change %+.2f pt" % (workload, flip, dacc), flush=True)
    assert abs(dacc) <= ACC_BOUND_PTS
    assert 2e-3 < flip < 3e-2     # the rate 4 significant bits give (not a parity check)


@pytest.mark.xfail(strict=True, reason="direct E4M3 rounds features above 16 to 4 significant bits: about 0.8% "
                                       "of the signs flip, over the 1e-3 bound; the split rung meets it")
@pytest.mark.parametrize("workload", ["speech", "image"])
def test_direct_e4m3_flip_bound(hdc, request, workload):
    X, y, P, Cw = request.getfixturevalue(workload)
    say("ladder direct fp8 flip bound", workload)
    flip, _ = _ladder(hdc, X, y, P, Cw, "fp8")
    assert flip <= FLIP_BOUND
