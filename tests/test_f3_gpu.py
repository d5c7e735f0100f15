"""Encode-side perforation and Level-ID encoding on the GPU against the
oracle, bit for bit."""
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


def _pad64(X):
    n, F = X.shape
    ld = max(64, (F + 63) // 64 * 64)
    Y = np.zeros((n, ld), dtype=X.dtype)
    Y[:, :F] = X
    return Y


# ------------------------------------------------------------ feature gather
@pytest.mark.parametrize("dtype", [np.int8, np.uint8, np.float32])
@pytest.mark.parametrize("fperf", [(0, 617, 2), (3, 600, 5), (616, 617, 1), (0, 617, 1)])
def test_feature_perforate_gather(hdc, dtype, fperf):
    print("[case] gather", dtype.__name__, fperf, flush=True)
    g = np.random.default_rng(1)
    n, F = 301, 617
    X = g.integers(-100, 100, size=(n, F)).astype(dtype)
    Y = hdc.feature_perforate(torch.as_tensor(_pad64(X)).cuda(), F, *fperf)
    torch.cuda.synchronize()
    cols = np.arange(*fperf)
    want = np.zeros((n, Y.shape[1]), dtype=dtype)
    want[:, :cols.size] = X[:, cols]
    assert np.array_equal(Y.cpu().numpy(), want)


@pytest.mark.parametrize("compute", ["int8", "bf16", "fp8"])
@pytest.mark.parametrize("fperf", [(0, 617, 2), (1, 617, 4), (5, 500, 3)])
def test_fperf_encode_bit_exact(hdc, compute, fperf):
    """Perforated features and projection rows through the encoder equal the
    oracle's rescaled perforated encoding."""
    print("[case] fperf encode", compute, fperf, flush=True)
    g = np.random.default_rng(2)
    n, F, D = 333, 617, 2080
    X = g.integers(-127, 128, size=(n, F), dtype=np.int8)
    P = dg.projection_matrix(D, F, 2)
    Xg = hdc.feature_perforate(torch.as_tensor(_pad64(X)).cuda(), F, *fperf)
    Pg = hdc.feature_perforate(torch.as_tensor(_pad64(P)).cuda(), F, *fperf)
    nf = O.dims_count(*fperf)
    H = hdc.encode(Xg, nf, Pg, D, compute)
    torch.cuda.synchronize()
    want = O.encode_fperf(X, P, *fperf, compute=compute)
    assert np.array_equal(H.cpu().numpy().view(np.uint64), want)


def test_fperf_classify_matches_oracle(hdc):
    """Fused classify on perforated features and projection rows, with
    dimension perforation on top; labels and distances."""
    print("[case] fperf classify", flush=True)
    g = np.random.default_rng(3)
    n, F, D, K = 500, 617, 4096, 26
    X = g.integers(-127, 128, size=(n, F), dtype=np.int8)
    P = dg.projection_matrix(D, F, 3)
    Cw = g.integers(0, 2 ** 63, size=(K, D // 64), dtype=np.int64).view(np.uint64)
    fperf, (s, e, k) = (2, 617, 3), (0, 4096, 2)
    Xg = hdc.feature_perforate(torch.as_tensor(_pad64(X)).cuda(), F, *fperf)
    Pg = hdc.feature_perforate(torch.as_tensor(_pad64(P)).cuda(), F, *fperf)
    lab, dists = hdc.classify(Xg, O.dims_count(*fperf), Pg, D, torch.as_tensor(Cw.view(np.int64)).cuda(),
                              start=s, d_trunc=e, stride=k, with_dists=True)
    torch.cuda.synchronize()
    Hq = O.encode_fperf(X, P, *fperf, start=s, end=e, stride=k)
    # compare query bit j with class bit s + j*k
    ref = np.zeros((n, K), dtype=np.int32)
    qb = np.unpackbits(Hq.view(np.uint8), axis=1, bitorder="little")
    cb = np.unpackbits(Cw.view(np.uint8), axis=1, bitorder="little")[:, s:e:k]
    ref = (qb[:, None, :cb.shape[1]] != cb[None, :, :]).sum(axis=2).astype(np.int32)
    assert np.array_equal(dists.cpu().numpy(), ref)
    assert np.array_equal(lab.cpu().numpy(), O.argmin(ref)[0])


# ------------------------------------------------------------ Level-ID
def test_level_quantize_bit_exact(hdc):
    print("[case] level quantize", flush=True)
    g = np.random.default_rng(4)
    n, F = 777, 93
    X = (g.standard_normal((n, F)) * 2).astype(np.float32)
    X[0, :5] = [np.nan, np.inf, -np.inf, 1e30, -1e30]
    lo, hi = X[1:].min(0) + 0.3, X[1:].max(0) - 0.3
    hi[7] = lo[7]                                              # empty range
    lo[8], hi[8] = 0.0, 37.0                                   # grid column
    X[1:, 8] = np.arange(n - 1, dtype=np.float32) % 37
    for L in (1, 2, 37, 128, 1024):
        lev = hdc.level_quantize(torch.as_tensor(X).cuda(), torch.as_tensor(lo).cuda(), torch.as_tensor(hi).cuda(), L)
        torch.cuda.synchronize()
        assert np.array_equal(lev.cpu().numpy().view(np.uint16), O.level_quantize(X, lo, hi, L)), L


CASES = [
    # n, F, L, D
    (1, 1, 1, 1),
    (37, 5, 4, 70),
    (300, 617, 128, 1024),
    (129, 100, 16, 10240),
    (65, 1024, 1024, 2000),
    (17, 33, 1000, 4095),
    (50, 16, 2, 64),
]


@pytest.mark.parametrize("case", CASES, ids=str)
def test_level_id_encode_bit_exact(hdc, case):
    n, F, L, D = case
    print("[case] level-id", case, flush=True)
    g = np.random.default_rng(n + F + L + D)
    ID = dg.id_hypervectors(F, D, 5)
    LV = dg.level_hypervectors(L, D, 6)
    lev = g.integers(0, L, size=(n, F)).astype(np.uint16)
    H = hdc.level_id_encode(torch.as_tensor(lev.view(np.int16)).cuda(), torch.as_tensor(ID.view(np.int64)).cuda(),
                            torch.as_tensor(LV.view(np.int64)).cuda(), D)
    torch.cuda.synchronize()
    assert np.array_equal(H.cpu().numpy().view(np.uint64), O.level_id_encode(lev, ID, LV, D))


def test_level_id_speech_pipeline(hdc):
    """Float speech-shaped features -> levels over the train ranges ->
    Level-ID hypervectors, against the oracle's chain."""
    print("[case] level-id speech chain", flush=True)
    sp = dg.SpeechLike(2)
    Xtr, _, Xte, _ = sp.float_split()
    lo, hi = dg.feature_ranges(Xtr)
    L, D = 128, 1024
    ID = dg.id_hypervectors(Xte.shape[1], D, 7)
    LV = dg.level_hypervectors(L, D, 8)
    Xd = torch.as_tensor(Xte).cuda()
    lev = hdc.level_quantize(Xd, torch.as_tensor(lo).cuda(), torch.as_tensor(hi).cuda(), L)
    H = hdc.level_id_encode(lev, torch.as_tensor(ID.view(np.int64)).cuda(), torch.as_tensor(LV.view(np.int64)).cuda(),
                            D)
    torch.cuda.synchronize()
    lref = O.level_quantize(Xte, lo, hi, L)
    assert np.array_equal(lev.cpu().numpy().view(np.uint16), lref)
    assert np.array_equal(H.cpu().numpy().view(np.uint64), O.level_id_encode(lref, ID, LV, D))


def test_level_id_full_size_sampled(hdc):
    """2^18 rows of 617 features at L = 128, D = 10240 (the launch the
    throughput figure times); 512 sampled rows checked bit for bit."""
    print("[case] level-id 2^18 x 617 x 10240", flush=True)
    n, F, L, D = 1 << 18, 617, 128, 10240
    gen = torch.Generator(device="cuda").manual_seed(9)
    lev = torch.randint(0, L, (n, F), dtype=torch.int16, device="cuda", generator=gen)
    ID = dg.id_hypervectors(F, D, 9)
    LV = dg.level_hypervectors(L, D, 10)
    H = hdc.level_id_encode(lev, torch.as_tensor(ID.view(np.int64)).cuda(), torch.as_tensor(LV.view(np.int64)).cuda(),
                            D)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(9).choice(n, 512, replace=False))
    rows[-1] = n - 1
    r = torch.as_tensor(rows).cuda()
    ls = lev[r].cpu().numpy().view(np.uint16)
    assert np.array_equal(H[r].cpu().numpy().view(np.uint64), O.level_id_encode(ls, ID, LV, D))


def test_fperf_full_size_sampled(hdc):
    """The bench batch: 2^18 speech-shaped int8 queries, features perforated
    with stride 2, gathered and classified by the fused kernel against 26
    classes at D = 10240; 512 sampled rows' labels and distances against the
    oracle's rescaled perforated encoding."""
    print("[case] fperf 2^18 x 617 x 10240", flush=True)
    n, F, D, K = 1 << 18, 617, 10240, 26
    gen = torch.Generator(device="cuda").manual_seed(41)
    Xd = torch.zeros((n, 640), dtype=torch.int8, device="cuda")
    Xd[:, :F] = torch.randint(-127, 128, (n, F), dtype=torch.int8, device="cuda", generator=gen)
    P = dg.projection_matrix(D, F, 41)
    Cw = torch.randint(-(1 << 62), 1 << 62, (K, D // 64), dtype=torch.int64, device="cuda", generator=gen)
    Pg = hdc.feature_perforate(torch.as_tensor(_pad64(P)).cuda(), F, 0, F, 2)
    nf = O.dims_count(0, F, 2)
    prep = hdc.Prepared(Cw, D, "int8")
    lab, dists = prep(hdc.feature_perforate(Xd, F, 0, F, 2), nf, Pg, with_dists=True)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(41).choice(n, 512, replace=False))
    rows[-1] = n - 1
    r = torch.as_tensor(rows).cuda()
    Xs = Xd[r, :F].cpu().numpy()
    Hq = O.encode_fperf(Xs, P, 0, F, 2)
    ref = O.hamming(Hq, Cw.cpu().numpy().view(np.uint64), 0, D, 1)
    assert np.array_equal(dists[r].cpu().numpy(), ref)
    assert np.array_equal(lab[r].cpu().numpy(), O.argmin(ref)[0])
