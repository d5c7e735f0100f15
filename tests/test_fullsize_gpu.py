"""Parity at the workloads' own sizes and shapes: the plain fp32 workload
end to end (fp32 features -> encode -> bundle -> fused classify), the
speech-shaped headline classify on a 2^18-query batch under every tile
variant (sampled rows, labels and distances against the oracle), and the
largest serving model (1024 features, 100 classes, D = 16384), plain and
tuned."""
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


def bits(H, nbits):
    H = np.ascontiguousarray(H).view(np.uint64)
    return np.unpackbits(H.view(np.uint8).reshape(H.shape[0], -1), axis=1, bitorder="little")[:, :nbits]


def u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("ct", ["fp32", "bf16", "fp8"])
def test_plain_fp32_workload_end_to_end(hdc, ct):
    """1000 train / 200 test vectors of 64 fp32 features, D = 2048.  Where
    the exact projection lies outside fp32 summation's error band the GPU
    sign must be the oracle's; integer steps (bundle, Hamming, argmin) on
    the GPU's bits must be the oracle's bit for bit; a query whose signs all
    lie outside the band gets the oracle's distances and label."""
    say("plain fp32 workload", ct)
    d = dg.config_c1(1)
    F, D, K = d.F, d.D, d.K
    Pd = hdc.pad_cols(d.P)
    Xtr, Xte = hdc.pad_cols(d.X_train), hdc.pad_cols(d.X_test)
    # Error band of fp32 summation.  For E4M3 the band is empty: every E4M3
    # value is an integer multiple of 2^-9 below 2^9 in magnitude, so each
    # partial sum of 64 products is a multiple of 2^-9 below 2^24 units and
    # fp32 accumulation is exact in any order, ties (y = 0) included.
    gamma = 0.0 if ct == "fp8" else 2 * F * 2.0 ** -24 / (1 - F * 2.0 ** -24)
    exact = ct == "fp8"
    # training encode: band-exact against the exact (rounded-input) sign
    Htr = hdc.encode(Xtr, F, Pd, D, ct)
    Ytr, abtr = O.project(d.X_train, d.P, ct)
    sure_tr = np.ones(Ytr.shape, bool) if exact else np.abs(Ytr) > gamma * abtr[:, None]
    got_tr = bits(u64(Htr), D)
    assert np.array_equal(got_tr[sure_tr], (Ytr < 0)[sure_tr])
    # bundle of the GPU's training bits: integer, bit for bit
    ytr = torch.as_tensor(d.y_train).cuda()
    Cw, counts = hdc.bundle(Htr, D, ytr, K)
    Cref, cref = O.bundle(u64(Htr), d.y_train, K, D)
    torch.cuda.synchronize()
    assert np.array_equal(u64(Cw), Cref) and np.array_equal(counts.cpu().numpy(), cref)
    # fused classify: labels and distances
    lab, dists = hdc.classify(Xte, F, Pd, D, Cw, ct, with_dists=True)
    Hte = hdc.encode(Xte, F, Pd, D, ct)
    torch.cuda.synchronize()
    Yte, abte = O.project(d.X_test, d.P, ct)
    sure = np.ones(Yte.shape, bool) if exact else np.abs(Yte) > gamma * abte[:, None]
    got = bits(u64(Hte), D)
    assert np.array_equal(got[sure], (Yte < 0)[sure])
    # the fused kernel's distances are the Hamming distances of its own
    # encoding, which differs from the exact one only inside the band
    dref_exact = O.hamming(O.encode(d.X_test, d.P, ct), Cref, 0, D, 1)
    nband = (~sure).sum(1)
    dg_ = dists.cpu().numpy()
    assert np.all(np.abs(dg_ - dref_exact) <= nband[:, None])
    clean = nband == 0
    assert clean.mean() > 0.9
    lref, _ = O.argmin(dref_exact)
    assert np.array_equal(dg_[clean], dref_exact[clean])
    assert np.array_equal(lab.cpu().numpy()[clean], lref[clean])
    # unfused: the GPU encoding searched on the GPU equals the oracle's
    # search of the same bits
    lu, _, du = hdc.hamming_argmin(Hte, Cw, 0, D, 1, with_dists=True, nbits=D)
    torch.cuda.synchronize()
    assert np.array_equal(du.cpu().numpy(), O.hamming(u64(Hte), Cref, 0, D, 1))
    acc = float((lab.cpu().numpy() == d.y_test).mean())
    print("[c1] %s accuracy %.3f, in-band elements %d" % (ct, acc, int(nband.sum())), flush=True)
    if ct == "fp32":
        assert acc > 0.9


@pytest.fixture(scope="module")
def speech_batch(hdc):
    sp = dg.SpeechLike(2)
    ds = sp.dataset()
    Xq, yq = sp.queries(1 << 18, stream=10)
    Cw, _ = O.train(ds.X_train, ds.y_train, ds.P, ds.K)
    return ds, Xq, yq, Cw


@pytest.mark.parametrize("cfg", [(10240, 1, 0), (8192, 2, 0)], ids=str)
def test_headline_shape_every_tile_sampled(hdc, speech_batch, cfg):
    """617 features, 26 classes, D = 10240, a 2^18-query batch (the batch the
    benchmark times), every compiled tile variant of the bucket, on the +-1
    projection and on the shifted one; 2048 sampled rows (including the
    first and last tiles) against the oracle, labels and distances."""
    ds, Xq, yq, Cw = speech_batch
    d_trunc, stride, start = cfg
    F, D, K = ds.F, ds.D, ds.K
    n = Xq.shape[0]
    g = np.random.default_rng(31)
    rows = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n), g.choice(n, 1920, replace=False)]))
    lref, dref = O.classify(Xq[rows], ds.P, Cw, "int8", start, d_trunc, stride, with_dists=True)
    Xd, Pd = hdc.pad_cols(Xq), hdc.pad_cols(ds.P)
    Ps = hdc.shift_projection(Pd, F)
    Cd = torch.as_tensor(Cw.view(np.int64)).cuda()
    runs = [("int8", v, Pd) for v in hdc.tile_variants("classify", "int8", "int8", F, K)]
    runs += [("int8shift", v, Ps) for v in hdc.tile_variants("classify", "int8", "int8shift", F, K)]
    assert len(runs) >= 4
    for form, v, P_ in runs:
        say("headline shape", cfg, form, "variant", v)
        prep = hdc.Prepared(Cd, D, form, start, d_trunc, stride, tile=v)
        lab, dists = prep(Xd, F, P_, with_dists=True)
        torch.cuda.synchronize()
        assert np.array_equal(lab.cpu().numpy()[rows], lref), v
        assert np.array_equal(dists.cpu().numpy()[rows], dref), v
        # every row: the label is the first minimum of its distances
        dd = dists.cpu().numpy()
        assert np.array_equal(lab.cpu().numpy(), dd.argmin(1).astype(np.int32)), v
    del Xd


@pytest.fixture(scope="module")
def big_model(hdc):
    from paper_2606_26547_amd import serve
    src = dg.serving_models(5)[-1]
    assert (src.F, src.K, src.D) == (1024, 100, 16384)
    say("largest serving model: train")
    m = serve.ResidentModel(src.P, src.X_train, src.y_train, src.K)
    Cref, _ = O.train(src.X_train, src.y_train, src.P, src.K)
    torch.cuda.synchronize()
    return src, m, Cref


def test_largest_serving_model_bundle(big_model):
    src, m, Cref = big_model
    assert np.array_equal(u64(m.C), Cref)


@pytest.mark.parametrize("tuned", [None, (8192, 2, 0, "int8"), (16384, 1, 0, "fp8"), (12000, 3, 1, "bf16")],
                         ids=str)
def test_largest_serving_model(hdc, big_model, tuned):
    """The widest resident model of the serving mix: F = 1024, K = 100,
    D = 16384 (the bucket whose kernels spill registers), plain and under
    tuned configurations; labels and distances against the oracle."""
    src, m, Cref = big_model
    say("largest serving model", tuned)
    Xq, _ = src.queries(700, 901)
    cfg = tuned or (src.D, 1, 0, "int8")
    if tuned:
        m.set_tuned(tuned)
    prep = m.tuned if tuned else m.plain
    d, k, s, t = cfg
    lref, dref = O.classify(Xq, src.P, Cref, t, s, d, k, with_dists=True)
    lab, dists = prep(hdc.pad_cols(Xq), src.F, prep.P, with_dists=True)
    torch.cuda.synchronize()
    assert np.array_equal(dists.cpu().numpy(), dref)
    assert np.array_equal(lab.cpu().numpy(), lref)
