"""GPU parity of the shared sweep path (tile HDC_TILE_SWEEP_SHARED): the
configurations of a compute type take their distances from one encoding of
the union of their dimension sets, by masked Hamming distance over chains
of prefix sets.  Every configuration's correct count must equal the
oracle's classification of that configuration, and the per-configuration
path's count, whatever the chain structure: unaligned starts, strides that
do not divide 64, ends inside one word, more ends per chain than one
search item holds, several query passes, ragged query counts, up to 128
classes, uint8 features."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg

pytestmark = pytest.mark.gpu

SHARED = 4


@pytest.fixture(scope="module")
def env():
    assert torch.cuda.is_available()
    from paper_2606_26547_amd import hdc
    sp = dg.SpeechLike(2)
    ds = sp.dataset()
    Cref, _ = O.train(ds.X_train, ds.y_train, ds.P, ds.K)
    Xs, ys = sp.queries(2000, stream=4)
    return dict(hdc=hdc, ds=ds, C=Cref, Xs=Xs, ys=ys)


def _run(hdc, X, F, y, P, D, C, cfgs, tile):
    return hdc.eval_configs(hdc.pad_cols(X), F, torch.as_tensor(y).cuda(), hdc.pad_cols(P), D,
                            torch.as_tensor(np.ascontiguousarray(C).view(np.int64)).cuda(), cfgs, tile=tile)


def test_shared_grid_matches_oracle(env):
    hdc, ds = env["hdc"], env["ds"]
    print("[case] shared sweep, 60-point grid, 300 queries", flush=True)
    X, y = env["Xs"][:300], env["ys"][:300]
    grid = [(d, k, 0, t) for (d, k, t) in dg.sweep_grid()]
    res = _run(hdc, X, ds.F, y, ds.P, ds.D, env["C"], grid, SHARED)
    ref = O.eval_configs(X, y, ds.P, env["C"], grid)
    assert np.array_equal(res["correct"], ref)
    assert (res["n"] == 300).all() and (res["device_us"] > 0).all()


def test_shared_256_slots_equal_per_config(env):
    hdc, ds = env["hdc"], env["ds"]
    print("[case] shared vs per-configuration sweep, 256 slots x 2000 queries", flush=True)
    slots = [(d, k, 0, t) for (d, k, t) in dg.sweep_slots(4)]
    a = _run(hdc, env["Xs"], ds.F, env["ys"], ds.P, ds.D, env["C"], slots, 0)["correct"]
    b = _run(hdc, env["Xs"], ds.F, env["ys"], ds.P, ds.D, env["C"], slots, SHARED)["correct"]
    assert np.array_equal(a, b)
    # mixed: every other configuration shared
    mixed = [s + ((SHARED if i % 2 else 0),) for i, s in enumerate(slots)]
    c = _run(hdc, env["Xs"], ds.F, env["ys"], ds.P, ds.D, env["C"], mixed, 0)["correct"]
    assert np.array_equal(a, c)
    for s in [(10240, 1, 0, "int8"), (4096, 2, 0, "fp8"), (1024, 8, 0, "bf16")]:
        ref = (O.classify(env["Xs"], ds.P, env["C"], s[3], s[2], s[0], s[1]) == env["ys"]).sum()
        assert b[slots.index(s)] == ref


CHAIN_CASES = [
    # (n, F, D, K, x dtype, seed)
    (300, 100, 1000, 40, np.int8, 1),
    (5000, 64, 700, 26, np.int8, 2),       # two query passes of 4096
    (63, 617, 2048, 128, np.int8, 3),
    (1, 300, 513, 7, np.uint8, 4),
    (129, 200, 4100, 100, np.uint8, 5),
]


@pytest.mark.parametrize("n,F,D,K,xdt,seed", CHAIN_CASES)
def test_shared_chains_match_oracle(env, n, F, D, K, xdt, seed):
    hdc = env["hdc"]
    print("[case] shared chains n=%d F=%d D=%d K=%d %s seed=%d" % (n, F, D, K, np.dtype(xdt).name, seed),
          flush=True)
    g = np.random.default_rng(seed)
    lo, hi = (-127, 128) if xdt == np.int8 else (0, 256)
    X = g.integers(lo, hi, size=(n, F)).astype(xdt)
    P = np.where(g.random((D, F)) < 0.5, -1, 1).astype(np.int8)
    C = g.integers(0, 1 << 63, size=(K, (D + 63) // 64), dtype=np.uint64)
    if D % 64:
        C[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    cfgs = []
    for t in ("int8", "bf16", "fp8"):
        # a chain of 20 ends (more than one search item holds), start 0, stride 1
        for e in np.linspace(8, D, 20).astype(int):
            cfgs.append((int(e), 1, 0, t))
        # unaligned starts, strides that do not divide 64, ends inside one word
        for s0, k in ((5, 3), (70, 5), (131, 7), (1, 64), (63, 100), (0, 2)):
            for e in sorted({s0 + 1, s0 + 2 * k + 1, (s0 + D) // 2, D - 1, D}):
                if e > s0:
                    cfgs.append((int(e), k, s0, t))
    truth = O.classify(X, P, C, "int8", 0, D, 1).astype(np.int32)
    truth[::3] = g.integers(0, K, size=truth[::3].shape)
    ref = O.eval_configs(X, truth, P, C, cfgs)
    res = _run(hdc, X, F, truth, P, D, C, cfgs, SHARED)
    assert np.array_equal(res["correct"], ref)
    assert (res["n"] == n).all()
    per = _run(hdc, X, F, truth, P, D, C, cfgs, 0)
    assert np.array_equal(per["correct"], ref)


def test_shared_invalid_configs_do_no_work(env):
    """Unsupported dtypes and empty or out-of-range sets report n = 0 and no
    time on the shared path too; the valid ones beside them are unaffected."""
    hdc, ds = env["hdc"], env["ds"]
    print("[case] shared sweep, invalid configurations", flush=True)
    X, y = env["Xs"][:100], env["ys"][:100]
    cfgs = [(99999, 1, 0, "int8"), (1024, 0, 0, "int8"), (1024, 1, 0, "fp32"), (1024, 1, 0, "int8"),
            (1024, 1, 1024, "bf16"), (2048, 3, 5, "fp8")]
    res = _run(hdc, X, ds.F, y, ds.P, ds.D, env["C"], cfgs, SHARED)
    c, t, n = res["correct"], res["device_us"], res["n"]
    assert (c[[0, 1, 2, 4]] == 0).all() and (t[[0, 1, 2, 4]] == 0).all() and (n[[0, 1, 2, 4]] == 0).all()
    assert n[3] == 100 and n[5] == 100
    assert c[3] == (O.classify(X, ds.P, env["C"], "int8", 0, 1024, 1) == y).sum()
    assert c[5] == (O.classify(X, ds.P, env["C"], "fp8", 5, 2048, 3) == y).sum()
