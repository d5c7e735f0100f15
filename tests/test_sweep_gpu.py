"""GPU parity of the persistent configuration sweep (hdc_eval_configs):
each slot's correct count equals the oracle's classification of that
configuration; duplicated slots agree; the one-launch sweep equals one
hdc_classify call per slot."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    assert torch.cuda.is_available()
    from paper_2606_26547_amd import hdc, tuner
    sp = dg.SpeechLike(2)
    ds = sp.dataset()
    Cref, _ = O.train(ds.X_train, ds.y_train, ds.P, ds.K)
    Xs, ys = sp.queries(2000, stream=4)
    return dict(hdc=hdc, tuner=tuner, ds=ds, C=Cref, Xs=Xs, ys=ys)


def test_sweep_grid_matches_oracle(env):
    hdc, ds = env["hdc"], env["ds"]
    print("[case] sweep grid vs oracle, 300 queries x 60 configs", flush=True)
    X, y = env["Xs"][:300], env["ys"][:300]
    grid = [(d, k, 0, t) for (d, k, t) in dg.sweep_grid()]
    res = hdc.eval_configs(hdc.pad_cols(X), ds.F, torch.as_tensor(y).cuda(), hdc.pad_cols(ds.P),
                           ds.D, torch.as_tensor(env["C"].view(np.int64)).cuda(), grid)
    ref = O.eval_configs(X, y, ds.P, env["C"], grid)
    assert np.array_equal(res["correct"], ref)
    assert (res["n"] == 300).all() and (res["device_us"] > 0).all()


def test_sweep_256_slots_consistent(env):
    hdc, ds = env["hdc"], env["ds"]
    print("[case] 256-slot sweep on 2000 queries", flush=True)
    slots = [(d, k, 0, t) for (d, k, t) in dg.sweep_slots(4)]
    Xd, yd = hdc.pad_cols(env["Xs"]), torch.as_tensor(env["ys"]).cuda()
    Pd, Cd = hdc.pad_cols(ds.P), torch.as_tensor(env["C"].view(np.int64)).cuda()
    c = hdc.eval_configs(Xd, ds.F, yd, Pd, ds.D, Cd, slots)["correct"]
    c2 = hdc.eval_configs(Xd, ds.F, yd, Pd, ds.D, Cd, slots)["correct"]
    c3 = hdc.eval_configs(Xd, ds.F, yd, Pd, ds.D, Cd, slots, max_workgroups=7)["correct"]   # few workers
    assert np.array_equal(c, c2)
    assert np.array_equal(c, c3)
    first = {}
    for s, v in zip(slots, c):
        assert first.setdefault(s, v) == v            # duplicates agree
    for s in sorted(first)[:60]:
        d, k, st, t = s
        lab = hdc.classify(Xd, ds.F, Pd, ds.D, Cd, t, st, d, k)
        assert int((lab == yd).sum().item()) == first[s], s
    # a few distinct slots against the oracle at full size
    for s in [(10240, 1, 0, "int8"), (4096, 2, 0, "fp8"), (1024, 8, 0, "bf16")]:
        ref = (O.classify(env["Xs"], ds.P, env["C"], s[3], s[2], s[0], s[1]) == env["ys"]).sum()
        lab = hdc.classify(Xd, ds.F, Pd, ds.D, Cd, s[3], s[2], s[0], s[1])
        assert int((lab == yd).sum().item()) == ref


def test_sweep_invalid_slots_do_no_work(env):
    hdc, ds = env["hdc"], env["ds"]
    X, y = env["Xs"][:100], env["ys"][:100]
    cfgs = [(99999, 1, 0, "int8"), (1024, 0, 0, "int8"), (1024, 1, 0, "fp32"), (1024, 1, 0, "int8")]
    res = hdc.eval_configs(hdc.pad_cols(X), ds.F, torch.as_tensor(y).cuda(), hdc.pad_cols(ds.P),
                           ds.D, torch.as_tensor(env["C"].view(np.int64)).cuda(), cfgs)
    c, t = res["correct"], res["device_us"]
    assert (c[:3] == 0).all() and (t[:3] == 0).all() and (res["n"][:3] == 0).all()
    assert res["n"][3] == 100
    assert c[3] == (O.classify(X, ds.P, env["C"], "int8", 0, 1024, 1) == y).sum()
