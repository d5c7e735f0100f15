"""Every tile variant of a bucket gives the oracle's result; the sweep's
work-item sizes agree; the autotuner picks a compiled variant."""
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


CASES = [
    # kind, x_type, compute, n, F, D, K
    ("classify", "int8", "int8", 300, 617, 2048, 26),
    ("classify", "int8", "int8", 200, 617, 1024, 100),
    ("classify", "uint8", "int8", 257, 512, 1024, 10),
    ("classify", "int8", "int8", 129, 300, 1000, 40),
    ("classify", "int8", "fp8", 129, 617, 1024, 26),
    ("encode", "int8", "int8", 300, 617, 2080, 1),
    ("encode", "uint8", "int8", 100, 100, 700, 1),
]


@pytest.mark.parametrize("case", CASES, ids=str)
def test_every_variant_matches_oracle(hdc, case):
    kind, xt, ct, n, F, D, K = case
    variants = hdc.tile_variants(kind, xt, ct, F, K)
    assert variants, case
    X, P = dg.random_case(n, F, D, xt, seed=n + F + D)
    g = np.random.default_rng(K)
    Cw = g.integers(0, 2 ** 63, size=(K, (D + 63) // 64), dtype=np.int64).view(np.uint64)
    if D % 64:
        Cw[:, -1] &= np.uint64((1 << (D % 64)) - 1)
    Xd, Pd = hdc.pad_cols(X), hdc.pad_cols(P)
    Cd = torch.as_tensor(Cw.view(np.int64)).cuda()
    if kind == "classify":
        lref, dref = O.classify(X, P, Cw, ct, with_dists=True)
    else:
        href = O.encode(X, P, ct)
    for v in variants:
        print("[case]", case, "variant", v, flush=True)
        if kind == "classify":
            lab, dists = hdc.classify(Xd, F, Pd, D, Cd, ct, with_dists=True, tile=v)
            torch.cuda.synchronize()
            assert np.array_equal(lab.cpu().numpy(), lref), v
            assert np.array_equal(dists.cpu().numpy(), dref), v
        else:
            H = hdc.encode(Xd, F, Pd, D, ct, tile=v)
            torch.cuda.synchronize()
            assert np.array_equal(H.cpu().numpy().view(np.uint64), href), v


@pytest.mark.parametrize("K,F,xt", [(26, 617, "int8"), (100, 617, "int8"), (26, 617, "uint8"), (10, 100, "int8")],
                         ids=str)
def test_sweep_item_sizes_agree_with_oracle(hdc, K, F, xt):
    """Work items of 128 and of 256 queries (int8 slots with two query tiles
    per wave) and the direct-staged bodies (int8 and E4M3 configurations,
    the latter on converted projection rows) give the oracle's correct
    counts for every slot."""
    n, D = 1000, 2048
    X, P = dg.random_case(n, F, D, xt, seed=K + F)
    g = np.random.default_rng(K + 1)
    Cw = g.integers(0, 2 ** 63, size=(K, D // 64), dtype=np.int64).view(np.uint64)
    truth = g.integers(0, K, size=n).astype(np.int32)
    cfgs = [(2048, 1, 0, "int8"), (1024, 2, 0, "int8"), (2048, 3, 1, "fp8"), (512, 1, 0, "bf16"),
            (2048, 4, 3, "int8"), (1536, 1, 0, "int8")]
    ref = O.eval_configs(X, truth, P, Cw, cfgs)
    Xd, Pd = hdc.pad_cols(X), hdc.pad_cols(P)
    Cd = torch.as_tensor(Cw.view(np.int64)).cuda()
    td = torch.as_tensor(truth).cuda()
    variants = hdc.tile_variants("sweep", xt, "int8", F, K)
    for v in variants:
        print("[case] sweep K", K, "F", F, xt, "variant", v, flush=True)
        res = hdc.eval_configs(Xd, F, td, Pd, D, Cd, cfgs, tile=v)
        assert np.array_equal(res["correct"], ref), v
        assert (res["n"] == n).all() and (res["device_us"] > 0).all()
    # a different work-item shape per configuration in one launch
    mixed = [c + (variants[i % len(variants)],) for i, c in enumerate(cfgs)]
    res = hdc.eval_configs(Xd, F, td, Pd, D, Cd, mixed)
    assert np.array_equal(res["correct"], ref)


def test_autotune_picks_a_compiled_variant(hdc, tmp_path):
    from paper_2606_26547_amd import autotune as AT
    shapes = [AT.Shape("classify", 617, 26, 2048, 8192), AT.Shape("encode", 617, 1, 2048, 8192),
              AT.Shape("sweep", 617, 26, 2048, 1000, cfgs=[(2048, 1, 0, "int8"), (1024, 2, 0, "fp8")])]
    choices = AT.autotune(shapes, reps=2)
    table = AT.TileTable.from_choices(choices)
    for c in choices:
        print("[case] autotune", c.shape.kind, c.chosen_name, c.variants, flush=True)
        assert c.chosen in hdc.tile_variants(c.shape.kind, "int8", "int8", c.shape.F, c.shape.K)
        assert table.get(c.shape.kind, "int8", "int8", c.shape.F, c.shape.K) == c.chosen
    path = str(tmp_path / "tiles.json")
    AT.save(choices, path)
    loaded = AT.load(path)
    assert len(loaded) == len(shapes)
    assert loaded.get("classify", "int8", "int8", 617, 26) == choices[0].chosen
    assert loaded.get("classify", "int8", "int8", 617, 40) == 0          # not tuned: built-in
