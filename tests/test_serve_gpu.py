"""Serving on the GPU: resident models of different shapes, requests served
alone and in a concurrent mix must give identical labels (the int8 path is
exact, so bit for bit), equal to the oracle's; configuration jobs in the mix
equal a standalone sweep; a tight HBM budget still completes everything."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    from paper_2606_26547_amd import serve
    shapes = [(64, 2, 1024), (256, 26, 4096), (617, 26, 10240), (1024, 100, 16384)]
    srcs = [dg.ClusterModelData(F, K, D, seed=20 + i) for i, (F, K, D) in enumerate(shapes)]
    models = [serve.ResidentModel(s.P, s.X_train, s.y_train, s.K, tuned_cfg=(s.D // 2, 2, 0, "int8"))
              for s in srcs]
    torch.cuda.synchronize()
    return serve, srcs, models


def run_alone(serve, models, reqs):
    ex = serve.GpuExecutor(models)
    srv = serve.Server(ex, budget=1 << 34)
    out = []
    for r in reqs:
        out.append(srv.submit(r).result(timeout=60))     # one at a time
    srv.close()
    return out


def test_alone_equals_mix_and_oracle(setup):
    serve, srcs, models = setup
    print("[case] serving alone vs mix", flush=True)
    g = np.random.default_rng(0)
    reqs = []
    for i in range(24):
        m = i % len(models)
        n = int(g.integers(1, 700))
        X, _ = srcs[m].queries(n, 300 + i)
        reqs.append((m, X, bool(i % 3 == 0)))
    mk = lambda: [serve.Request(model=m, X=X, tuned=t) for (m, X, t) in reqs]   # noqa: E731
    alone = run_alone(serve, models, mk())
    ex = serve.GpuExecutor(models)
    srv = serve.Server(ex, budget=1 << 34, max_batch=2048)
    futs = [srv.submit(r) for r in mk()]                 # all at once: batched and overlapped
    mix = [f.result(timeout=120) for f in futs]
    srv.close()
    for a, b in zip(alone, mix):
        assert np.array_equal(a, b)
    # labels equal the oracle's for a sample of requests
    for idx in (0, 5, 10):
        m, X, t = reqs[idx]
        C = models[m].C.cpu().numpy().view(np.uint64)
        d, k, s, dt = models[m].tuned_cfg if t else (models[m].D, 1, 0, "int8")
        ref = O.classify(X, srcs[m].P, C, dt, s, d, k)
        assert np.array_equal(mix[idx], ref)


def test_config_jobs_in_mix_and_tight_budget(setup):
    serve, srcs, models = setup
    print("[case] serving configs + tight budget", flush=True)
    cfgs = [(models[2].D, 1, 0, "int8"), (4096, 2, 0, "fp8"), (2048, 1, 0, "bf16")]
    X, y = srcs[2].queries(512, 77)
    ex = serve.GpuExecutor(models)
    srv = serve.Server(ex, budget=3 * 1024 * 1024, max_batch=4096)      # a few requests at a time
    job = srv.submit(serve.Request(model=2, X=X, kind="configs", cfgs=cfgs, truth=y))
    infer = [srv.submit(serve.Request(model=i % 4, X=srcs[i % 4].queries(1000, 500 + i)[0]))
             for i in range(12)]
    got = job.result(timeout=120)
    for f in infer:
        f.result(timeout=120)
    srv.close()
    assert srv.sched.peak_used <= 3 * 1024 * 1024
    C = models[2].C.cpu().numpy().view(np.uint64)
    ref = O.eval_configs(X, y, srcs[2].P, C, cfgs)
    assert np.array_equal(got, ref)


def test_warm_with_tile_tuning_keeps_labels(setup):
    """Tuning the resident models' tiles at warm-up changes no label."""
    serve, srcs, models = setup
    print("[case] serving tile tuning", flush=True)
    from paper_2606_26547_amd import hdc
    reqs = [(m, srcs[m].queries(300, 700 + m)[0]) for m in range(len(models))]
    before = run_alone(serve, models, [serve.Request(model=m, X=X) for m, X in reqs])
    ex = serve.GpuExecutor(models)
    job = lambda i: [(models[i].D, 1, 0, "int8"), (models[i].D // 2, 2, 0, "fp8")]   # noqa: E731
    choices = ex.warm(job, tune_tiles=True)
    assert len(choices) == 2 * len(models)
    for c in choices:
        assert c.chosen in hdc.tile_variants(c.shape.kind, "int8", "int8", c.shape.F, c.shape.K)
    after = run_alone(serve, models, [serve.Request(model=m, X=X) for m, X in reqs])
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("cfg", [(10240, 1, 0, "int8"), (5120, 2, 0, "int8"), (10240, 1, 0, "fp8"),
                                 (4096, 2, 1, "fp8"), (8192, 2, 0, "bf16")], ids=str)
def test_resident_model_forms_against_oracle(setup, cfg):
    """The 617-feature model keeps shifted projections for int8 and E4M3:
    its prepared classifiers of those types read them (the others the +-1
    projection), and every configuration served through the executor gives
    the oracle's labels."""
    serve, srcs, models = setup
    print("[case] resident model forms", cfg, flush=True)
    src, m = srcs[2], models[2]
    assert set(m.shifted) == {"int8", "fp8"}
    m.set_tuned(cfg)
    d, k, s, t = cfg
    assert m.tuned.compute == {"int8": "int8shift", "fp8": "fp8shift"}.get(t, t)
    assert (m.tuned.P is m.shifted[t]) if t in m.shifted else (m.tuned.P is m.P)
    X, _ = src.queries(777, 55)
    ex = serve.GpuExecutor(models)
    srv = serve.Server(ex, budget=1 << 34)
    got = srv.submit(serve.Request(model=2, X=X, tuned=True)).result(timeout=60)
    srv.close()
    C = m.C.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, O.classify(X, src.P, C, t, s, d, k))
    m.set_tuned((src.D // 2, 2, 0, "int8"))
