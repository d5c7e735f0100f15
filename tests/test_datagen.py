"""Synthetic inputs: shapes, determinism and the distributions each
workload is specified with."""
import numpy as np

from paper_2606_26547_amd import datagen as dg


def test_c1_shapes_and_determinism():
    a, b = dg.config_c1(1), dg.config_c1(1)
    assert a.X_train.shape == (1000, 64) and a.X_test.shape == (200, 64)
    assert a.X_train.dtype == np.float32 and a.P.shape == (2048, 64)
    assert np.array_equal(a.X_train, b.X_train) and np.array_equal(a.P, b.P)
    assert set(np.unique(a.P)) == {-1, 1}
    assert np.bincount(a.y_train).tolist() == [100] * 10


def test_c2_quantised_shapes():
    s = dg.SpeechLike(2)
    d = s.dataset()
    assert d.X_train.shape == (6238, 617) and d.X_test.shape == (1559, 617)
    assert d.X_train.dtype == np.int8 and d.P.shape == (10240, 617)
    assert np.abs(d.X_train.astype(int)).max() == 127
    assert d.X_train.min() >= -127
    q, y = s.queries(100, 7)
    assert q.shape == (100, 617) and q.dtype == np.int8 and y.max() < 26
    assert np.array_equal(q, s.queries(100, 7)[0])


def test_c3_sparsity_and_range():
    im = dg.ImageLike(3)
    X, y = im.queries(2000, 1)
    assert X.dtype == np.uint8 and X.shape == (2000, 784)
    zero = (X == 0).mean()
    assert 0.75 < zero < 0.85
    assert X[X > 0].min() >= 1 and X.max() == 255
    assert 0.25 < im.masks.mean() < 0.40


def test_sweep_slots():
    slots = dg.sweep_slots(4)
    assert len(slots) == 256 and len(set(slots)) <= 60
    assert all(s in dg.sweep_grid() for s in slots)
    assert slots == dg.sweep_slots(4)


def test_serving_models_shapes():
    ms = dg.serving_models(5)
    assert [(m.F, m.K, m.D) for m in ms] == dg.SERVING_SHAPES
    q, y = ms[0].queries(10, 0)
    assert q.shape == (10, 64) and q.dtype == np.int8
