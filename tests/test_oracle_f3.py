"""Pins for the oracle's encode-side perforation and Level-ID encoding,
against brute force from the definitions, closed forms and invariants."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2606_26547_amd import datagen as dg


def _bits(H, nbits):
    return np.unpackbits(H.view(np.uint8), axis=1, bitorder="little")[:, :nbits]


# --------------------------------------------------------- feature perforation
@pytest.mark.parametrize("fperf", [(0, 13, 1), (1, 13, 2), (0, 13, 3), (5, 11, 4), (12, 13, 1)])
def test_fperf_brute_force_int8(fperf):
    """Exact integer sum over S_F, rescaled by F/|S_F| (a positive rational),
    sign with zero -> +1, written out with Python integers and fractions."""
    fs, fe, fk = fperf
    g = np.random.default_rng(3)
    n, F, D = 6, 13, 70
    X = g.integers(-3, 4, size=(n, F), dtype=np.int8)          # small values: many zero sums
    P = (1 - 2 * g.integers(0, 2, size=(D, F))).astype(np.int8)
    H = O.encode_fperf(X, P, fs, fe, fk)
    SF = list(range(fs, fe, fk))
    want = np.zeros((n, D), dtype=np.uint8)
    for i in range(n):
        for d in range(D):
            y = Fraction(F, len(SF)) * sum(int(X[i, f]) * int(P[d, f]) for f in SF)
            want[i, d] = 1 if y < 0 else 0
    assert np.array_equal(_bits(H, D), want)


def test_fperf_brute_force_fp32():
    """Float features: the exact rational sum decides the sign."""
    g = np.random.default_rng(4)
    n, F, D = 5, 9, 40
    X = (g.standard_normal((n, F)) * 3).astype(np.float32)
    X[0, :] = np.float32(0.5)                                  # cancelling sums -> 0 -> +1
    P = (1 - 2 * g.integers(0, 2, size=(D, F))).astype(np.int8)
    H = O.encode_fperf(X, P, 1, 9, 2, compute="fp32")
    want = np.zeros((n, D), dtype=np.uint8)
    for i in range(n):
        for d in range(D):
            y = sum(Fraction(float(X[i, f])) * int(P[d, f]) for f in range(1, 9, 2))
            want[i, d] = 1 if Fraction(F, 4) * y < 0 else 0
    assert np.array_equal(_bits(H, D), want)


def test_fperf_stride_one_is_plain_encoding():
    g = np.random.default_rng(5)
    X = g.integers(-127, 128, size=(40, 100), dtype=np.int8)
    P = dg.projection_matrix(300, 100, 5)
    assert np.array_equal(O.encode_fperf(X, P, 0, 100, 1), O.encode(X, P))
    assert np.array_equal(O.encode_fperf(X, P, 0, 100, 1, start=3, end=290, stride=3),
                          O.encode(X, P, start=3, end=290, stride=3))


@pytest.mark.parametrize("compute", ["int8", "bf16", "fp8"])
def test_fperf_equals_encoding_of_gathered_columns(compute):
    """Perforating the reduction over features is encoding the gathered
    feature columns (the rescale never changes a sign)."""
    g = np.random.default_rng(6)
    X = g.integers(-127, 128, size=(30, 97), dtype=np.int8)
    P = dg.projection_matrix(256, 97, 6)
    for fs, fe, fk in [(0, 97, 2), (3, 90, 5), (96, 97, 1)]:
        cols = np.arange(fs, fe, fk)
        assert np.array_equal(O.encode_fperf(X, P, fs, fe, fk, compute=compute),
                              O.encode(np.ascontiguousarray(X[:, cols]), np.ascontiguousarray(P[:, cols]),
                                       compute=compute))


# --------------------------------------------------------------- level quantiser
def test_level_quantize_hand_cases():
    """lo = 0, hi = 1, L = 4: levels are [0, 1/4) -> 0, [1/4, 1/2) -> 1, ...,
    everything at or above 3/4 (including past hi) -> 3; below lo and NaN ->
    0; a feature with hi == lo -> 0."""
    X = np.array([[0.0, 0.2499, 0.25, 0.5, 0.74, 0.75, 1.0, 2.0, -1.0, np.nan, 0.3]], dtype=np.float32)
    F = X.shape[1]
    lo = np.zeros(F, dtype=np.float32)
    hi = np.ones(F, dtype=np.float32)
    hi[-1] = 0.0                                               # empty range
    lev = O.level_quantize(X, lo, hi, 4)
    assert lev.tolist() == [[0, 0, 1, 2, 2, 3, 3, 3, 0, 0, 0]]


def test_level_quantize_integer_grid_and_monotone():
    """Range [0, L] with L levels: x in [k, k+1) is level k (all values
    dyadic, so every step is exact); levels never decrease with x."""
    L = 37
    x = np.arange(0, L, 0.5, dtype=np.float32)
    X = x[:, None].copy()
    lev = O.level_quantize(X, np.zeros(1, np.float32), np.full(1, L, np.float32), L)[:, 0]
    assert np.array_equal(lev, np.minimum(np.floor(x), L - 1).astype(np.uint16))
    g = np.random.default_rng(7)
    xs = np.sort(g.uniform(-2, 7, size=5000).astype(np.float32))
    lv = O.level_quantize(xs[:, None].copy(), np.full(1, -1.5, np.float32), np.full(1, 6.25, np.float32), 128)[:, 0]
    assert (np.diff(lv.astype(np.int64)) >= 0).all() and lv[0] == 0 and lv[-1] == 127


def test_level_quantize_one_level():
    X = np.random.default_rng(8).standard_normal((4, 6)).astype(np.float32)
    assert (O.level_quantize(X, X.min(0), X.max(0), 1) == 0).all()


# --------------------------------------------------------------- Level-ID encode
def test_level_id_brute_force():
    g = np.random.default_rng(9)
    n, F, L, D = 4, 5, 6, 70
    ID = dg.id_hypervectors(F, D, 9)
    LV = dg.level_hypervectors(L, D, 9)
    lev = g.integers(0, L, size=(n, F)).astype(np.uint16)
    H = O.level_id_encode(lev, ID, LV, D)
    idb, lvb = _bits(ID, D), _bits(LV, D)
    want = np.zeros((n, D), dtype=np.uint8)
    for i in range(n):
        for d in range(D):
            s = 0
            for f in range(F):
                a = -1 if idb[f, d] else 1
                b = -1 if lvb[lev[i, f], d] else 1
                s += a * b
            want[i, d] = 1 if s < 0 else 0
    assert np.array_equal(_bits(H, D), want)
    assert (H[:, -1] >> np.uint64(D % 64) == 0).all()          # pad bits clear


def test_level_id_single_feature_is_xor():
    """F = 1: the bound pair itself, ID xor LV of the row's level."""
    D, L = 200, 8
    ID = dg.id_hypervectors(1, D, 10)
    LV = dg.level_hypervectors(L, D, 10)
    lev = np.arange(L, dtype=np.uint16)[:, None].copy()
    H = O.level_id_encode(lev, ID, LV, D)
    assert np.array_equal(H, ID[0][None, :] ^ LV)


def test_level_id_matching_identity_gives_all_plus_one():
    """Every ID equal to its row's level vector: every product is +1."""
    D, L, F = 130, 5, 7
    LV = dg.level_hypervectors(L, D, 11)
    lev = np.array([[f % L for f in range(F)]], dtype=np.uint16)
    ID = LV[lev[0]].copy()
    assert not O.level_id_encode(lev, ID, LV, D).any()


def test_level_id_flip_invariance_and_tie():
    """Odd F (no ties): negating dimension d of every ID negates bit d of
    every row.  Even F with a cancelling pair gives +1 (bit 0)."""
    g = np.random.default_rng(12)
    D, L, F = 190, 9, 11
    ID = dg.id_hypervectors(F, D, 12)
    LV = dg.level_hypervectors(L, D, 12)
    lev = g.integers(0, L, size=(20, F)).astype(np.uint16)
    mask = dg.pack_bits(g.integers(0, 2, size=(1, D), dtype=np.uint8))
    assert np.array_equal(O.level_id_encode(lev, ID ^ mask, LV, D), O.level_id_encode(lev, ID, LV, D) ^ mask)
    ID2 = np.stack([LV[0], LV[0] ^ dg.pack_bits(np.ones((1, D), np.uint8))[0]])
    assert not O.level_id_encode(np.zeros((1, 2), np.uint16), ID2, LV, D).any()


def test_level_hypervector_distances():
    """Level l differs from level 0 in floor(l * (D/2) / (L-1)) positions."""
    D, L = 1000, 11
    LV = _bits(dg.level_hypervectors(L, D, 13), D)
    for l in range(L):
        assert int((LV[l] != LV[0]).sum()) == (l * (D // 2)) // (L - 1)
