"""Pins of the oracle's ADC-chunked similarity (the reading of the
quantiser: clip to [floor, ceil], round to the nearest of 2^res levels
floor + step*j, half up; partial dot products over 128-dimension chunks).
Checked against closed forms, the unquantised dot product / Hamming
relation, brute force on small chunks, and the paper's reference
configuration (8-bit, step 1, window [-127, 128]), which is the identity on
every partial a 128-element chunk of +-1 products can take except -128."""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.fixture(scope="module", autouse=True)
def built():
    O.build()


def rand_hv(n, nbits, seed):
    g = np.random.default_rng(seed)
    W = (nbits + 63) // 64
    H = g.integers(0, 2 ** 63, size=(n, W), dtype=np.int64).view(np.uint64).copy()
    if nbits % 64:
        H[:, -1] &= np.uint64((1 << (nbits % 64)) - 1)
    return H


def test_quantiser_closed_forms():
    # reference configuration: identity on [-127, 128], -128 clips to -127
    for s in range(-128, 129):
        assert O.adc_quantize(s, 8, 1, -127, 128) == max(s, -127)
    # step 2 from floor -3: levels -3, -1, 1, 3, ...; ties round up
    assert [O.adc_quantize(s, 8, 2, -3, 128) for s in (-10, -3, -2, -1, 0, 1, 2)] == [-3, -3, -1, -1, 1, 1, 3]
    # 2-bit ADC: 4 levels floor, floor+step, ...; the top level caps
    assert [O.adc_quantize(s, 2, 10, 0, 100) for s in (0, 4, 5, 14, 15, 25, 30, 100)] == [0, 0, 10, 10, 20, 30, 30, 30]


def test_quantiser_properties():
    for res, step, fl, ce in [(8, 2, -3, 128), (6, 9, -3, 128), (4, 16, -127, 128), (3, 1, -2, 2)]:
        v = [O.adc_quantize(s, res, step, fl, ce) for s in range(-130, 131)]
        assert all(a <= b for a, b in zip(v, v[1:]))                       # monotone
        levels = sorted(set(v))
        assert len(levels) <= 2 ** res
        assert all((x - fl) % step == 0 for x in levels)                      # on the grid
        assert all(O.adc_quantize(x, res, step, fl, ce) == x for x in levels if x <= ce)   # idempotent


def test_reference_config_is_the_dot_product():
    Q = rand_hv(40, 1000, 1)
    Cw = rand_hv(7, 1000, 2)
    sc = O.adc_scores(Q, Cw, 0, 1000, 1, 8, 1, -127, 128)
    dist = O.hamming(Q, Cw, 0, 1000, 1)
    assert np.array_equal(sc, 1000 - 2 * dist)          # no chunk of random vectors reaches -128
    lab, _ = O.argmax(sc)
    ref, _ = O.argmin(dist)
    assert np.array_equal(lab, ref)


def test_chunk_partials_by_brute_force():
    Q = rand_hv(6, 300, 3)
    Cw = rand_hv(3, 300, 4)
    bq = 1 - 2 * np.unpackbits(Q.view(np.uint8), axis=1, bitorder="little")[:, :300].astype(np.int64)
    bc = 1 - 2 * np.unpackbits(Cw.view(np.uint8), axis=1, bitorder="little")[:, :300].astype(np.int64)
    for (s, e, k) in [(0, 300, 1), (5, 290, 3), (128, 256, 2)]:
        for (res, step, fl, ce) in [(8, 1, -127, 128), (5, 4, -3, 60), (2, 40, -64, 64)]:
            sc = O.adc_scores(Q, Cw, s, e, k, res, step, fl, ce)
            for i in range(6):
                for j in range(3):
                    tot = 0
                    for c in range(0, 300, 128):
                        dims = [d for d in range(c, min(c + 128, e)) if d >= s and (d - s) % k == 0]
                        if not dims:                     # chunks without a dimension of S are not converted
                            continue
                        part = int(sum(bq[i, d] * bc[j, d] for d in dims))
                        x = min(max(part, fl), ce)
                        code = min((2 * (x - fl) + step) // (2 * step), 2 ** res - 1)
                        tot += fl + step * code
                    assert sc[i, j] == tot


def test_argmax_first_maximum():
    lab, mx = O.argmax(np.array([[3, 5, 5], [-1, -1, -2]], dtype=np.int32))
    assert lab.tolist() == [1, 0] and mx.tolist() == [5, -1]
