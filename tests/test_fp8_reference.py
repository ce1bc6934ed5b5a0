"""Pins of the fp8 reference quantiser (tests/fp8_reference.py) against the
OCP e4m3 ("fn") definition: representable values, ties to even, the
subnormal quantum, saturation, and the block scale rule."""
import numpy as np

from fp8_reference import round_e4m3, block_quantize, round_bf16


def all_e4m3_values():
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue                          # NaN encoding
            vals.append(m * 2.0 ** -9 if e == 0 else (1 + m / 8) * 2.0 ** (e - 7))
    return np.array(sorted(set(vals)))


def test_representable_values_are_fixed_points_and_the_largest_is_448():
    v = all_e4m3_values()
    assert v.max() == 448.0 and v[1] == 2.0 ** -9
    assert np.array_equal(round_e4m3(v), v)
    assert np.array_equal(round_e4m3(-v), -v)


def test_rounding_is_to_nearest_with_ties_to_even():
    v = all_e4m3_values()
    mid = (v[:-1] + v[1:]) / 2                    # exact ties
    r = round_e4m3(mid)
    # the even neighbour: mantissa bits of the chosen value end in 0
    for x, y in zip(mid, r):
        lo, hi = v[v < x].max(), v[v > x].min()
        assert y in (lo, hi)
        m = round(((y / 2.0 ** np.floor(np.log2(y))) - 1) * 8) if y >= 2.0 ** -6 else round(y / 2.0 ** -9)
        assert m % 2 == 0, (x, y)
    assert round_e4m3(np.array([17.0]))[0] == 16.0 and round_e4m3(np.array([19.0]))[0] == 20.0
    rng = np.random.default_rng(0)
    x = rng.uniform(-448, 448, 20000)
    r = round_e4m3(x)
    # nearest: no representable value is closer
    for xi, ri in zip(x[:300], r[:300]):
        assert np.abs(np.abs(v) - abs(xi)).min() == abs(abs(ri) - abs(xi))


def test_block_scale_maps_each_run_max_into_range_without_waste():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((7, 100)) * np.exp(rng.uniform(-20, 20, (7, 1)))
    Q = block_quantize(M)
    assert Q.shape == M.shape
    # relative error of the largest entry of each run <= half an e4m3 quantum (2^-4)
    P = np.zeros((7, 128)); P[:, :100] = M
    Pq = np.zeros((7, 128)); Pq[:, :100] = Q
    for r in range(7):
        for b in range(4):
            run, qrun = P[r, 32 * b:32 * b + 32], Pq[r, 32 * b:32 * b + 32]
            k = np.argmax(np.abs(run))
            if run[k] != 0:
                assert abs(qrun[k] - run[k]) <= 2.0 ** -4 * abs(run[k])
                # the scale is the smallest power of two that fits: max / 2^s in (224, 448]
                s = np.ceil(np.log2(abs(run[k]) / 448))
                assert 224 < abs(run[k]) / 2 ** s <= 448
    # exactly representable scaled data is unchanged
    E = np.array([[1.0, -0.5, 448.0 / 64, 0.0] * 8])
    assert np.array_equal(block_quantize(E), E)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    ulp = 2.0 ** -7
    assert round_bf16(np.array([one + ulp / 2]))[0] == one          # tie -> even (1.0)
    assert round_bf16(np.array([one + 1.5 * ulp]))[0] == one + 2 * ulp
    assert round_bf16(np.array([one + 0.6 * ulp]))[0] == one + ulp
