"""Pins of oracle.lowprec (the dense formats of the shared-Phi solve)
against the format definitions and against torch's own casts."""

import numpy as np
import pytest

from oracle import lowprec as lp

torch = pytest.importorskip("torch")


def test_e4m3_value_set_from_the_definition():
    v = lp.e4m3_values()
    pos = v[v > 0]
    assert pos.max() == 448.0 and pos.min() == 2.0 ** -9
    assert len(v) == 253  # 126 positive, 126 negative, and one zero (+0 and -0)
    # every representable value maps to itself
    np.testing.assert_array_equal(lp.round_to(v, "e4m3"), v)


def test_e4m3_midpoints_round_to_even():
    v = lp.e4m3_values()
    pos = v[v >= 0]
    mids = (pos[:-1] + pos[1:]) / 2
    got = lp.round_to(mids, "e4m3")
    for m, lo, hi, g in zip(mids, pos[:-1], pos[1:], got):
        assert g in (lo, hi)
        # the even neighbour: significand field ends in 0
        even = lo if _e4m3_mant(lo) % 2 == 0 else hi
        assert g == even, (m, lo, hi, g)


def _e4m3_mant(x):
    if x == 0:
        return 0
    e = max(int(np.floor(np.log2(x))), -6)
    return int(round(x / 2.0 ** (e - 3))) & 7


def test_e4m3_matches_torch_cast():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 4000),
                        rng.standard_normal(4000) * 2.0 ** rng.integers(-12, 8, 4000),
                        [0.0, 448.0, -448.0, 460.0, 2.0 ** -10, 3 * 2.0 ** -10, 2.0 ** -7 * 1.0625]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(lp.round_to(x32.astype(np.float64), "e4m3"), want)


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.standard_normal(20000) * 2.0 ** rng.integers(-140, 120, 20000),
                        [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0, 2.0 ** -133]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(lp.round_to(x32.astype(np.float64), "bf16"), want)


def test_bf16_from_fp64_is_single_rounding():
    # 1 + 2^-8 + 2^-30 is above the bf16 midpoint 1 + 2^-8 and must round up;
    # going through FP32 first would land exactly on the midpoint and round
    # down to 1.
    x = 1 + 2.0 ** -8 + 2.0 ** -30
    assert lp.round_to(np.array([x]), "bf16")[0] == 1 + 2.0 ** -7


@pytest.mark.parametrize("fmt,top", [("bf16", 1.0), ("e4m3", 448.0)])
def test_row_scale_is_the_smallest_fitting_power_of_two(fmt, top):
    rng = np.random.default_rng(3)
    phi = rng.standard_normal((50, 40)) * 2.0 ** rng.integers(-20, 20, (50, 1))
    phi[7] = 0.0
    phi[8, 3] = top * 2.0 ** 5  # an exact boundary: fits with e = 5
    e = lp.row_exponents(phi, fmt)
    mx = np.abs(phi).max(axis=1)
    for i in range(50):
        if mx[i] == 0:
            assert e[i] == 0
            continue
        assert mx[i] / 2.0 ** e[i] <= top < mx[i] / 2.0 ** (e[i] - 1)
    assert e[8] == 5


@pytest.mark.parametrize("fmt", lp.FORMATS)
def test_store_matrix_error_within_half_a_unit(fmt):
    rng = np.random.default_rng(4)
    phi = (rng.standard_normal((64, 96)) / 8).astype(np.float32)
    st, e, a = lp.store_matrix(phi, fmt)
    np.testing.assert_array_equal(a, st * np.ldexp(1.0, e)[:, None])
    rel = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "e4m3": 2.0 ** -4}[fmt]
    err = np.abs(a - phi.astype(np.float64))
    # relative to each entry, or to the subnormal spacing near zero
    floor = {"f32": 0.0, "bf16": 0.0, "e4m3": 2.0 ** -10}[fmt] * np.ldexp(1.0, e)[:, None]
    assert np.all(err <= rel * np.abs(phi) + floor)
    if fmt == "e4m3":
        np.testing.assert_array_equal(np.isin(st, lp.e4m3_values()), True)


def test_e4m3_decode_matches_torch_bit_patterns():
    b = np.arange(256, dtype=np.uint8)
    want = torch.from_numpy(b).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = lp.e4m3_decode(b)
    fin = ~np.isnan(want)
    assert np.array_equal(np.isnan(got), ~fin)
    np.testing.assert_array_equal(got[fin], want[fin])
