"""Pins of the oracle's FP8 e4m3 encoding against the format's definition:
closed-form code values, round trips, brute-force nearest values, tie and
saturation cases, and exact row norms."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import fp8


@pytest.mark.parametrize("code,value", [
    (0x00, 0.0), (0x01, 2.0 ** -9), (0x07, 7 * 2.0 ** -9), (0x08, 2.0 ** -6), (0x0F, 1.875 * 2.0 ** -6),
    (0x38, 1.0), (0x39, 1.125), (0x3F, 1.875), (0x40, 2.0), (0x77, 1.875 * 2.0 ** 7), (0x78, 256.0),
    (0x7E, 448.0), (0xB8, -1.0), (0xFE, -448.0), (0x81, -(2.0 ** -9)),
])
def test_decode_closed_forms(code, value):
    assert fp8.decode(code) == value


def test_decode_nan_codes_and_order():
    assert np.isnan(fp8.decode(0x7F)) and np.isnan(fp8.decode(0xFF))
    v = fp8.decode(np.arange(0x7F))
    assert np.all(np.diff(v) > 0)              # positive codes increase with value
    assert len(np.unique(np.abs(fp8.decode(np.arange(256))[~np.isnan(fp8.decode(np.arange(256)))]))) == 127


def test_round_trip_every_finite_code():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F and c != 0x80])
    assert np.array_equal(fp8.encode(fp8.decode(codes)), codes.astype(np.uint8))
    assert fp8.encode(-0.0) == 0x00


def test_ties_go_to_even_code_and_saturate():
    assert fp8.encode(1.0625) == 0x38          # halfway 1 .. 1.125
    assert fp8.encode(1.1875) == 0x3A          # halfway 1.125 .. 1.25 -> 1.25 (even)
    assert fp8.encode(0.5 * 2.0 ** -9) == 0x00  # halfway 0 .. 2^-9
    assert fp8.encode(-0.25 * 2.0 ** -9) == 0x80  # a negative value rounds to -0
    assert fp8.encode(1.5 * 2.0 ** -9) == 0x02  # halfway 2^-9 .. 2^-8
    assert fp8.encode(432.0) == 0x7E            # halfway 416 .. 448
    assert fp8.encode(1e6) == 0x7E and fp8.encode(-1e6) == 0xFE
    assert fp8.encode(460.0) == 0x7E


def test_encode_is_nearest_by_brute_force():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 30, 4000), rng.normal(0, 0.01, 2000), rng.uniform(-500, 500, 2000)])
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F])
    vals = fp8.decode(codes)
    got = fp8.decode(fp8.encode(x))
    best = np.abs(np.clip(x, -448, 448)[:, None] - vals[None, :]).min(axis=1)
    assert np.array_equal(np.abs(np.clip(x, -448, 448) - got), best)


def test_quantize_rows_scale_and_norm():
    rng = np.random.default_rng(4)
    A = rng.normal(0, 1, (6, 37)).astype(np.float32)
    A[2] = 0.0
    A[3, :] = np.float32(1e-30)
    Q, s, N = fp8.quantize_rows(A)
    assert s[2] == 1.0 and np.all(Q[2] == 0) and N[2] == 0.0
    for i in (0, 1, 3, 4, 5):
        k = np.argmax(np.abs(A[i]))
        assert abs(fp8.decode(Q[i, k])) == 448.0          # the largest entry maps to 448
        assert s[i] == np.float32(np.abs(A[i]).max() / np.float32(448.0))
        exact = sum(Fraction(float(v)) ** 2 for v in fp8.decode(Q[i])) * Fraction(float(s[i])) ** 2
        assert N[i] == float(exact)                        # one rounding of the exact value
    # relative error of the encoding: |q s - a| <= 2^-4 |a| for normal-range codes
    v = fp8.decode(Q) * s[:, None]
    big = np.abs(A / s[:, None]) >= 2.0 ** -6
    assert np.all(np.abs(v - A)[big] <= 2.0 ** -4 * np.abs(A)[big] * (1 + 1e-7))
