"""Pins of the 16-bit codec reference against the IEEE formats (known bit patterns, ties)."""
import numpy as np

from oracle import codec


def test_binary16_known_codes():
    v = np.array([0.0, 1.0, -2.0, 0.5, 65504.0, 1e6, -1e6, 2.0 ** -24])
    assert codec.encode_f16(v, 0.0, 1.0).tolist() == [0x0000, 0x3C00, 0xC000, 0x3800, 0x7BFF, 0x7BFF, 0xFBFF, 0x0001]


def test_binary16_round_to_nearest_even():
    # 1 + 2^-11 is halfway between 1 and 1 + 2^-10: ties to the even code 0x3C00
    assert codec.encode_f16(np.array([1.0 + 2.0 ** -11]), 0.0, 1.0).tolist() == [0x3C00]
    assert codec.encode_f16(np.array([1.0 + 3 * 2.0 ** -11]), 0.0, 1.0).tolist() == [0x3C02]


def test_bfloat16_known_codes_and_ties():
    v = np.array([1.0, -2.0, 3.140625, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])
    assert codec.encode_bf16(v, 0.0, 1.0).tolist() == [0x3F80, 0xC000, 0x4049, 0x3F80, 0x3F82]


def test_scale_and_reference_round_trip():
    rng = np.random.default_rng(0)
    ref, scale = 0.0555, 2.0 ** -12
    h = rng.integers(-2000, 2000, size=100).astype(np.float64)  # exactly representable codes
    v = ref + scale * h
    codes = codec.encode_f16(v, ref, scale)
    np.testing.assert_allclose(codec.decode_f16(codes, ref, scale), v.astype(np.float32), rtol=1e-6)
    np.testing.assert_array_equal(codes.view(np.float16).astype(np.float64), h)
