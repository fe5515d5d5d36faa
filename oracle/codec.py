"""Reference of the 16-bit deviation codec (test infrastructure).

A value v is coded as follows: the deviation v - ref is formed in binary64 and rounded to
binary32 (round to nearest even), multiplied by the power of two 1/scale (exact), and rounded to
IEEE binary16 (numpy's float16 cast, round to nearest even, saturated at +-65504) or to bfloat16
(the upper 16 bits of the binary32 value after round to nearest even on the dropped bits).  It
decodes as ref + scale * h.  Written from the IEEE 754 formats.
"""
import numpy as np


def _deviation32(v, ref, scale):
    d = (np.asarray(v, dtype=np.float64) - np.float64(ref)).astype(np.float32)
    return d * np.float32(1.0 / scale)


def encode_f16(v, ref, scale):
    h = _deviation32(v, ref, scale)
    h = np.clip(h, -65504.0, 65504.0)
    return h.astype(np.float16).view(np.uint16)


def decode_f16(codes, ref, scale):
    return np.float32(ref) + np.float32(scale) * codes.view(np.float16).astype(np.float32)


def encode_bf16(v, ref, scale):
    h = _deviation32(v, ref, scale)
    u = h.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFFFFFF
    return (u >> 16).astype(np.uint16)


def decode_bf16(codes, ref, scale):
    f = (codes.astype(np.uint32) << 16).view(np.float32)
    return np.float32(ref) + np.float32(scale) * f
