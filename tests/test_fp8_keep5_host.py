"""Host check of the reduced form in which the FP8 quantisation keeps a
column between reading it and knowing its scale (no GPU).

An FP32 value is cut to its sign, exponent, top 4 mantissa bits and one
sticky bit at bit 18 (set when any lower mantissa bit is).  Round-to-nearest-
even to E4M3 at a power-of-two scale 2^e must give the same code for the cut
value as for the full one at every e up to 116 whenever the scaled value lies
within +-448; above 116 an FP32 subnormal can land on a nonzero code, and
there the cut loses bits (which is why such columns are quantised again from
the full values).  The E4M3 rounding here is the oracle's, in FP64."""
from __future__ import annotations

import numpy as np

from oracle import rpid_oracle as O


def keep5(x32: np.ndarray) -> np.ndarray:
    b = x32.view(np.uint32)
    c = (b | ((b & np.uint32(0x3FFFF)) + np.uint32(0x3FFFF))) & np.uint32(0xFFFC0000)
    return c.view(np.float32)


def random_floats(rng, size):
    """FP32 bit patterns over every finite exponent, subnormals included, plus
    midpoints of E4M3 codes at random scales (ties once scaled back)."""
    bits = rng.integers(0, 0x7F800000, size=size, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32) * np.where(rng.random(size) < 0.5, -1, 1).astype(np.float32)
    t = O.e4m3_values()
    k = rng.integers(0, t.size - 1, size=size)
    mids = ((t[k] + t[k + 1]) / 2.0 * np.ldexp(1.0, -rng.integers(-20, 140, size=size))).astype(np.float32)
    return np.concatenate([x, mids])


def test_keep5_rounds_like_the_full_value_up_to_scale_116():
    rng = np.random.default_rng(23)
    x = random_floats(rng, 200_000)
    a = np.abs(x.astype(np.float64))
    cut = keep5(x).astype(np.float64)
    checked = 0
    for e in list(range(-40, 117, 3)) + [116]:
        sel = (a * 2.0**e <= 448.0) & (a > 0)
        full = O.e4m3_round(x[sel].astype(np.float64) * 2.0**e)
        short = O.e4m3_round(cut[sel] * 2.0**e)
        assert np.array_equal(full, short), e
        checked += int(np.count_nonzero(full))
    assert checked > 100_000  # most comparisons are of nonzero codes


def test_keep5_is_not_enough_for_subnormals_above_scale_116():
    """A subnormal with significant bits below the kept ones: 2^-140 (1 + 2^-3)
    rounds to a nonzero code at scale 2^136, the cut value to another."""
    x = np.array([2.0**-140 * (1 + 2.0**-3)], dtype=np.float32)
    e = 136
    full = O.e4m3_round(x.astype(np.float64) * 2.0**e)
    short = O.e4m3_round(keep5(x).astype(np.float64) * 2.0**e)
    assert full[0] != 0.0 and full[0] != short[0]


def test_keep5_keeps_non_finite_values():
    x = np.array([np.inf, -np.inf, np.nan], dtype=np.float32)
    y = keep5(x)
    assert np.isposinf(y[0]) and np.isneginf(y[1]) and np.isnan(y[2])
    # a NaN whose payload lies only in the low bits stays NaN through the sticky bit
    low_nan = np.array([0x7F800001], dtype=np.uint32).view(np.float32)
    assert np.isnan(keep5(low_nan)[0])
