"""Host checks of integer arithmetic the kernels do in binary32 (no GPU).

The refined mask and combine find a fine point's coarse parent coordinate v / r as
trunc(fma(v, RN(1/r), RN(0.5/r))) in binary32 (csrc/combine.hip).  Exhaustively over every
fine coordinate a grid can have (v < 1024) and every ratio the library accepts
(1 <= r <= 1024), that equals the integer quotient; the fused multiply-add is emulated in
binary64, where the product of two binary32 values and the sum are exact before the one
rounding to binary32.
"""
import numpy as np


def test_parent_coordinate_by_reciprocal_is_exact():
    v = np.arange(1024, dtype=np.int64)
    for r in range(1, 1025):
        inv = np.float32(1.0) / np.float32(r)
        half = np.float32(np.float32(0.5) * inv)
        t = (v.astype(np.float64) * np.float64(inv) + np.float64(half)).astype(np.float32)
        q = np.trunc(t).astype(np.int64)
        assert np.array_equal(q, v // r), r
