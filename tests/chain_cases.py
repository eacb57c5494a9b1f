"""Inputs whose exact sums make carries or borrows run through many 32-bit
digits of the small superaccumulator (shared by the GPU parity tests)."""
import math

import numpy as np


def long_chain_cases():
    """After two parallel carry steps some digit of these sums still sits on a
    bound (-1 or 2^32), so the rounding takes its serial route."""
    p = math.ldexp
    cases = [
        [p(1, 1000), -p(1, -1000)],
        [-p(1, 1000), p(1, -1000)],
        [p(1, 1023), -p(1, -1074)],
        [-p(1, -1074), -p(1, 1023)],
        [1.0, -p(1, -1074)],
        [-1.0, p(1, -1074), p(1, -1074)],
        [p(1, 600)] + [-p(1, -900)] * 3,
    ]
    # digits of exactly 2^32 - 1 with a carry into the bottom one
    up = [p(2.0 ** 32 - 1, 32 * i - 1075) for i in range(3, 40)] + [p(1, 32 * 3 - 1075)]
    cases.append(up)
    cases.append([-v for v in up])
    return [np.array(c, dtype=np.float64) for c in cases]
