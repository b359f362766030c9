"""Pins of the oracle's exact EUC_2D length c = nint(sqrt(D)) (Sec. 5.1:
TSPLIB coordinates; the length function is the TSPLIB EUC_2D rounding)."""
import math
import random
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import core


def test_isqrt_matches_library():
    rnd = random.Random(7)
    xs = list(range(0, 5000)) + [rnd.randrange(0, 1 << 62) for _ in range(3000)]
    xs += [k * k + d for k in (1 << 20, (1 << 31) - 1, 1 << 30) for d in (-1, 0, 1) if k * k + d < (1 << 62)]
    for x in xs:
        assert core.isqrt(x) == math.isqrt(x), x


def test_nint_defining_inequality_exhaustive_small():
    # k - 1/2 <= sqrt(D) < k + 1/2 is the definition of k = nint(sqrt(D));
    # squared (k >= 1): (2k-1)^2 <= 4D < (2k+1)^2.  No ties: 4D is even and
    # (2k+1)^2 is odd.
    for D in range(0, 200000):
        k = core.nint_sqrt(D)
        assert k >= 0
        assert (max(2 * k - 1, 0)) ** 2 <= 4 * D < (2 * k + 1) ** 2, D


def test_nint_rounding_boundaries():
    # sqrt(k^2 + k) < k + 1/2 < sqrt(k^2 + k + 1): closed form of the
    # rounding boundary, checked up to the largest length of a 2^20 span
    ks = list(range(0, 3000)) + list(range(1482900, 1482911)) + \
        random.Random(3).sample(range(3000, 1482911), 4000)
    for k in ks:
        assert core.nint_sqrt(k * k + k) == k
        assert core.nint_sqrt(k * k + k + 1) == k + 1
        assert core.nint_sqrt(k * k) == k


def test_nint_against_decimal_sqrt():
    getcontext().prec = 40
    rnd = random.Random(11)
    for _ in range(3000):
        D = rnd.randrange(0, 2 * (1 << 40))
        ref = int((Decimal(D).sqrt() + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR"))
        assert core.nint_sqrt(D) == ref


def test_cost_symmetric_and_translation_invariant():
    rnd = np.random.default_rng(5)
    xy = rnd.integers(0, 1 << 20, size=(50, 2)).astype(np.int32)
    sh = (xy + np.array([-123456, 654321])).astype(np.int32)
    for _ in range(200):
        u, v = rnd.integers(0, 50, 2)
        assert core.cost(xy, u, v) == core.cost(xy, v, u) == core.cost(sh, u, v)


def test_coordinate_range_check():
    ok = np.array([[0, 0], [(1 << 20) - 1, 5]], np.int32)
    bad = np.array([[0, 0], [1 << 20, 5]], np.int32)
    assert core.check_coords(ok) == 0
    assert core.check_coords(bad) == -2
