"""Pins for the windowing definition used to check the bucket grouping."""

import random

import pytest

from oracle import ref


@pytest.mark.parametrize("c", [2, 3, 5, 8, 13, 16, 20])
def test_signed_digits_reconstruct_scalar(c):
    rnd = random.Random(c)
    bits = 255
    W = (bits + 1 + c - 1) // c
    for s in [0, 1, (1 << bits) - 1, 1 << (bits - 1), (1 << c) - 1, 1 << (c - 1), (1 << (c - 1)) + 1] + \
            [rnd.getrandbits(bits) for _ in range(200)]:
        d = ref.signed_digits(s, c, W)
        assert len(d) == W
        assert all(-(1 << (c - 1)) <= x <= (1 << (c - 1)) for x in d)
        assert sum(x << (c * w) for w, x in enumerate(d)) == s


def test_signed_digits_need_enough_windows():
    with pytest.raises(ValueError):
        ref.signed_digits((1 << 16) - 1, 8, 1)


def test_bucket_lists_weighting_matches_msm_identity():
    """sum over buckets of |d| (+/-) 2^(cw) reproduces every scalar."""
    rnd = random.Random(3)
    c, bits = 5, 30
    W = (bits + 1 + c - 1) // c
    scalars = [rnd.getrandbits(bits) for _ in range(40)]
    lists = ref.bucket_lists(scalars, c, W)
    D = 1 << (c - 1)
    rebuilt = [0] * len(scalars)
    for b, entries in lists.items():
        w, mag = b // D, b % D + 1
        for i, neg in entries:
            rebuilt[i] += (-mag if neg else mag) << (c * w)
    assert rebuilt == scalars
