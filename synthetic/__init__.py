"""Seeded synthetic inputs shared by the tests, the oracle and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
elliptic-curve or finite-field arithmetic of the method.  Every draw is
counter-based (SplitMix64 of a per-stream key plus a counter), so the value at
index i never depends on how many other values were drawn or on vectorisation.

SplitMix64 is the generator published by Steele, Lea and Flood ("Fast
splittable pseudorandom number generators", OOPSLA 2014): state advances by the
golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state passed
through the variant-13 finaliser (shifts 30/27/31, multipliers
0xBF58476D1CE4E5B9 and 0x94D049BB133111EB).

Layout conventions used by callers:
  * multi-word integers are little-endian arrays of uint64 limbs, one row per
    value, shape (n, limbs);
  * byte strings are uint8 arrays of shape (n, k).
"""

from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# stream tags: one per kind of draw, so that e.g. the scalars of a workload
# never coincide with the discrete logs of its bases
TAG_SCALARS = 1
TAG_BASE_DLOG = 2
TAG_SIZES = 3
TAG_HASH = 4
TAG_KEYS = 5
TAG_NONCES = 6
TAG_CORRUPT = 7
TAG_ARRIVALS = 8
TAG_EDGE = 9
TAG_MISC = 10


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _key(seed: int, tag: int) -> np.uint64:
    """Per-stream key: SplitMix64 output of (seed, tag) mixed twice."""
    s = np.array([(seed & _MASK64)], dtype=np.uint64)
    t = np.array([(tag & _MASK64)], dtype=np.uint64)
    with np.errstate(over="ignore"):
        k = _mix(_mix(s + _GAMMA) ^ _mix(t * _GAMMA + _GAMMA))
    return k[0]


def u64(seed: int, tag: int, n: int, offset: int = 0) -> np.ndarray:
    """n uint64 words: word j is SplitMix64 output number (offset + j) of the stream."""
    ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = _key(seed, tag) + ctr * _GAMMA
    return _mix(state)


def uniform_bits(seed: int, tag: int, n: int, bits: int, limbs: int | None = None,
                 offset: int = 0) -> np.ndarray:
    """n integers uniform in [0, 2**bits) as (n, limbs) uint64 little-endian rows."""
    words = (bits + 63) // 64
    if limbs is None:
        limbs = words
    if words > limbs:
        raise ValueError("bits do not fit in limbs")
    out = np.zeros((n, limbs), dtype=np.uint64)
    if n == 0 or bits == 0:
        return out
    raw = u64(seed, tag, n * words, offset * words).reshape(n, words)
    top = bits - 64 * (words - 1)
    if top < 64:
        raw[:, words - 1] &= np.uint64((1 << top) - 1)
    out[:, :words] = raw
    return out


def _rows_below(rows: np.ndarray, bound: int) -> np.ndarray:
    """Row-wise rows < bound for (n, limbs) little-endian uint64 rows."""
    n, limbs = rows.shape
    lt = np.zeros(n, dtype=bool)
    eq = np.ones(n, dtype=bool)
    if bound >> (64 * limbs):
        return np.ones(n, dtype=bool)
    for i in reversed(range(limbs)):
        bi = np.uint64((bound >> (64 * i)) & _MASK64)
        lt |= eq & (rows[:, i] < bi)
        eq &= rows[:, i] == bi
    return lt


def uniform_below(seed: int, tag: int, n: int, bound: int, limbs: int) -> np.ndarray:
    """n integers uniform in [0, bound) by rejection; attempt t of item j uses
    counter block t*n + j, so item j's value is independent of n's other items
    only through the attempt index."""
    if bound <= 0:
        raise ValueError("bound must be positive")
    bits = bound.bit_length()
    out = np.zeros((n, limbs), dtype=np.uint64)
    todo = np.arange(n)
    attempt = 0
    while todo.size:
        cand = uniform_bits(seed, tag, n, bits, limbs, offset=attempt * n)[todo]
        ok = _rows_below(cand, bound)
        out[todo[ok]] = cand[ok]
        todo = todo[~ok]
        attempt += 1
        if attempt > 200:
            raise RuntimeError("rejection sampling did not terminate")
    return out


def _rows_plus(rows: np.ndarray, value: int) -> np.ndarray:
    """Row-wise rows + value (value >= 0), raising if a sum does not fit."""
    n, limbs = rows.shape
    if value >> (64 * limbs):
        raise ValueError("value does not fit")
    out = rows.copy()
    carry = np.zeros(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for i in range(limbs):
            a = out[:, i]
            t = a + np.uint64((value >> (64 * i)) & _MASK64)
            c1 = t < a
            s = t + carry
            c2 = s < t
            out[:, i] = s
            carry = (c1 | c2).astype(np.uint64)
    if carry.any():
        raise ValueError("value does not fit")
    return out


def uniform_range(seed: int, tag: int, n: int, lo: int, hi: int, limbs: int) -> np.ndarray:
    """n integers uniform in [lo, hi) as (n, limbs) rows."""
    base = uniform_below(seed, tag, n, hi - lo, limbs)
    if lo == 0:
        return base
    return _rows_plus(base, lo)


def unit_doubles(seed: int, tag: int, n: int, offset: int = 0) -> np.ndarray:
    """n doubles uniform in [0, 1) from the top 53 bits of each word."""
    w = u64(seed, tag, n, offset)
    return (w >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def log_uniform_sizes(seed: int, tag: int, m: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    """m sizes round(2**U) with U uniform in [lo_exp, hi_exp]."""
    u = lo_exp + (hi_exp - lo_exp) * unit_doubles(seed, tag, m)
    return np.rint(np.exp2(u)).astype(np.int64)


def exponential_gaps(seed: int, tag: int, m: int, mean: float) -> np.ndarray:
    """m exponential inter-arrival gaps with the given mean (Poisson arrivals)."""
    u = unit_doubles(seed, tag, m)
    return -mean * np.log1p(-u)


def random_bytes(seed: int, tag: int, n: int, k: int) -> np.ndarray:
    """(n, k) uint8 array of uniform bytes."""
    words = (k + 7) // 8
    w = u64(seed, tag, n * words).reshape(n, words)
    return w.view(np.uint8).reshape(n, words * 8)[:, :k].copy()


def choice_indices(seed: int, tag: int, n: int, count: int) -> np.ndarray:
    """count distinct indices from [0, n), ordered by a seeded random key."""
    if count > n:
        raise ValueError("count > n")
    keys = u64(seed, tag, n)
    return np.sort(np.argsort(keys, kind="stable")[:count])


# ---- layout helpers (pure data marshalling) ---------------------------------

def limbs_to_int(row) -> int:
    v = 0
    for i, w in enumerate(row):
        v |= int(w) << (64 * i)
    return v


def ints_to_limbs(values, limbs: int) -> np.ndarray:
    vals = list(values)
    out = np.zeros((len(vals), limbs), dtype=np.uint64)
    for j, v in enumerate(vals):
        if v < 0 or v >> (64 * limbs):
            raise ValueError("value does not fit")
        for i in range(limbs):
            out[j, i] = (v >> (64 * i)) & _MASK64
    return out
