"""Helpers shared by the tests: seeded workloads, conversions, oracle calls."""

from __future__ import annotations

import functools
import os

import numpy as np

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves, ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CURVE_BY_ID = curves.BY_ID


def rows_to_points(c, rows, inf=None):
    pts = []
    for i, row in enumerate(np.asarray(rows).reshape(-1, 2 * c.limbs)):
        x = syn.limbs_to_int(row[: c.limbs])
        y = syn.limbs_to_int(row[c.limbs:])
        if (inf is not None and inf[i]) or (x == 0 and y == 0):
            pts.append(None)
        else:
            pts.append((x, y))
    return pts


def points_to_rows(c, pts):
    out = np.zeros((len(pts), 2 * c.limbs), dtype=np.uint64)
    for i, P in enumerate(pts):
        if P is not None:
            out[i, : c.limbs] = syn.ints_to_limbs([P[0]], c.limbs)[0]
            out[i, c.limbs:] = syn.ints_to_limbs([P[1]], c.limbs)[0]
    return out


@functools.lru_cache(maxsize=16)
def seeded_bases(curve_name: str, n: int, seed: int):
    """(k, bases): k_i uniform in [1, r) from the seed, bases P_i = k_i G from the C oracle."""
    c = curves.CURVES[curve_name]
    k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, n, 1, c.r, 4)
    bases = co.fixed_base(c.cid, c.limbs, k)
    return k, bases


def seeded_scalars(curve_name: str, n: int, seed: int, kind: str = "mod_r"):
    c = curves.CURVES[curve_name]
    if kind == "mod_r":
        return syn.uniform_below(seed, syn.TAG_SCALARS, n, c.r, 4)
    if kind == "bits":
        return syn.uniform_bits(seed, syn.TAG_SCALARS, n, c.scalar_bits, 4)
    raise ValueError(kind)


def oracle_msm(c, bases, scalars, threads=None):
    out, inf = co.msm(c.cid, c.limbs, bases, scalars, threads=threads)
    return None if inf else (syn.limbs_to_int(out[: c.limbs]), syn.limbs_to_int(out[c.limbs:]))


def dlog_msm_expected(c, ks, scalars):
    """sum_i s_i (k_i G) = (sum_i s_i k_i mod r) G."""
    e = 0
    for kr, sr in zip(ks, scalars):
        e += syn.limbs_to_int(kr) * syn.limbs_to_int(sr)
    e %= c.r
    return ref.scalar_mul(c, e, ref.generator(c))


def limbs_to_objects(a: np.ndarray) -> np.ndarray:
    """Rows of u64 little-endian limbs -> a numpy array of Python integers."""
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(a.shape[0], -1)
    out = a[:, 0].astype(object)
    for j in range(1, a.shape[1]):
        out = out + (a[:, j].astype(object) << (64 * j))
    return out


def dlog_batch_expected(c, k: np.ndarray, s: np.ndarray, offs: np.ndarray) -> np.ndarray:
    """Rows (u64[m, 2L], zeros for O) of (sum over MSM j of s_i k_i mod r) G for
    every MSM j of a batch with bases k_i G: the products are summed in Python
    integers per MSM, then the C oracle multiplies G by each exponent."""
    offs = np.asarray(offs, dtype=np.int64)
    m = len(offs) - 1
    prod = limbs_to_objects(k) * limbs_to_objects(s)
    e = np.zeros(m, dtype=object)
    nonempty = offs[1:] > offs[:-1]
    if nonempty.any():
        sums = np.add.reduceat(prod, offs[:-1][nonempty])
        e[nonempty] = sums
    e = [int(x) % c.r for x in e]
    ex = syn.ints_to_limbs(e, 4)
    return co.fixed_base(c.cid, c.limbs, ex)


def seeded_signatures(m: int, seed: int, corrupt_every: int = 16, c=curves.SECP256R1):
    """m verification requests on curve c (secp256r1 or SM2): seeded keys d_i,
    32-byte random hashes, signatures made by the oracle (nonces from the
    seed); every corrupt_every-th request is corrupted (hash bit, r, s or key).
    Returns (hashes u8[m,32], pubkeys u64[m,8], sigs u64[m,8])."""
    n = c.r
    d = syn.uniform_range(seed, syn.TAG_KEYS, m, 1, n, 4)
    k = syn.uniform_range(seed, syn.TAG_NONCES, m, 1, n, 4)
    hashes = syn.random_bytes(seed, syn.TAG_HASH, m, 32)
    Q = co.fixed_base(c.cid, c.limbs, d)
    R = co.fixed_base(c.cid, c.limbs, k)
    sigs = np.zeros((m, 8), dtype=np.uint64)
    for i in range(m):
        di, ki = syn.limbs_to_int(d[i]), syn.limbs_to_int(k[i])
        r = syn.limbs_to_int(R[i, :4]) % n
        e = int.from_bytes(bytes(hashes[i]), "big")
        s = pow(ki, -1, n) * (e + r * di) % n
        if r == 0 or s == 0:  # probability ~2^-256; keep the request, it is simply invalid
            pass
        sigs[i, :4] = syn.ints_to_limbs([r], 4)[0]
        sigs[i, 4:] = syn.ints_to_limbs([s], 4)[0]
    pub = Q.copy()
    if corrupt_every:
        sel = syn.u64(seed, syn.TAG_CORRUPT, m)
        for i in range(0, m, corrupt_every):
            kind = int(sel[i] % 4)
            if kind == 0:
                hashes[i, int(sel[i] >> 8) % 32] ^= np.uint8(1 << int((sel[i] >> 16) % 8))
            elif kind == 1:
                r = (syn.limbs_to_int(sigs[i, :4]) + 1) % n
                sigs[i, :4] = syn.ints_to_limbs([r], 4)[0]
            elif kind == 2:
                s = syn.limbs_to_int(sigs[i, 4:]) * 2 % n
                sigs[i, 4:] = syn.ints_to_limbs([s], 4)[0]
            else:
                pub[i] = Q[(i + 1) % m]
    return hashes, pub, sigs
