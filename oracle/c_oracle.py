"""ctypes wrapper of the C oracle (oracle/c/ecc_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays are numpy
uint64 with canonical affine coordinates, L limbs for x then L for y per point,
(0, 0) meaning the point at infinity; scalars are 4 little-endian u64 limbs.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "ecc_oracle.c")
LIB = os.path.join(HERE, "c", "libecc_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/c/libecc_oracle.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wno-unused-function", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        sz = ctypes.c_size_t
        ci = ctypes.c_int
        L.orc_curve_limbs.argtypes = [ci]
        L.orc_fp_mul.argtypes = [ci, u64p, u64p, u64p, sz]
        L.orc_fp_inv.argtypes = [ci, u64p, u64p, sz]
        L.orc_on_curve.argtypes = [ci, u64p, sz, u8p]
        L.orc_add.argtypes = [ci, u64p, u64p, sz, u64p, u8p]
        L.orc_scalar_mul.argtypes = [ci, u64p, u64p, sz, u64p, u8p]
        L.orc_msm.argtypes = [ci, u64p, u64p, sz, ci, u64p, u8p]
        L.orc_msm_batch.argtypes = [ci, u64p, u64p, u64p, sz, ci, u64p, u8p]
        L.orc_fixed_base.argtypes = [ci, u64p, sz, ci, u64p]
        L.orc_ecdsa_verify.argtypes = [ci, u8p, u64p, u64p, sz, u8p]
        for f in ("orc_curve_limbs", "orc_fp_mul", "orc_fp_inv", "orc_on_curve", "orc_add",
                  "orc_scalar_mul", "orc_msm", "orc_msm_batch", "orc_fixed_base", "orc_ecdsa_verify"):
            getattr(L, f).restype = ci
        _lib = L
    return _lib


def _p64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _p8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check(rc: int):
    if rc != 0:
        raise RuntimeError(f"C oracle returned {rc}")


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def fp_mul(cid: int, L: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, L)
    b = np.ascontiguousarray(b, dtype=np.uint64).reshape(-1, L)
    r = np.zeros_like(a)
    _check(lib().orc_fp_mul(cid, _p64(a), _p64(b), _p64(r), a.shape[0]))
    return r


def fp_inv(cid: int, L: int, a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, L)
    r = np.zeros_like(a)
    _check(lib().orc_fp_inv(cid, _p64(a), _p64(r), a.shape[0]))
    return r


def on_curve(cid: int, L: int, pts: np.ndarray) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.uint64).reshape(-1, 2 * L)
    ok = np.zeros(pts.shape[0], dtype=np.uint8)
    _check(lib().orc_on_curve(cid, _p64(pts), pts.shape[0], _p8(ok)))
    return ok.astype(bool)


def add(cid: int, L: int, p: np.ndarray, q: np.ndarray):
    p = np.ascontiguousarray(p, dtype=np.uint64).reshape(-1, 2 * L)
    q = np.ascontiguousarray(q, dtype=np.uint64).reshape(-1, 2 * L)
    r = np.zeros_like(p)
    inf = np.zeros(p.shape[0], dtype=np.uint8)
    _check(lib().orc_add(cid, _p64(p), _p64(q), p.shape[0], _p64(r), _p8(inf)))
    return r, inf


def scalar_mul(cid: int, L: int, k: np.ndarray, p: np.ndarray):
    k = np.ascontiguousarray(k, dtype=np.uint64).reshape(-1, 4)
    p = np.ascontiguousarray(p, dtype=np.uint64).reshape(-1, 2 * L)
    r = np.zeros_like(p)
    inf = np.zeros(p.shape[0], dtype=np.uint8)
    _check(lib().orc_scalar_mul(cid, _p64(k), _p64(p), p.shape[0], _p64(r), _p8(inf)))
    return r, inf


def msm(cid: int, L: int, bases: np.ndarray, scalars: np.ndarray, threads: int | None = None):
    bases = np.ascontiguousarray(bases, dtype=np.uint64).reshape(-1, 2 * L)
    scalars = np.ascontiguousarray(scalars, dtype=np.uint64).reshape(-1, 4)
    if bases.shape[0] != scalars.shape[0]:
        raise ValueError("length mismatch")
    out = np.zeros(2 * L, dtype=np.uint64)
    inf = np.zeros(1, dtype=np.uint8)
    t = threads or default_threads()
    _check(lib().orc_msm(cid, _p64(bases), _p64(scalars), bases.shape[0], t, _p64(out), _p8(inf)))
    return out, bool(inf[0])


def msm_batch(cid: int, L: int, bases: np.ndarray, scalars: np.ndarray, offsets: np.ndarray,
              threads: int | None = None):
    bases = np.ascontiguousarray(bases, dtype=np.uint64).reshape(-1, 2 * L)
    scalars = np.ascontiguousarray(scalars, dtype=np.uint64).reshape(-1, 4)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    m = offsets.shape[0] - 1
    out = np.zeros((m, 2 * L), dtype=np.uint64)
    inf = np.zeros(m, dtype=np.uint8)
    t = threads or default_threads()
    _check(lib().orc_msm_batch(cid, _p64(bases), _p64(scalars), _p64(offsets), m, t, _p64(out), _p8(inf)))
    return out, inf.astype(bool)


def fixed_base(cid: int, L: int, ks: np.ndarray, threads: int | None = None) -> np.ndarray:
    """k_i * G as canonical affine rows (k_i must be nonzero mod the group order)."""
    ks = np.ascontiguousarray(ks, dtype=np.uint64).reshape(-1, 4)
    out = np.zeros((ks.shape[0], 2 * L), dtype=np.uint64)
    t = threads or default_threads()
    _check(lib().orc_fixed_base(cid, _p64(ks), ks.shape[0], t, _p64(out)))
    return out


def ecdsa_verify(cid: int, hashes: np.ndarray, pubkeys: np.ndarray, sigs: np.ndarray) -> np.ndarray:
    hashes = np.ascontiguousarray(hashes, dtype=np.uint8).reshape(-1, 32)
    pubkeys = np.ascontiguousarray(pubkeys, dtype=np.uint64).reshape(-1, 8)
    sigs = np.ascontiguousarray(sigs, dtype=np.uint64).reshape(-1, 8)
    m = hashes.shape[0]
    valid = np.zeros(m, dtype=np.uint8)
    _check(lib().orc_ecdsa_verify(cid, _p8(hashes), _p64(pubkeys), _p64(sigs), m, _p8(valid)))
    return valid.astype(bool)


def ecdsa_sign(cid: int, hashes: np.ndarray, privkeys: np.ndarray, nonces: np.ndarray) -> np.ndarray:
    """Textbook ECDSA signature generation (the signing side of Section 5.2's
    workload): with 1 <= d, k < n, R = k G, r = R.x mod n, e = the 32-byte
    hash read big-endian, s = k^-1 (e + r d) mod n.  Rows (r[4], s[4]) of u64;
    a row is all zero when d or k is out of range or r or s comes out zero.
    k G comes from the C oracle's fixed-base multiplication, the rest from
    Python integers."""
    from . import curves
    c = curves.BY_ID[cid]
    n = c.r
    hashes = np.ascontiguousarray(hashes, dtype=np.uint8).reshape(-1, 32)
    privkeys = np.ascontiguousarray(privkeys, dtype=np.uint64).reshape(-1, 4)
    nonces = np.ascontiguousarray(nonces, dtype=np.uint64).reshape(-1, 4)
    m = hashes.shape[0]

    def to_int(row):
        return sum(int(v) << (64 * j) for j, v in enumerate(row))

    def to_row(x):
        return [(x >> (64 * j)) & ((1 << 64) - 1) for j in range(4)]

    ds = [to_int(r) for r in privkeys]
    ks = [to_int(r) for r in nonces]
    ok = [1 <= d < n and 1 <= k < n for d, k in zip(ds, ks)]
    kk = np.array([to_row(k if o else 1) for k, o in zip(ks, ok)], dtype=np.uint64).reshape(-1, 4)
    R = fixed_base(cid, c.limbs, kk) if m else np.zeros((0, 8), dtype=np.uint64)
    out = np.zeros((m, 8), dtype=np.uint64)
    for i in range(m):
        if not ok[i]:
            continue
        r = to_int(R[i, :4]) % n
        e = int.from_bytes(bytes(hashes[i]), "big")
        s = pow(ks[i], -1, n) * (e + r * ds[i]) % n
        if r == 0 or s == 0:
            continue
        out[i, :4] = to_row(r)
        out[i, 4:] = to_row(s)
    return out
