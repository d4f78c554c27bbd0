"""CPU derivation of the endomorphism-split constants held by the library.

The library splits every scalar as k = k1 + lambda k2 (mod r) on BN254 and
BLS12-381 (a = 0, where (x, y) -> (beta x, y) multiplies the order-r subgroup by
lambda).  Its constants (beta, the reduced lattice basis and the 2^320 Babai
multipliers) are compile-time numbers in csrc/curves.h.  This test re-derives
each of them with Python integers from the curve parameters alone and compares
with the header text:

* lambda: a nontrivial cube root of unity mod r (lambda^2 + lambda + 1 = 0);
* beta: the cube root of unity mod p for which (beta Gx, Gy) = lambda G, the
  group law checked by the oracle's Python reference;
* the basis: the short vectors of the lattice {(x, y) : x + lambda y = 0 mod r}
  from the extended Euclidean algorithm on (r, lambda), the construction of
  the GLV paper (Gallant, Lambert, Vanstone, CRYPTO 2001, Section 4);
* G1 = round(2^320 |B2| / r), G2 = round(2^320 |B1| / r);
* end to end: the split recipe stated in the header gives k1 + lambda k2 = k
  mod r with |k1|, |k2| below 2^BITS on random and edge scalars.
"""

from __future__ import annotations

import math
import os
import random
import re

import pytest

from oracle import curves, ref

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_2501_03245_amd", "csrc", "curves.h")


def _header() -> str:
    with open(HEADER) as f:
        return f.read()


def _hex_const(name: str) -> int:
    m = re.search(r'inline constexpr char %s\[\]\s*=\s*((?:\s*"[0-9a-fA-F]*")+)\s*;' % name, _header())
    assert m, name
    return int("".join(re.findall(r'"([0-9a-fA-F]*)"', m.group(1))), 16)


def _glv_block(curve: str) -> str:
    src = _header()
    start = src.index("struct Glv<%s>" % curve)
    return src[start: src.index("\n};", start)]


def _words(block: str, name: str, nwords: int) -> int:
    """A little-endian array of 64-bit words as a two's complement integer."""
    m = re.search(r"%s\[%d\]\s*=\s*\{([^}]*)\}" % (name, nwords), block)
    assert m, name
    ws = [int(w.strip().rstrip("ull").rstrip("u"), 16) for w in m.group(1).split(",")]
    assert len(ws) == nwords
    v = sum(w << (64 * i) for i, w in enumerate(ws))
    if v >> (64 * nwords - 1):
        v -= 1 << (64 * nwords)
    return v


def _bits(block: str) -> int:
    return int(re.search(r"BITS\s*=\s*(\d+)", block).group(1))


def cube_roots_of_unity(m: int) -> list:
    """The two nontrivial cube roots of unity mod a prime m = 1 (mod 3)."""
    assert (m - 1) % 3 == 0
    for g in range(2, 1000):
        w = pow(g, (m - 1) // 3, m)
        if w != 1:
            return sorted({w, w * w % m})
    raise AssertionError("no cube root found")


def glv_basis(r: int, lam: int):
    """GLV paper, Section 4: run the extended Euclidean algorithm on (r, lambda)
    keeping r_i = s_i r + t_i lambda; with l the largest index with
    r_l >= sqrt(r), v1 = (r_{l+1}, -t_{l+1}) and v2 the shorter of
    (r_l, -t_l) and (r_{l+2}, -t_{l+2})."""
    rs, ts = [r, lam], [0, 1]
    while rs[-1] != 0:
        q = rs[-2] // rs[-1]
        rs.append(rs[-2] - q * rs[-1])
        ts.append(ts[-2] - q * ts[-1])
    root = math.isqrt(r)
    l = max(i for i, v in enumerate(rs) if v >= root)
    v1 = (rs[l + 1], -ts[l + 1])
    c1, c2 = (rs[l], -ts[l]), (rs[l + 2], -ts[l + 2])
    v2 = c1 if c1[0] ** 2 + c1[1] ** 2 <= c2[0] ** 2 + c2[1] ** 2 else c2
    return v1, v2


def _same_lattice_vector(u, v) -> bool:
    return u == v or u == (-v[0], -v[1])


CASES = [("BN254", curves.BN254, "BN254_BETA"), ("BLS12_381", curves.BLS12_381, "BLS_BETA")]


@pytest.mark.parametrize("name,c,beta_name", CASES, ids=[n for n, _, _ in CASES])
def test_beta_lambda_pair(name, c, beta_name):
    beta = _hex_const(beta_name)
    assert beta in cube_roots_of_unity(c.p)
    G = ref.generator(c)
    phiG = (beta * c.gx % c.p, c.gy)
    assert ref.on_curve(c, phiG)
    lams = [lam for lam in cube_roots_of_unity(c.r) if ref.scalar_mul(c, lam, G) == phiG]
    assert len(lams) == 1, "exactly one cube root of unity mod r matches beta"
    # the other root of p pairs with the other root of r
    other = [b for b in cube_roots_of_unity(c.p) if b != beta][0]
    assert ref.scalar_mul(c, [x for x in cube_roots_of_unity(c.r) if x != lams[0]][0], G) == \
        (other * c.gx % c.p, c.gy)


def _lambda(c, beta_name) -> int:
    beta = _hex_const(beta_name)
    G = ref.generator(c)
    phiG = (beta * c.gx % c.p, c.gy)
    return [lam for lam in cube_roots_of_unity(c.r) if ref.scalar_mul(c, lam, G) == phiG][0]


def test_bls_lambda_is_z_squared_minus_one():
    z = -0xD201000000010000  # BLS12-381 curve parameter
    lam = _lambda(curves.BLS12_381, "BLS_BETA")
    assert lam == z * z - 1
    assert curves.BLS12_381.r == lam * lam + lam + 1


@pytest.mark.parametrize("name,c,beta_name", CASES, ids=[n for n, _, _ in CASES])
def test_basis_and_multipliers(name, c, beta_name):
    lam = _lambda(c, beta_name)
    blk = _glv_block(name)
    A1, B1, A2, B2 = (_words(blk, k, 3) for k in ("A1", "B1", "A2", "B2"))
    G1, G2 = _words(blk, "G1", 4), _words(blk, "G2", 4)
    # lattice membership and determinant +-r
    for a, b in ((A1, B1), (A2, B2)):
        assert (a + lam * b) % c.r == 0
    det = A1 * B2 - A2 * B1
    assert abs(det) == c.r
    # the same short vectors as the GLV extended-Euclid construction
    v1, v2 = glv_basis(c.r, lam)
    got = [(A1, B1), (A2, B2)]
    assert any(_same_lattice_vector(got[0], v) for v in (v1, v2))
    assert any(_same_lattice_vector(got[1], v) for v in (v1, v2))
    assert not _same_lattice_vector(got[0], got[1])
    # Babai multipliers: rounding of 2^320 |B2| / r and 2^320 |B1| / r
    assert G1 == (2 * (abs(B2) << 320) + c.r) // (2 * c.r)
    assert G2 == (2 * (abs(B1) << 320) + c.r) // (2 * c.r)
    # the header's sign statement: k B2 / det and -k B1 / det are non-negative
    assert B2 * det > 0 and -B1 * det > 0


@pytest.mark.parametrize("name,c,beta_name", CASES, ids=[n for n, _, _ in CASES])
def test_split_recipe_bounds(name, c, beta_name):
    lam = _lambda(c, beta_name)
    blk = _glv_block(name)
    A1, B1, A2, B2 = (_words(blk, k, 3) for k in ("A1", "B1", "A2", "B2"))
    G1, G2 = _words(blk, "G1", 4), _words(blk, "G2", 4)
    bits = _bits(blk)
    rng = random.Random(0x61F)
    ks = [0, 1, 2, lam - 1, lam, lam + 1, 2 * lam, c.r - 1, c.r - lam, (c.r - 1) // 2]
    ks += [rng.randrange(c.r) for _ in range(3000)]
    ks += [rng.randrange(1 << 64) for _ in range(100)]
    for k in ks:
        c1 = (k * G1 + (1 << 319)) >> 320
        c2 = (k * G2 + (1 << 319)) >> 320
        k1 = k - c1 * A1 - c2 * A2
        k2 = -c1 * B1 - c2 * B2
        assert (k1 + lam * k2 - k) % c.r == 0
        assert abs(k1) < (1 << bits) and abs(k2) < (1 << bits), hex(k)
