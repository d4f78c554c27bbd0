"""Python-integer reference for the elliptic-curve operations of the path.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Points are affine pairs (x, y) of canonical integers in [0, p); the point at
infinity O is ``None``.  Field arithmetic is plain ``%`` with inversion by the
standard library's ``pow(x, -1, p)``.
"""

from __future__ import annotations

from typing import Iterable, Optional, Sequence, Tuple

from .curves import Curve

Point = Optional[Tuple[int, int]]
INF: Point = None


def on_curve(c: Curve, P: Point) -> bool:
    """Eqn 1: y^2 = x^3 + a x + b over F_p (O counts as on the curve)."""
    if P is None:
        return True
    x, y = P
    if not (0 <= x < c.p and 0 <= y < c.p):
        return False
    return (y * y - (x * x * x + c.a * x + c.b)) % c.p == 0


def neg(c: Curve, P: Point) -> Point:
    if P is None:
        return None
    x, y = P
    return (x, (-y) % c.p)


def add(c: Curve, P: Point, T: Point) -> Point:
    """Affine group law with every case.

    Generic case (x_p != x_t) is Eqns 2-3: lambda = (y_p - y_t)/(x_p - x_t),
    x_r = lambda^2 - x_p - x_t, y_r = lambda (x_p - x_r) - y_p.  When P = T the
    slope is the tangent (3 x_p^2 + a) / (2 y_p) (the PDBL paragraph of
    Section 2.1).  P + (-P) = O and O is the identity.
    """
    p = c.p
    if P is None:
        return T
    if T is None:
        return P
    xp, yp = P
    xt, yt = T
    if xp == xt:
        if (yp + yt) % p == 0:
            return None
        lam = (3 * xp * xp + c.a) * pow(2 * yp, -1, p) % p
    else:
        lam = (yp - yt) * pow(xp - xt, -1, p) % p
    xr = (lam * lam - xp - xt) % p
    yr = (lam * (xp - xr) - yp) % p
    return (xr, yr)


def double(c: Curve, P: Point) -> Point:
    return add(c, P, P)


def scalar_mul(c: Curve, s: int, P: Point) -> Point:
    """Algorithm 1 (double-and-add, least significant bit first):
    for each bit s_i from i = 0: if s_i = 1 then Q = Q + P; then P = P + P."""
    if s < 0:
        raise ValueError("negative scalar")
    Q: Point = None
    while s:
        if s & 1:
            Q = add(c, Q, P)
        P = add(c, P, P)
        s >>= 1
    return Q


def msm(c: Curve, scalars: Sequence[int], points: Sequence[Point]) -> Point:
    """The plain definition of a multi-scalar multiplication: sum_i s_i * P_i."""
    if len(scalars) != len(points):
        raise ValueError("length mismatch")
    acc: Point = None
    for s, P in zip(scalars, points):
        acc = add(c, acc, scalar_mul(c, s, P))
    return acc


def generator(c: Curve) -> Point:
    return (c.gx, c.gy)


def fixed_base(c: Curve, ks: Iterable[int]) -> list:
    """k_i * G for every k_i (slow; for small inputs)."""
    G = generator(c)
    return [scalar_mul(c, k, G) for k in ks]


# ---- ECDSA (the verify call of the library is the standard ECDSA check) ----

def hash_to_int(c: Curve, h: bytes) -> int:
    """Leftmost bitlen(n) bits of the hash, read big-endian."""
    e = int.from_bytes(h, "big")
    excess = 8 * len(h) - c.r.bit_length()
    if excess > 0:
        e >>= excess
    return e


def ecdsa_sign(c: Curve, d: int, k: int, h: bytes):
    """Signature (r, s) with nonce k, or None when r or s would be zero."""
    n = c.r
    R = scalar_mul(c, k, generator(c))
    if R is None:
        return None
    r = R[0] % n
    if r == 0:
        return None
    e = hash_to_int(c, h)
    s = pow(k, -1, n) * (e + r * d) % n
    if s == 0:
        return None
    return r, s


def ecdsa_verify(c: Curve, Q: Point, h: bytes, r: int, s: int) -> bool:
    """Valid iff 1 <= r, s < n, Q is a curve point other than O, and with
    w = s^-1, u1 = e w, u2 = r w (mod n) the point R = u1 G + u2 Q is not O
    and R.x mod n == r."""
    n = c.r
    if not (1 <= r < n and 1 <= s < n):
        return False
    if Q is None or not on_curve(c, Q):
        return False
    e = hash_to_int(c, h)
    w = pow(s, -1, n)
    u1 = e * w % n
    u2 = r * w % n
    R = add(c, scalar_mul(c, u1, generator(c)), scalar_mul(c, u2, Q))
    if R is None:
        return False
    return R[0] % n == r


# ---- Montgomery-form helpers (the boundary accepts Montgomery-form input) ---

def to_montgomery(c: Curve, x: int) -> int:
    """x * R mod p with R = 2^(64 * limbs)."""
    return x * (1 << (64 * c.limbs)) % c.p


def from_montgomery(c: Curve, x: int) -> int:
    return x * pow(1 << (64 * c.limbs), -1, c.p) % c.p


# ---- Pippenger windows (bucket grouping definition) -------------------------

def signed_digits(s: int, c: int, W: int) -> list:
    """Digits d_0..d_{W-1} with |d_w| <= 2^(c-1) and sum_w d_w 2^(c w) = s.

    Window w takes bits [c w, c w + c) of s plus the carry from window w - 1;
    a value above 2^(c-1) is replaced by value - 2^c with a carry of one into
    the next window.  W must be large enough that the last carry is zero."""
    digits = []
    carry = 0
    for w in range(W):
        d = ((s >> (c * w)) & ((1 << c) - 1)) + carry
        carry = 0
        if d > (1 << (c - 1)):
            d -= 1 << c
            carry = 1
        digits.append(d)
    if carry or (s >> (c * W)):
        raise ValueError("too few windows for this scalar")
    return digits


def bucket_lists(scalars, c: int, W: int, skip=None) -> dict:
    """bucket id (w 2^(c-1) + |d| - 1) -> sorted list of (index, negative)."""
    D = 1 << (c - 1)
    out = {}
    for i, s in enumerate(scalars):
        if skip is not None and skip[i]:
            continue
        for w, d in enumerate(signed_digits(s, c, W)):
            if d:
                out.setdefault(w * D + abs(d) - 1, []).append((i, d < 0))
    return {b: sorted(v) for b, v in out.items()}
