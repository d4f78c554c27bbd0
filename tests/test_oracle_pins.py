"""Pins for the CPU oracle: facts fixed by mathematics or external sources,
chosen so that a dropped term, a wrong sign or index, or a transposed operand
in either oracle implementation fails at least one of them."""

import math
import os
import random

import numpy as np
import pytest

from oracle import c_oracle as co
from oracle import curves, ref
from synthetic import ints_to_limbs, limbs_to_int

ALL = list(curves.CURVES.values())
HERE = os.path.dirname(os.path.abspath(__file__))


def pt_rows(c, pts):
    rows = []
    for P in pts:
        if P is None:
            rows.append([0] * (2 * c.limbs))
        else:
            rows.append(list(ints_to_limbs([P[0]], c.limbs)[0]) + list(ints_to_limbs([P[1]], c.limbs)[0]))
    return np.array(rows, dtype=np.uint64).reshape(-1, 2 * c.limbs)


def row_pt(c, row, inf=False):
    if inf:
        return None
    x, y = limbs_to_int(row[: c.limbs]), limbs_to_int(row[c.limbs:])
    if x == 0 and y == 0:
        return None
    return (x, y)


def is_probable_prime(n):
    if n < 2:
        return False
    for sp in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % sp == 0:
            return n == sp
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


# ---- curve constants --------------------------------------------------------

def test_bn254_from_family_polynomial():
    u = 4965661367192848881
    assert curves.BN254.p == 36 * u**4 + 36 * u**3 + 24 * u**2 + 6 * u + 1
    assert curves.BN254.r == 36 * u**4 + 36 * u**3 + 18 * u**2 + 6 * u + 1


def test_bls12_381_from_family_polynomial():
    x = -0xD201000000010000
    r = x**4 - x**2 + 1
    assert curves.BLS12_381.r == r
    assert curves.BLS12_381.p == (x - 1) ** 2 * r // 3 + x
    assert ((x - 1) ** 2 * r) % 3 == 0


def test_p256_prime_form_and_qinv():
    c = curves.SECP256R1
    assert c.p == 2**256 - 2**224 + 2**192 + 2**96 - 1
    # Section 2.2: these special primes have q_inv = -q^-1 mod D equal to 1
    assert (-pow(c.p, -1, 2**64)) % 2**64 == 1
    assert (-pow(c.p, -1, 2**32)) % 2**32 == 1


def test_sm2_prime_form_and_qinv():
    """Section 4.2 states SM2's prime as 2^256 - 2^224 - 2^96 + 2^64 - 1 and
    its q_inv as 1; a = -3 and the cofactor is 1 (r is within the Hasse
    interval around p + 1)."""
    c = curves.SM2
    assert c.p == 2**256 - 2**224 - 2**96 + 2**64 - 1
    assert (-pow(c.p, -1, 2**64)) % 2**64 == 1
    assert (-pow(c.p, -1, 2**32)) % 2**32 == 1
    assert c.a == c.p - 3
    assert abs(c.p + 1 - c.r) <= 2 * math.isqrt(c.p) + 1


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_primes_and_generator_order(c):
    assert is_probable_prime(c.p)
    assert is_probable_prime(c.r)
    G = ref.generator(c)
    assert ref.on_curve(c, G)
    assert ref.scalar_mul(c, c.r, G) is None
    assert ref.scalar_mul(c, 1, G) == G
    assert ref.scalar_mul(c, c.r - 1, G) == ref.neg(c, G)
    # Hasse bound: the group order (a multiple of r) is within 2 sqrt(p) of p + 1
    h = round((c.p + 1) / c.r)
    assert abs(c.p + 1 - h * c.r) <= 2 * int(c.p ** 0.5) + 2 or h > 1


def test_p256_double_generator_matches_published_vector():
    c = curves.SECP256R1
    with open(os.path.join(HERE, "golden", "p256_2G.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    k, x, y = int(rows[0][0]), int(rows[0][1], 16), int(rows[0][2], 16)
    assert ref.scalar_mul(c, k, ref.generator(c)) == (x, y)
    out, inf = co.scalar_mul(c.cid, c.limbs, ints_to_limbs([k], 4), pt_rows(c, [ref.generator(c)]))
    assert row_pt(c, out[0], inf[0]) == (x, y)


def test_no_two_torsion():
    """(0,0) is the infinity sentinel at the boundary: it is off every curve
    (b != 0) and no curve point has y = 0 because each group order is odd."""
    for c in ALL:
        assert not ref.on_curve(c, (0, 0))
        assert c.r % 2 == 1
    # BN254 and secp256r1 have cofactor 1; BLS12-381 G1's full group order is odd too
    bls = curves.BLS12_381
    x = -0xD201000000010000
    h = (x - 1) ** 2 // 3
    assert (h * bls.r) % 2 == 1


# ---- field arithmetic -------------------------------------------------------

@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_c_field_mul_matches_python_ints(c):
    rnd = random.Random(11)
    R = 1 << (64 * c.limbs)
    edge = [0, 1, 2, c.p - 1, c.p - 2, R % c.p, R * R % c.p, (c.p + 1) // 2]
    a = edge + [rnd.randrange(c.p) for _ in range(300)]
    b = [c.p - 1] * len(edge) + [rnd.randrange(c.p) for _ in range(300)]
    r = co.fp_mul(c.cid, c.limbs, ints_to_limbs(a, c.limbs), ints_to_limbs(b, c.limbs))
    for i in range(len(a)):
        assert limbs_to_int(r[i]) == a[i] * b[i] % c.p
    aa = [x for x in a if x]
    inv = co.fp_inv(c.cid, c.limbs, ints_to_limbs(aa, c.limbs))
    for i, x in enumerate(aa):
        assert limbs_to_int(inv[i]) * x % c.p == 1
        assert limbs_to_int(inv[i]) == pow(x, -1, c.p)


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_montgomery_round_trip(c):
    rnd = random.Random(5)
    for _ in range(50):
        x = rnd.randrange(c.p)
        m = ref.to_montgomery(c, x)
        assert ref.from_montgomery(c, m) == x
        assert m == x * 2 ** (64 * c.limbs) % c.p


# ---- group law --------------------------------------------------------------

def rand_points(c, n, seed):
    rnd = random.Random(seed)
    G = ref.generator(c)
    return [ref.scalar_mul(c, rnd.randrange(1, c.r), G) for _ in range(n)]


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_group_axioms_python(c):
    P, Q, T = rand_points(c, 3, 3)
    for X in (P, Q, T):
        assert ref.on_curve(c, X)
    assert ref.add(c, P, Q) == ref.add(c, Q, P)
    assert ref.add(c, ref.add(c, P, Q), T) == ref.add(c, P, ref.add(c, Q, T))
    assert ref.add(c, P, None) == P and ref.add(c, None, P) == P
    assert ref.add(c, P, ref.neg(c, P)) is None
    S = ref.add(c, P, Q)
    D = ref.double(c, P)
    assert ref.on_curve(c, S) and ref.on_curve(c, D)
    # (P + Q) - Q = P exercises the generic slope in both directions
    assert ref.add(c, S, ref.neg(c, Q)) == P
    # 2P - P = P ties the tangent slope to the chord slope
    assert ref.add(c, D, ref.neg(c, P)) == P


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_c_add_matches_python(c):
    pts = rand_points(c, 8, 4)
    ps = pts + [pts[0], pts[1], None, pts[2], None]
    qs = list(reversed(pts)) + [pts[0], ref.neg(c, pts[1]), pts[3], None, None]
    r, inf = co.add(c.cid, c.limbs, pt_rows(c, ps), pt_rows(c, qs))
    for i in range(len(ps)):
        assert row_pt(c, r[i], inf[i]) == ref.add(c, ps[i], qs[i])


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_scalar_mul_brute_force(c):
    P = rand_points(c, 1, 6)[0]
    acc = None
    ks = list(range(0, 65))
    expect = []
    for k in ks:
        expect.append(acc)
        acc = ref.add(c, acc, P)
    for k in ks:
        assert ref.scalar_mul(c, k, P) == expect[k]
    r, inf = co.scalar_mul(c.cid, c.limbs, ints_to_limbs(ks, 4), pt_rows(c, [P] * len(ks)))
    for k in ks:
        assert row_pt(c, r[k], inf[k]) == expect[k]


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_scalar_mul_linearity(c):
    rnd = random.Random(8)
    P = rand_points(c, 1, 9)[0]
    for _ in range(3):
        a, b = rnd.randrange(c.r), rnd.randrange(c.r)
        lhs = ref.scalar_mul(c, a + b, P)
        rhs = ref.add(c, ref.scalar_mul(c, a, P), ref.scalar_mul(c, b, P))
        assert lhs == rhs
        assert ref.scalar_mul(c, a * b % c.r, P) == ref.scalar_mul(c, a, ref.scalar_mul(c, b, P))


# ---- MSM ----------------------------------------------------------------------

@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_msm_brute_force_tiny(c):
    rnd = random.Random(12)
    for n in range(0, 9):
        pts = rand_points(c, n, 100 + n)
        ss = [rnd.randrange(16) for _ in range(n)]
        acc = None
        for s, P in zip(ss, pts):
            for _ in range(s):
                acc = ref.add(c, acc, P)
        assert ref.msm(c, ss, pts) == acc
        out, inf = co.msm(c.cid, c.limbs, pt_rows(c, pts), ints_to_limbs(ss, 4).reshape(-1, 4), threads=3)
        assert row_pt(c, out, inf) == acc


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_msm_c_matches_python_and_linearity(c):
    rnd = random.Random(13)
    n = 24
    pts = rand_points(c, n, 14)
    s = [rnd.randrange(c.r) for _ in range(n)]
    t = [rnd.randrange(c.r) for _ in range(n)]
    rows = pt_rows(c, pts)
    out_s, inf_s = co.msm(c.cid, c.limbs, rows, ints_to_limbs(s, 4), threads=4)
    assert row_pt(c, out_s, inf_s) == ref.msm(c, s, pts)
    out_t, inf_t = co.msm(c.cid, c.limbs, rows, ints_to_limbs(t, 4), threads=2)
    st = [(a + b) % c.r for a, b in zip(s, t)]
    out_st, inf_st = co.msm(c.cid, c.limbs, rows, ints_to_limbs(st, 4), threads=5)
    assert row_pt(c, out_st, inf_st) == ref.add(c, row_pt(c, out_s, inf_s), row_pt(c, out_t, inf_t))


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_msm_special_cases(c):
    pts = rand_points(c, 4, 15)
    rows = pt_rows(c, pts)
    z = ints_to_limbs([0, 0, 0, 0], 4)
    out, inf = co.msm(c.cid, c.limbs, rows, z)
    assert inf
    out, inf = co.msm(c.cid, c.limbs, rows[:0], z[:0])
    assert inf
    out, inf = co.msm(c.cid, c.limbs, rows[:1], ints_to_limbs([12345], 4))
    assert row_pt(c, out, inf) == ref.scalar_mul(c, 12345, pts[0])
    # duplicated and negated bases: P + P and P + (-P)
    P = pts[0]
    dup = pt_rows(c, [P, P, ref.neg(c, P), pts[1]])
    out, inf = co.msm(c.cid, c.limbs, dup, ints_to_limbs([5, 7, 12, 0], 4), threads=4)
    assert inf  # 5P + 7P - 12P
    out, inf = co.msm(c.cid, c.limbs, dup, ints_to_limbs([5, 7, 11, 1], 4), threads=2)
    assert row_pt(c, out, inf) == ref.add(c, P, pts[1])
    # infinity inputs contribute nothing
    withinf = pt_rows(c, [None, pts[2]])
    out, inf = co.msm(c.cid, c.limbs, withinf, ints_to_limbs([99, 3], 4))
    assert row_pt(c, out, inf) == ref.scalar_mul(c, 3, pts[2])


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_msm_discrete_log_identity(c):
    """With P_i = k_i G, sum s_i P_i = (sum s_i k_i mod r) G: the identity the
    full-size GPU tests use, pinned here on the oracle itself."""
    rnd = random.Random(16)
    n = 40
    ks = [rnd.randrange(1, c.r) for _ in range(n)]
    s = [rnd.randrange(1 << c.scalar_bits) for _ in range(n)]
    bases = co.fixed_base(c.cid, c.limbs, ints_to_limbs(ks, 4))
    for i in range(0, n, 13):
        assert row_pt(c, bases[i]) == ref.scalar_mul(c, ks[i], ref.generator(c))
    out, inf = co.msm(c.cid, c.limbs, bases, ints_to_limbs(s, 4), threads=4)
    e = sum(a * b for a, b in zip(s, ks)) % c.r
    assert row_pt(c, out, inf) == ref.scalar_mul(c, e, ref.generator(c))


def test_msm_batch_segments():
    c = curves.BN254
    rnd = random.Random(17)
    pts = rand_points(c, 10, 18)
    s = [rnd.randrange(c.r) for _ in range(10)]
    offsets = np.array([0, 3, 3, 10], dtype=np.uint64)
    out, inf = co.msm_batch(c.cid, c.limbs, pt_rows(c, pts), ints_to_limbs(s, 4), offsets)
    assert row_pt(c, out[0], inf[0]) == ref.msm(c, s[:3], pts[:3])
    assert inf[1]
    assert row_pt(c, out[2], inf[2]) == ref.msm(c, s[3:], pts[3:])


# ---- ECDSA --------------------------------------------------------------------

@pytest.mark.parametrize("c", [curves.SECP256R1, curves.SM2], ids=lambda c: c.name)
def test_ecdsa_round_trip_and_rejections(c):
    rnd = random.Random(19)
    hashes, keys, sigs, expect = [], [], [], []
    for i in range(12):
        d = rnd.randrange(1, c.r)
        Q = ref.scalar_mul(c, d, ref.generator(c))
        h = bytes(rnd.randrange(256) for _ in range(32))
        sig = None
        while sig is None:
            sig = ref.ecdsa_sign(c, d, rnd.randrange(1, c.r), h)
        r, s = sig
        assert ref.ecdsa_verify(c, Q, h, r, s)
        bad = bytearray(h)
        bad[i % 32] ^= 1 << (i % 8)
        assert not ref.ecdsa_verify(c, Q, bytes(bad), r, s)
        cases = [(h, Q, r, s, True), (bytes(bad), Q, r, s, False), (h, Q, 0, s, False), (h, Q, r, 0, False),
                 (h, Q, r + c.r, s, False), (h, None, r, s, False), (h, Q, r, s % (c.r - 1) + 1, False),
                 (h, Q, r, c.r - s, True)]  # (r, -s) also verifies: R flips sign, x is unchanged
        for hh, QQ, rr, ss, ok in cases:
            if rr >= 1 << 256:
                continue
            assert ref.ecdsa_verify(c, QQ, hh, rr, ss) == ok
            hashes.append(list(hh))
            keys.append(QQ)
            sigs.append(list(ints_to_limbs([rr], 4)[0]) + list(ints_to_limbs([ss], 4)[0]))
            expect.append(ok)
    got = co.ecdsa_verify(c.cid, np.array(hashes, dtype=np.uint8), pt_rows(c, keys),
                          np.array(sigs, dtype=np.uint64))
    assert list(got) == expect


@pytest.mark.parametrize("c", [curves.SECP256R1, curves.SM2], ids=lambda c: c.name)
def test_ecdsa_sign_batch_round_trip(c):
    """The batch signer (C fixed-base k G, Python integers for the rest) agrees
    with the pure-Python signer, every signature it makes verifies under
    Q = d G, and out-of-range keys or nonces give empty rows."""
    rnd = random.Random(23)
    m = 10
    d = [rnd.randrange(1, c.r) for _ in range(m)]
    k = [rnd.randrange(1, c.r) for _ in range(m)]
    d[3], k[4], d[5], k[6] = 0, c.r, c.r + 1, 0
    h = [bytes(rnd.randrange(256) for _ in range(32)) for _ in range(m)]
    h[7] = b"\xff" * 32  # e >= n
    h[8] = bytes(32)      # e = 0
    sig = co.ecdsa_sign(c.cid, np.array([list(x) for x in h], dtype=np.uint8), ints_to_limbs(d, 4),
                        ints_to_limbs(k, 4))
    for i in range(m):
        r, s = limbs_to_int(sig[i, :4]), limbs_to_int(sig[i, 4:])
        if i in (3, 4, 5, 6):
            assert r == s == 0
            continue
        assert (r, s) == ref.ecdsa_sign(c, d[i], k[i], h[i])
        assert ref.ecdsa_verify(c, ref.scalar_mul(c, d[i], ref.generator(c)), h[i], r, s)


@pytest.mark.parametrize("c", ALL, ids=lambda c: c.name)
def test_c_on_curve_matches_definition(c):
    """The C oracle's point check agrees with Eqn 1 evaluated on Python
    integers, with the range check x, y < p, on points on the curve, their
    negations, off-curve neighbours, out-of-range coordinates and (0, 0)."""
    rnd = random.Random(31)
    G = ref.generator(c)
    pts = [ref.scalar_mul(c, rnd.randrange(1, c.r), G) for _ in range(6)] + [G]
    rows = []
    for x, y in pts:
        rows += [(x, y), (x, c.p - y), (x, (y + 1) % c.p), ((x + 1) % c.p, y), (x + c.p, y), (x, y + c.p)]
    rows += [(0, 0), (c.p - 1, c.p - 1), (0, 1)]
    rows = [r for r in rows if r[0] < 1 << (64 * c.limbs) and r[1] < 1 << (64 * c.limbs)]

    def eqn1(x, y):
        return x < c.p and y < c.p and (y * y - x * x * x - c.a * x - c.b) % c.p == 0

    arr = np.array([list(ints_to_limbs([x], c.limbs)[0]) + list(ints_to_limbs([y], c.limbs)[0]) for x, y in rows],
                   dtype=np.uint64)
    got = co.on_curve(c.cid, c.limbs, arr)
    want = [eqn1(x, y) for x, y in rows]
    assert list(got) == want
    assert sum(want) == 2 * len(pts)  # each point and its negation, nothing else


def off_curve_key_signature(c, seed):
    """A key Q' off the curve (on y^2 = x^3 + a x + b + 1) with a signature on
    the all-zero hash that passes every other step of verification: e = 0 makes
    u1 = 0, and (r, s) are chosen so that u2 = t and R = t Q' has R.x = r mod n.
    The group law of Eqns 2-3 and PDBL never reads b, so only the on-curve test
    tells this request apart from a valid one."""
    rnd = random.Random(seed)
    b2 = (c.b + 1) % c.p
    assert c.p % 4 == 3
    while True:
        x = rnd.randrange(c.p)
        rhs = (x ** 3 + c.a * x + b2) % c.p
        y = pow(rhs, (c.p + 1) // 4, c.p)
        if y * y % c.p == rhs and y != 0:
            break
    Qbad = (x, y)
    while True:
        t = rnd.randrange(1, c.r)
        R = ref.scalar_mul(c, t, Qbad)
        if R is not None and R[0] % c.r != 0:
            break
    r = R[0] % c.r
    s = r * pow(t, -1, c.r) % c.r
    return bytes(32), Qbad, r, s


@pytest.mark.parametrize("c", [curves.SECP256R1, curves.SM2], ids=lambda c: c.name)
def test_ecdsa_rejects_off_curve_key_that_would_verify(c, monkeypatch):
    h, Qbad, r, s = off_curve_key_signature(c, 37)
    assert not ref.on_curve(c, Qbad)
    assert not ref.ecdsa_verify(c, Qbad, h, r, s)
    got = co.ecdsa_verify(c.cid, np.array([list(h)], dtype=np.uint8), pt_rows(c, [Qbad]),
                          np.array([list(ints_to_limbs([r], 4)[0]) + list(ints_to_limbs([s], 4)[0])],
                                   dtype=np.uint64))
    assert list(got) == [False]
    # without the on-curve test the same request verifies: the rejection is
    # that test's, not an accident of the arithmetic
    monkeypatch.setattr(ref, "on_curve", lambda cc, P: True)
    assert ref.ecdsa_verify(c, Qbad, h, r, s)


# ---- planted mistakes: the pins above must catch plausible oracle bugs -----

def _broken_add_sign(c, P, T):
    if P is None:
        return T
    if T is None:
        return P
    xp, yp = P
    xt, yt = T
    if xp == xt:
        if (yp + yt) % c.p == 0:
            return None
        lam = (3 * xp * xp + c.a) * pow(2 * yp, -1, c.p) % c.p
    else:
        lam = (yp - yt) * pow(xp - xt, -1, c.p) % c.p
    xr = (lam * lam - xp - xt) % c.p
    yr = (lam * (xp - xr) + yp) % c.p  # wrong sign on the last term
    return (xr, yr)


def _broken_add_dropped_a(c, P, T):
    if P is None:
        return T
    if T is None:
        return P
    xp, yp = P
    xt, yt = T
    if xp == xt:
        if (yp + yt) % c.p == 0:
            return None
        lam = (3 * xp * xp) * pow(2 * yp, -1, c.p) % c.p  # dropped the a term
    else:
        lam = (yp - yt) * pow(xp - xt, -1, c.p) % c.p
    xr = (lam * lam - xp - xt) % c.p
    yr = (lam * (xp - xr) - yp) % c.p
    return (xr, yr)


def test_planted_mistakes_are_caught(monkeypatch):
    c = curves.BN254
    monkeypatch.setattr(ref, "add", lambda cc, P, T: _broken_add_sign(cc, P, T))
    G = ref.generator(c)
    assert not (ref.on_curve(c, ref.add(c, G, ref.double(c, G))) and ref.scalar_mul(c, c.r, G) is None)
    monkeypatch.undo()
    p256 = curves.SECP256R1
    monkeypatch.setattr(ref, "add", lambda cc, P, T: _broken_add_dropped_a(cc, P, T))
    G = ref.generator(p256)
    assert ref.scalar_mul(p256, p256.r, G) is not None or not ref.on_curve(p256, ref.double(p256, G))


def test_stored_p256_requests_match_the_oracle():
    """The benchmark's stored verification requests are reproduced by their
    generator and their stored verdicts are the oracle's."""
    import os
    from tests.common import seeded_signatures
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "p256_requests.npz"))
    h, q, s = seeded_signatures(64, int(z["seed"][0]))
    # the generator draws per index, so the first rows of a longer run agree
    # except for corruptions that pick a neighbour key (index-dependent wrap)
    assert np.array_equal(h, z["hashes"][:64])
    assert np.array_equal(s, z["sigs"][:64])
    v = co.ecdsa_verify(curves.SECP256R1.cid, z["hashes"][:512], z["pubkeys"][:512], z["sigs"][:512])
    assert np.array_equal(v.astype(np.uint8), z["valid"][:512])
    assert int(z["valid"].sum()) == z["valid"].shape[0] - z["valid"].shape[0] // 16
