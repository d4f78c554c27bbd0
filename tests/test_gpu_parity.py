"""Parity of the HIP path with the CPU oracle, through the C ABI.

Every comparison is bit-exact: field elements, points and bucket contents are
integers, and the group sum is unique."""

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves, ref
from tests.common import (dlog_msm_expected, oracle_msm, points_to_rows, rows_to_points, seeded_bases,
                          seeded_scalars)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")

MSM_CURVES = [curves.BN254, curves.BLS12_381]
ALL_CURVES = [curves.BN254, curves.BLS12_381, curves.SECP256R1, curves.SM2]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.close()


def dev(a: np.ndarray):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).cuda()
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32).copy()).cuda()
    if a.dtype == np.uint8:
        return torch.from_numpy(a.copy()).cuda()
    raise TypeError(a.dtype)


def host64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def host32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def empty64(n):
    return torch.zeros(max(1, n), dtype=torch.int64, device="cuda")


def empty32(n):
    return torch.zeros(max(1, n), dtype=torch.int32, device="cuda")


def run_msm(ctx, c, bases, scalars, flags=0, window_c=0):
    n = bases.shape[0]
    out = empty64(2 * c.limbs)
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
    eccmi.ecc_msm(ctx, c.cid, dev(bases) if n else None, dev(scalars) if n else None, n, out, inf, flags=flags,
                  window_c=window_c)
    torch.cuda.synchronize()
    return rows_to_points(c, host64(out).reshape(1, -1), inf.cpu().numpy())[0]


def field_cases(c, n, seed):
    R = 1 << (64 * c.limbs)
    edge = [0, 1, 2, 3, c.p - 1, c.p - 2, R % c.p, R * R % c.p, (c.p + 1) // 2, (1 << 32) - 1, 1 << 32,
            (1 << (32 * (2 * c.limbs - 1))) % c.p]
    # values whose working (Montgomery, R = 2^e) form is 1 or -1, for each
    # curve's e: products of tiny limbs, where a reduction column that
    # subtracts a digit of p can go negative
    for e in (261, 280, 392):
        edge += [pow(2, -e, c.p), c.p - pow(2, -e, c.p), 3 * pow(2, -e, c.p) % c.p]
    vals = edge + [syn.limbs_to_int(r) for r in syn.uniform_below(seed, syn.TAG_MISC, n, c.p, c.limbs)]
    return vals


# ---- field ----------------------------------------------------------------

@pytest.mark.parametrize("c", ALL_CURVES, ids=lambda c: c.name)
def test_fp_mul_parity(ctx, c):
    a = field_cases(c, 5000, 1)
    b = list(reversed(field_cases(c, 5000, 2)))
    A, B = syn.ints_to_limbs(a, c.limbs), syn.ints_to_limbs(b, c.limbs)
    out = empty64(A.size)
    eccmi.ecc_test_fp_mul(ctx, c.cid, dev(A), dev(B), out, len(a))
    got = host64(out).reshape(-1, c.limbs)
    exp = co.fp_mul(c.cid, c.limbs, A, B)
    assert np.array_equal(got, exp)
    # the same array for both operands selects the squaring routine
    Ad = dev(A)
    eccmi.ecc_test_fp_mul(ctx, c.cid, Ad, Ad, out, len(a))
    assert np.array_equal(host64(out).reshape(-1, c.limbs), co.fp_mul(c.cid, c.limbs, A, A))


@pytest.mark.parametrize("c", ALL_CURVES, ids=lambda c: c.name)
@pytest.mark.parametrize("op", range(8), ids=["mul", "sub", "mixed", "dbl_t", "add_t", "add_x3", "lazy_y_sq", "lazy_y"])
def test_lane_field_parity(ctx, c, op):
    """The lane-parallel field of the window combination (limbs spread over a
    16-lane row) against integer arithmetic mod p, with a ragged last wave."""
    a = field_cases(c, 3001, 4)
    b = list(reversed(field_cases(c, 3001, 5)))
    A, B = syn.ints_to_limbs(a, c.limbs), syn.ints_to_limbs(b, c.limbs)
    out = empty64(A.size)
    eccmi.ecc_test_lane_field(ctx, c.cid, op, dev(A), dev(B), out, len(a))
    got = [syn.limbs_to_int(r) for r in host64(out).reshape(-1, c.limbs)]
    p = c.p
    if op == 0:
        exp = [x * y % p for x, y in zip(a, b)]
    elif op == 1:
        exp = [(x - y) % p for x, y in zip(a, b)]
    elif op == 2:
        exp = [(3 * x * (x + y) - 2 * y) % p for x, y in zip(a, b)]
    elif op == 3:
        exp = [(3 * x * y - x * x) % p for x, y in zip(a, b)]
    elif op == 4:
        exp = [(3 * y * y + x * y - x * x) % p for x, y in zip(a, b)]
    elif op == 5:
        exp = [(x * x - x * y - 2 * y * y) % p for x, y in zip(a, b)]
    elif op == 6:
        exp = [(2 * (x * y - x * x)) ** 2 % p for x, y in zip(a, b)]
    else:
        exp = [(x * y - x * x) % p for x, y in zip(a, b)]
    assert got == exp


@pytest.mark.parametrize("c", ALL_CURVES, ids=lambda c: c.name)
def test_fp_inv_parity(ctx, c):
    a = [x for x in field_cases(c, 3000, 3)]
    A = syn.ints_to_limbs(a, c.limbs)
    out = empty64(A.size)
    eccmi.ecc_test_fp_inv(ctx, c.cid, dev(A), out, len(a))
    got = host64(out).reshape(-1, c.limbs)
    nz = np.array([x != 0 for x in a])
    exp = np.zeros_like(A)
    exp[nz] = co.fp_inv(c.cid, c.limbs, A[nz])
    assert np.array_equal(got, exp)


# ---- batch-affine addition --------------------------------------------------

@pytest.mark.parametrize("c", ALL_CURVES, ids=lambda c: c.name)
def test_batch_add_parity_with_exceptional_lanes(ctx, c):
    k, base = seeded_bases(c.name, 1200, 11)
    pts = rows_to_points(c, base)
    P, Q = [], []
    P += pts[:1000]
    Q += pts[200:1200]                       # generic (a few coincide by design of the slices)
    P += pts[:60]
    Q += pts[:60]                            # doubling
    P += pts[60:120]
    Q += [ref.neg(c, x) for x in pts[60:120]]  # P + (-P) = O
    P += pts[120:140]
    Q += [None] * 20                         # P + O
    P += [None] * 20
    Q += pts[140:160]                        # O + P
    P += [None] * 5
    Q += [None] * 5                          # O + O
    order = np.argsort(syn.u64(5, syn.TAG_MISC, len(P)), kind="stable")
    P = [P[i] for i in order]
    Q = [Q[i] for i in order]
    Pr, Qr = points_to_rows(c, P), points_to_rows(c, Q)
    out = empty64(Pr.size)
    eccmi.ecc_test_batch_add(ctx, c.cid, dev(Pr), dev(Qr), out, len(P))
    got = host64(out).reshape(-1, 2 * c.limbs)
    exp, inf = co.add(c.cid, c.limbs, Pr, Qr)
    assert np.array_equal(got, exp)


# ---- bucket grouping ----------------------------------------------------------

@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
@pytest.mark.parametrize("wc", [4, 13, 16])
@pytest.mark.parametrize("method", [1, 2], ids=["atomic", "lds"])
def test_bucket_sort_parity(ctx, c, wc, method):
    n = 3001 if method == 1 else 20001
    s = seeded_scalars(c.name, n, 21 + wc, kind="bits")
    top = (1 << c.scalar_bits) - 1
    s[:4] = syn.ints_to_limbs([0, 1, top, 1 << (c.scalar_bits - 1)], 4)
    W, D, B = eccmi.bucket_geometry(c.cid, wc)
    counts, offsets, srt = empty32(B + 1), empty32(B + 1), empty32(n * W)
    eccmi.ecc_test_bucket_sort(ctx, c.cid, dev(s), n, wc, counts, offsets, srt, method=method)
    counts, offsets, srt = host32(counts), host32(offsets), host32(srt)
    lists = ref.bucket_lists([syn.limbs_to_int(r) for r in s], wc, W)
    exp_counts = np.zeros(B + 1, dtype=np.uint32)
    for b, v in lists.items():
        exp_counts[b] = len(v)
    assert np.array_equal(counts, exp_counts)
    exp_off = np.concatenate([[0], np.cumsum(exp_counts[:B])]).astype(np.uint32)
    assert np.array_equal(offsets, exp_off)
    for b, v in lists.items():
        seg = srt[offsets[b]: offsets[b] + counts[b]]
        got = sorted((int(e) & 0x7FFFFFFF, bool(int(e) >> 31)) for e in seg)
        assert got == v


@pytest.mark.parametrize("case", ["equal_scalars", "few_keys", "multi_chunk"])
def test_bucket_sort_two_level_shapes(ctx, case):
    """The two-level sort on inputs that leave its common path: one bucket per
    window holding every entry (a coarse bin too large for LDS); one coarse
    bin too large for LDS spread over 64 buckets (scalars in [1, 64], so the
    aggregated counter increments see several keys per wave); and several
    chunks per window with ragged ends."""
    c = curves.BLS12_381
    if case == "equal_scalars":
        n, wc = 20001, 16
        one = seeded_scalars(c.name, 1, 77, kind="bits")
        s = np.repeat(one, n, axis=0)
    elif case == "few_keys":
        n, wc = 20001, 16
        s = syn.uniform_range(79, syn.TAG_SCALARS, n, 1, 65, 4)
    else:
        n, wc = 2 * 16384 + 5, 10
        s = seeded_scalars(c.name, n, 78, kind="bits")
    W, D, B = eccmi.bucket_geometry(c.cid, wc)
    counts, offsets, srt = empty32(B + 1), empty32(B + 1), empty32(n * W)
    eccmi.ecc_test_bucket_sort(ctx, c.cid, dev(s), n, wc, counts, offsets, srt, method=2)
    counts, offsets, srt = host32(counts), host32(offsets), host32(srt)
    if case == "equal_scalars":
        lists = {b: [(i, sg) for i in range(n)] for b, v in ref.bucket_lists([syn.limbs_to_int(one[0])], wc, W).items()
                 for (_, sg) in v}
    else:
        lists = ref.bucket_lists([syn.limbs_to_int(r) for r in s], wc, W)
    exp_counts = np.zeros(B + 1, dtype=np.uint32)
    for b, v in lists.items():
        exp_counts[b] = len(v)
    assert np.array_equal(counts, exp_counts)
    assert np.array_equal(offsets, np.concatenate([[0], np.cumsum(exp_counts[:B])]).astype(np.uint32))
    for b, v in lists.items():
        seg = srt[offsets[b]: offsets[b] + counts[b]]
        assert sorted((int(e) & 0x7FFFFFFF, bool(int(e) >> 31)) for e in seg) == v


# ---- fixed-base multiplication (the seeded base generator) -------------------

@pytest.mark.parametrize("c", ALL_CURVES, ids=lambda c: c.name)
def test_fixed_base_parity(ctx, c):
    n = 1000
    k = syn.uniform_range(31, syn.TAG_BASE_DLOG, n, 1, c.r, 4)
    edge = syn.ints_to_limbs([0, 1, 2, c.r - 1, c.r, c.r + 1, (1 << 256) - 1], 4)
    k = np.concatenate([edge, k])
    out = empty64(k.shape[0] * 2 * c.limbs)
    eccmi.ecc_fixed_base_mul(ctx, c.cid, dev(k), k.shape[0], out)
    got = host64(out).reshape(-1, 2 * c.limbs)
    exp = co.fixed_base(c.cid, c.limbs, k)
    assert np.array_equal(got, exp)


# ---- MSM ------------------------------------------------------------------------

def test_msm_bn254_2p12_montgomery_input(ctx):
    """BN254, N = 2^12, k_i in [1, r), scalars in [0, r), bases given in
    Montgomery form."""
    c = curves.BN254
    n = 1 << 12
    k, bases = seeded_bases(c.name, n, 0xECC0)
    s = seeded_scalars(c.name, n, 0xECC0)
    mont = points_to_rows(c, [(ref.to_montgomery(c, P[0]), ref.to_montgomery(c, P[1]))
                              for P in rows_to_points(c, bases)])
    got = run_msm(ctx, c, mont, s, flags=eccmi.ECC_IN_MONTGOMERY)
    assert got == oracle_msm(c, bases, s)
    assert got == dlog_msm_expected(c, k, s)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 64, 333, 2500])
def test_msm_sizes(ctx, c, n):
    k, bases = seeded_bases(c.name, max(n, 1), 40 + n)
    bases = bases[:n]
    s = seeded_scalars(c.name, n, 41 + n, kind="bits")
    got = run_msm(ctx, c, bases, s)
    assert got == oracle_msm(c, bases, s)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_msm_graph_replay(ctx, c):
    """A single MSM captured as a graph (its rounds, the finishing pass and
    the reduction read their parameters on the device) and replayed three
    times with eager calls in between, then once more after new scalars were
    written into the same buffer: every replay equals the oracle's MSM."""
    n = 20000
    k, bases = seeded_bases(c.name, n, 0x6A)
    s = seeded_scalars(c.name, n, 0x6B, kind="bits")
    bd, sd = dev(bases), dev(s)
    want = dlog_msm_expected(c, k, s)
    out = empty64(2 * c.limbs)
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")

    def call(flags):
        eccmi.ecc_msm(ctx, c.cid, bd, sd, n, out, inf, flags=flags)
        torch.cuda.synchronize()
        return rows_to_points(c, host64(out).reshape(1, -1), inf.cpu().numpy())[0]

    for rep in range(3):
        assert call(eccmi.ECC_USE_GRAPH) == want, rep
        assert run_msm(ctx, c, bases[:300], s[:300]) == oracle_msm(c, bases[:300], s[:300])
    s2 = seeded_scalars(c.name, n, 0x6C, kind="bits")
    sd.copy_(dev(s2))
    assert call(eccmi.ECC_USE_GRAPH) == dlog_msm_expected(c, k, s2)
    assert call(0) == dlog_msm_expected(c, k, s2)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
@pytest.mark.parametrize("wc", [2, 3, 7, 11])
def test_msm_window_widths(ctx, c, wc):
    n = 700
    k, bases = seeded_bases(c.name, n, 50)
    s = seeded_scalars(c.name, n, 51, kind="bits")
    assert run_msm(ctx, c, bases, s, window_c=wc) == oracle_msm(c, bases, s)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_msm_skewed_top_window(ctx, c):
    """c = 14 over the split's half-length scalars: the top window holds two
    or three bits of every scalar, so a few buckets take thousands of points
    (more than 256 pairs in a round, written by the whole planning
    workgroup; several such buckets share one workgroup)."""
    n = 3000
    k, bases = seeded_bases(c.name, n, 52)
    s = seeded_scalars(c.name, n, 53, kind="bits")
    assert run_msm(ctx, c, bases, s, window_c=14) == oracle_msm(c, bases, s)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_msm_adversarial(ctx, c):
    k, bases = seeded_bases(c.name, 300, 60)
    pts = rows_to_points(c, bases)
    top = (1 << c.scalar_bits) - 1
    # every point in the same bucket of every window
    same = syn.ints_to_limbs([0x1234567890ABCDEF1122334455667788] * 300, 4)
    assert run_msm(ctx, c, bases, same) == oracle_msm(c, bases, same)
    # duplicated and negated bases: sums collide inside buckets (doublings, P + (-P))
    dup_pts = pts[:50] * 3 + [ref.neg(c, P) for P in pts[:50]] + [None] * 10
    dup = points_to_rows(c, dup_pts)
    sd = syn.ints_to_limbs([7] * 100 + [7] * 50 + [7] * 50 + [5] * 10, 4)
    assert run_msm(ctx, c, dup, sd) == oracle_msm(c, dup, sd)
    sd2 = seeded_scalars(c.name, len(dup_pts), 61, kind="bits")
    sd2[:50] = sd2[150:200]  # P and -P with equal scalars cancel
    assert run_msm(ctx, c, dup, sd2) == oracle_msm(c, dup, sd2)
    # extreme scalars and zeros
    ext = syn.ints_to_limbs([0, top, 1, c.r - 1, c.r, 1 << (c.scalar_bits - 1)] * 50, 4)
    assert run_msm(ctx, c, bases, ext) == oracle_msm(c, bases, ext)
    zeros = syn.ints_to_limbs([0] * 300, 4)
    assert run_msm(ctx, c, bases, zeros) is None
    # a sum that is exactly O: s P + (r - s) P
    two = points_to_rows(c, [pts[0], pts[0]])
    assert run_msm(ctx, c, two, syn.ints_to_limbs([12345, c.r - 12345], 4)) is None


# The endomorphism (x, y) -> (beta x, y) acts on the order-r subgroup as
# multiplication by a cube root of unity lambda mod r; a single MSM splits each
# scalar as k = k1 + lambda k2 with Babai rounding of k |b| / r against a short
# lattice basis, whose |b| entries are listed here (the rounding steps where
# k |b| / r crosses a half-integer).
SPLIT = {
    "bn254": (0xb3c4d79d41a917585bfc41088d8daaa78b17ea66b99c90dd,
              [0x89d3256894d213e3, 0x6f4d8248eeb859fc8211bbeb7d4f1128]),
    "bls12_381": (0xac45a4010001a40200000000ffffffff, [1, 0xac45a4010001a4020000000100000000]),
}


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_msm_endomorphism_split_edge_scalars(ctx, c):
    """Scalars at the edges of the split: lambda, its neighbours and multiples,
    the steps of the Babai rounding, and scalars >= r."""
    lam, dens = SPLIT[c.name]
    assert pow(lam, 3, c.r) == 1 and lam != 1
    top = (1 << c.scalar_bits) - 1
    edge = [0, 1, 2, lam - 1, lam, lam + 1, lam * lam % c.r, lam // 2, lam // 2 + 1, c.r - lam,
            c.r - 1, c.r, c.r + 1, top - 1, top]
    edge += [j * lam for j in (2, 3, 1000, (1 << 64) + 1)]
    for b in dens:
        for j in (0, 1, 7, 1 << 40, b // 3):
            mid = (2 * j + 1) * c.r // (2 * b)
            edge += [mid - 1, mid, mid + 1]
    edge = sorted({e for e in edge if 0 <= e <= top})
    n = len(edge)
    k, bases = seeded_bases(c.name, n, 62)
    s = syn.ints_to_limbs(edge, 4)
    assert run_msm(ctx, c, bases, s) == oracle_msm(c, bases, s)
    for j in range(n):
        assert run_msm(ctx, c, bases[j:j + 1], s[j:j + 1]) == oracle_msm(c, bases[j:j + 1], s[j:j + 1]), hex(edge[j])


def bls_points_outside_g1(n: int, x0: int):
    """Curve points (x, sqrt(x^3 + 4)) for x = x0, x0 + 1, ...: almost surely
    outside the order-r subgroup (the cofactor of BLS12-381 G1 is about 2^126)."""
    c = curves.BLS12_381
    p = c.p
    out = []
    x = x0
    while len(out) < n:
        rhs = (x * x * x + 4) % p
        y = pow(rhs, (p + 1) // 4, p)  # p = 3 mod 4
        if y * y % p == rhs:
            out.append((x, y))
        x += 1
    return out


def test_msm_no_endomorphism_flag(ctx):
    """Bases outside G1 need ECC_NO_ENDOMORPHISM; on G1 the flag changes nothing."""
    c = curves.BLS12_381
    pts = bls_points_outside_g1(40, 5)
    assert all(ref.on_curve(c, P) for P in pts)
    assert all(ref.scalar_mul(c, c.r, P) is not None for P in pts[:3])
    rows = points_to_rows(c, pts)
    s = seeded_scalars(c.name, 40, 64, kind="bits")
    want = oracle_msm(c, rows, s)
    assert run_msm(ctx, c, rows, s, flags=eccmi.ECC_NO_ENDOMORPHISM) == want
    assert run_msm(ctx, c, rows, s) != want  # the split assumes the order-r subgroup
    k, g1 = seeded_bases(c.name, 40, 63)
    exp = oracle_msm(c, g1, s)
    assert run_msm(ctx, c, g1, s, flags=eccmi.ECC_NO_ENDOMORPHISM) == exp
    assert run_msm(ctx, c, g1, s) == exp


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_msm_errors_leave_outputs_untouched(ctx, c):
    k, bases = seeded_bases(c.name, 64, 70)
    s = seeded_scalars(c.name, 64, 71, kind="bits")
    out = torch.full((2 * c.limbs,), 77, dtype=torch.int64, device="cuda")
    inf = torch.full((1,), 9, dtype=torch.uint8, device="cuda")

    def call(b, sc, flags=0):
        with pytest.raises(eccmi.EccError) as e:
            eccmi.ecc_msm(ctx, c.cid, dev(b), dev(sc), b.shape[0], out, inf, flags=flags)
        assert torch.all(out == 77) and int(inf[0]) == 9
        return e.value.name

    big = s.copy()
    big[5] = syn.ints_to_limbs([1 << c.scalar_bits], 4)[0]
    assert call(bases, big) == "ECC_ERR_RANGE"
    bad = bases.copy()
    bad[3, : c.limbs] = syn.ints_to_limbs([c.p], c.limbs)[0]
    assert call(bad, s) == "ECC_ERR_RANGE"
    off = bases.copy()
    off[7, c.limbs] ^= np.uint64(1)
    assert call(off, s, eccmi.ECC_CHECK_ON_CURVE) == "ECC_ERR_NOT_ON_CURVE"
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_msm(ctx, c.cid, dev(bases), dev(s), 64, out, inf, window_c=25)
    assert e.value.name == "ECC_ERR_ARG"
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_msm(ctx, curves.SECP256R1.cid, dev(bases), dev(s), 64, out, inf)
    assert e.value.name == "ECC_ERR_UNSUPPORTED"


def test_msm_host_pointers(ctx):
    c = curves.BLS12_381
    k, bases = seeded_bases(c.name, 200, 80)
    s = seeded_scalars(c.name, 200, 81, kind="bits")
    out = np.zeros(2 * c.limbs, dtype=np.uint64)
    inf = np.zeros(1, dtype=np.uint8)
    eccmi.ecc_msm(ctx, c.cid, np.ascontiguousarray(bases), np.ascontiguousarray(s), 200, out, inf)
    assert rows_to_points(c, out.reshape(1, -1), inf)[0] == oracle_msm(c, bases, s)


def test_msm_bls12_381_2p20_full_size(ctx):
    """BLS12-381 G1, N = 2^20, uniform 255-bit scalars, window 16 (the timed
    configuration).  Bases P_i = k_i G come from the GPU's fixed-base kernel
    (sampled rows checked against the oracle); the result is checked exactly
    through sum_i s_i k_i G = (sum_i s_i k_i mod r) G."""
    c = curves.BLS12_381
    n = 1 << 20
    k = syn.uniform_range(0xECC2, syn.TAG_BASE_DLOG, n, 1, c.r, 4)
    s = syn.uniform_bits(0xECC2, syn.TAG_SCALARS, n, 255, 4)
    kd = dev(k)
    bases = empty64(n * 2 * c.limbs)
    eccmi.ecc_fixed_base_mul(ctx, c.cid, kd, n, bases)
    idx = syn.choice_indices(7, syn.TAG_MISC, n, 48)
    hb = host64(bases).reshape(n, 2 * c.limbs)
    assert np.array_equal(hb[idx], co.fixed_base(c.cid, c.limbs, k[idx]))
    out = empty64(2 * c.limbs)
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
    eccmi.ecc_msm(ctx, c.cid, bases, dev(s), n, out, inf, window_c=16)
    got = rows_to_points(c, host64(out).reshape(1, -1), inf.cpu().numpy())[0]
    assert got == dlog_msm_expected(c, k, s)
