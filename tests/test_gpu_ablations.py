"""The design variants of the bucket rounds (ecc_ctx_set_round_variant:
stored denominators, per-lane chain layout, unfused decompress and additions,
per-lane inversion; the finishing pass for batches too, or rounds to the end
for every call) give exactly the oracle's MSM, on seeded and adversarial
BLS12-381 inputs that take every exceptional lane class; and the variant
knob's argument checks."""

import numpy as np
import pytest

from oracle import curves, ref
from tests.common import oracle_msm, points_to_rows, rows_to_points, seeded_bases, seeded_scalars
import synthetic as syn

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")

C = curves.BLS12_381
VARIANTS = [1, 2, 3, 4, 7, 8, 64, 16, 32, 1 | 32, 8 | 16, 64 | 32]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.set_round_variant(0)
    c.close()


def _msm(ctx, bases, scalars, window_c=0):
    n = bases.shape[0]
    b = torch.from_numpy(np.ascontiguousarray(bases).view(np.int64).copy()).cuda()
    s = torch.from_numpy(np.ascontiguousarray(scalars).view(np.int64).copy()).cuda()
    out = torch.zeros(2 * C.limbs, dtype=torch.int64, device="cuda")
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
    eccmi.ecc_msm(ctx, C.cid, b, s, n, out, inf, window_c=window_c)
    torch.cuda.synchronize()
    return rows_to_points(C, out.cpu().numpy().view(np.uint64).reshape(1, -1), inf.cpu().numpy())[0]


@pytest.mark.parametrize("variant", VARIANTS)
def test_round_variant_matches_oracle(ctx, variant):
    k, bases = seeded_bases(C.name, 3000, 81)
    s = seeded_scalars(C.name, 3000, 82, kind="bits")
    want = oracle_msm(C, bases, s)
    ctx.set_round_variant(variant)
    try:
        # a narrow window makes deep buckets: several rounds, chains of several additions per lane
        assert _msm(ctx, bases, s, window_c=7) == want
        assert _msm(ctx, bases, s) == want
        # duplicated and negated bases: doublings, P + (-P) and infinity inside the rounds
        pts = rows_to_points(C, bases[:60])
        dup_pts = pts * 3 + [ref.neg(C, P) for P in pts] + [None] * 8
        dup = points_to_rows(C, dup_pts)
        sd = syn.ints_to_limbs([9] * len(dup_pts), 4)
        assert _msm(ctx, dup, sd) == oracle_msm(C, dup, sd)
    finally:
        ctx.set_round_variant(0)


def test_round_variant_argument_checks(ctx):
    for bad in (5, 16 | 32, 128, 64 | 1, -1):
        with pytest.raises(eccmi.EccError) as e:
            ctx.set_round_variant(bad)
        assert e.value.name == "ECC_ERR_ARG"
    ctx.set_round_variant(1)
    try:
        b = torch.zeros(8, dtype=torch.int64, device="cuda")
        out = torch.zeros(8, dtype=torch.int64, device="cuda")
        inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
        with pytest.raises(eccmi.EccError) as e:
            eccmi.ecc_msm(ctx, curves.BN254.cid, b, b[:4], 1, out, inf)
        assert e.value.name == "ECC_ERR_UNSUPPORTED"
    finally:
        ctx.set_round_variant(0)


@pytest.mark.parametrize("variant", [16, 32])
def test_finishing_pass_on_bn254_and_batches(ctx, variant):
    """The per-lane finishing pass for batches too (16) and the rounds run to
    the end for single MSMs too (32) on BN254; deep buckets (narrow window)
    make the finishing pass take over after a few rounds."""
    from tests.test_gpu_batch import oracle_batch, run_batch
    c = curves.BN254
    k, bases = seeded_bases(c.name, 4000, 83)
    s = seeded_scalars(c.name, 4000, 84, kind="bits")
    want = oracle_msm(c, bases, s)
    ctx.set_round_variant(variant)
    try:
        out = torch.zeros(2 * c.limbs, dtype=torch.int64, device="cuda")
        inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
        for wc in (5, 0):
            eccmi.ecc_msm(ctx, c.cid, torch.from_numpy(bases.view(np.int64).copy()).cuda(),
                          torch.from_numpy(s.view(np.int64).copy()).cuda(), 4000, out, inf, window_c=wc)
            torch.cuda.synchronize()
            got = rows_to_points(c, out.cpu().numpy().view(np.uint64).reshape(1, -1), inf.cpu().numpy())[0]
            assert got == want, wc
        offs = np.array([0, 1500, 1500, 4000], dtype=np.uint64)
        assert run_batch(ctx, c, bases, s, offs, window_c=4) == oracle_batch(c, bases, s, offs)
    finally:
        ctx.set_round_variant(0)


def test_profile_stats_count_the_round_additions(ctx):
    """With profiling on, the stats count every batch-affine addition of the
    rounds run: with the rounds run to the end, exactly sum_b (n_b - 1) over
    the oracle's bucket lists; with the finishing pass, the additions of the
    rounds before the hand-over, its time apart.  The phases fit in the
    call's total time."""
    c = C
    n, wc = 8192, 10
    k, bases = seeded_bases(c.name, n, 91)
    s = seeded_scalars(c.name, n, 92, kind="bits")
    W, D, B = eccmi.bucket_geometry(c.cid, wc)
    lists = ref.bucket_lists([syn.limbs_to_int(r) for r in s], wc, W)
    total = sum(len(v) - 1 for v in lists.values())
    want = oracle_msm(c, bases, s)
    bd = torch.from_numpy(np.ascontiguousarray(bases).view(np.int64).copy()).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(s).view(np.int64).copy()).cuda()
    out = torch.zeros(2 * c.limbs, dtype=torch.int64, device="cuda")
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
    got = {}
    try:
        for variant in (0, eccmi.RV_ROUNDS_ONLY):
            ctx.set_round_variant(variant)
            ctx.set_profiling(True)
            eccmi.ecc_msm(ctx, c.cid, bd, sd, n, out, inf, flags=eccmi.ECC_NO_ENDOMORPHISM, window_c=wc)
            torch.cuda.synchronize()
            got[variant] = ctx.stats()
            ctx.set_profiling(False)
            res = rows_to_points(c, out.cpu().numpy().view(np.uint64).reshape(1, -1), inf.cpu().numpy())[0]
            assert res == want, variant
    finally:
        ctx.set_profiling(False)
        ctx.set_round_variant(0)
    full, dflt = got[eccmi.RV_ROUNDS_ONLY], got[0]
    assert full["msm_calls"] == 1 and full["points"] == n
    assert full["round_adds"] == total and full["finish_ms"] == 0.0
    if dflt["round_launches"] < full["round_launches"]:
        assert 0 < dflt["round_adds"] < total and dflt["finish_ms"] > 0.0
    else:
        assert dflt["round_adds"] == total and dflt["finish_ms"] == 0.0
    for st in (full, dflt):
        parts = st["prepare_ms"] + st["round_ms"] + st["finish_ms"] + st["reduce_ms"] + st["combine_ms"]
        assert 0.0 < parts <= st["total_ms"] * 1.01 + 0.01
