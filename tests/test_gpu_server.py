"""The request server (continuous batching): each result of a mixed stream of
MSM and verification requests equals the request's result alone and the
oracle's, whatever else was batched with it."""

import time

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves
from tests.common import rows_to_points, seeded_bases, seeded_scalars, seeded_signatures

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")


def test_served_mix_matches_alone_and_oracle():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B = curves.BLS12_381
    P = curves.SECP256R1
    nb = 6000
    k, bases = seeded_bases(B.name, nb, 500)
    sizes = syn.log_uniform_sizes(501, syn.TAG_SIZES, 14, 4.0, 12.0)
    firsts = (syn.u64(502, syn.TAG_MISC, 14) % np.uint64(nb - 4096)).astype(np.int64)
    scal = [seeded_scalars(B.name, int(n), 510 + j, kind="bits") for j, n in enumerate(sizes)]
    hashes, pubs, sigs = seeded_signatures(400, 520)
    gaps = syn.exponential_gaps(503, syn.TAG_ARRIVALS, 414, 0.0004)

    srv = eccmi.Server(0, slots=2, max_batch_points=1 << 16, max_batch_verify=128)
    try:
        bid = srv.add_bases(B.cid, bases)
        tickets = []
        vi = mi = 0
        for step in range(414):
            if step % 30 == 7 and mi < len(sizes):
                tickets.append(("msm", mi, srv.submit_msm(bid, int(firsts[mi]), scal[mi])))
                mi += 1
            elif vi < 400:
                tickets.append(("verify", vi, srv.submit_verify(hashes[vi], pubs[vi], sigs[vi])))
                vi += 1
            time.sleep(float(gaps[step]))
        while mi < len(sizes):
            tickets.append(("msm", mi, srv.submit_msm(bid, int(firsts[mi]), scal[mi])))
            mi += 1
        got_v = np.zeros(400, dtype=bool)
        got_m = {}
        for kind, i, t in tickets:
            xy, flag, lat = srv.wait(t)
            assert lat >= 0
            if kind == "verify":
                got_v[i] = bool(flag)
            else:
                got_m[i] = rows_to_points(B, xy.reshape(1, -1), np.array([flag]))[0]
        st = srv.stats()
    finally:
        srv.close()
    assert st["done_verify"] == 400 and st["done_msm"] == len(sizes)
    assert st["batches"] >= 2 and st["p99_verify_ms"] >= st["p50_verify_ms"] > 0

    # verification: equal to the oracle and to single-request calls
    want_v = co.ecdsa_verify(P.cid, hashes, pubs, sigs)
    assert np.array_equal(got_v, want_v)
    ctx = eccmi.Context(0)
    try:
        for i in range(0, 400, 37):
            v = np.zeros(1, dtype=np.uint8)
            eccmi.ecc_verify_batch(ctx, P.cid, hashes[i:i + 1], pubs[i:i + 1], sigs[i:i + 1], 1, v)
            assert bool(v[0]) == got_v[i]
        # MSMs: equal to the oracle and to ecc_msm alone
        for j, n in enumerate(sizes):
            lo = int(firsts[j])
            b = bases[lo:lo + int(n)]
            out, inf = co.msm(B.cid, B.limbs, b, scal[j])
            assert got_m[j] == rows_to_points(B, out.reshape(1, -1), np.array([inf]))[0]
            o = np.zeros(2 * B.limbs, dtype=np.uint64)
            f = np.zeros(1, dtype=np.uint8)
            eccmi.ecc_msm(ctx, B.cid, np.ascontiguousarray(b), np.ascontiguousarray(scal[j]), int(n), o, f)
            assert rows_to_points(B, o.reshape(1, -1), f)[0] == got_m[j]
    finally:
        ctx.close()


def test_served_msms_under_a_budget_that_splits_batches():
    """An HBM budget that holds the scratch of about two of the queued MSMs per
    slot: admission forms several batches from one burst, and every result
    still equals the oracle's and the request's result alone."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B = curves.BLS12_381
    nb = 9000
    k, bases = seeded_bases(B.name, nb, 530)
    sizes = [int(x) for x in syn.log_uniform_sizes(531, syn.TAG_SIZES, 10, 10.0, 13.0)]
    firsts = [int(x) for x in (syn.u64(532, syn.TAG_MISC, 10) % np.uint64(nb - 8192))]
    scal = [seeded_scalars(B.name, n, 540 + j, kind="bits") for j, n in enumerate(sizes)]
    with eccmi.Context(0) as ctx:
        one = max(eccmi.ecc_msm_batch_scratch_bytes(ctx, B.cid, [0, n], flags=eccmi.ECC_BASES_PER_MSM)
                  for n in sizes)
        two = max(eccmi.ecc_msm_batch_scratch_bytes(ctx, B.cid, [0, sizes[j], sizes[j] + sizes[j + 1]],
                                                    flags=eccmi.ECC_BASES_PER_MSM) for j in range(9))
        allb = eccmi.ecc_msm_batch_scratch_bytes(ctx, B.cid, np.concatenate([[0], np.cumsum(sizes)]),
                                                 flags=eccmi.ECC_BASES_PER_MSM)
    share = max(one, two) + (1 << 20)
    assert share < allb  # the whole burst does not fit one slot's share
    srv = eccmi.Server(0, slots=2, hbm_budget_bytes=2 * share, max_batch_points=1 << 20)
    try:
        bid = srv.add_bases(B.cid, bases)
        tickets = [srv.submit_msm(bid, firsts[j], scal[j]) for j in range(10)]
        got = []
        for t in tickets:
            xy, flag, lat = srv.wait(t)
            got.append(rows_to_points(B, xy.reshape(1, -1), np.array([flag]))[0])
        st = srv.stats()
    finally:
        srv.close()
    assert st["done_msm"] == 10 and st["batches"] >= 3
    with eccmi.Context(0) as ctx:
        for j, n in enumerate(sizes):
            b = bases[firsts[j]:firsts[j] + n]
            out, inf = co.msm(B.cid, B.limbs, b, scal[j])
            assert got[j] == rows_to_points(B, out.reshape(1, -1), np.array([inf]))[0], j
            o = np.zeros(2 * B.limbs, dtype=np.uint64)
            f = np.zeros(1, dtype=np.uint8)
            eccmi.ecc_msm(ctx, B.cid, np.ascontiguousarray(b), np.ascontiguousarray(scal[j]), n, o, f)
            assert rows_to_points(B, o.reshape(1, -1), f)[0] == got[j]
