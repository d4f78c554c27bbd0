"""Behaviour of the C ABI around the computation: ordering with the caller's
stream, asynchronous calls (ECC_ASYNC, ecc_ctx_sync), bases read in place
from per-MSM pointers (ECC_BASES_PER_MSM), and the scratch plan behind HBM
admission (ecc_msm_batch_scratch_bytes).  Every result is checked against the
CPU oracle."""

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves
from tests.common import dlog_batch_expected, seeded_bases, seeded_scalars

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")

C = curves.BLS12_381


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.close()


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).cuda()


def oracle_rows(c, bases, scalars, offs):
    rows = np.zeros((len(offs) - 1, 2 * c.limbs), dtype=np.uint64)
    for j in range(len(offs) - 1):
        a, b = int(offs[j]), int(offs[j + 1])
        if b > a:
            rows[j] = co.msm(c.cid, c.limbs, bases[a:b], scalars[a:b])[0]
    return rows


def test_inputs_written_on_a_busy_side_stream(ctx):
    """Inputs and the output fill are written by torch on a side stream that is
    still busy with earlier work; a call without an explicit stream, made
    while that stream is current, runs after them."""
    n = 3000
    k, bases = seeded_bases(C.name, n, 0x51DE)
    s = seeded_scalars(C.name, n, 0x51DF, kind="bits")
    want, want_inf = co.msm(C.cid, C.limbs, bases, s)
    hb = torch.from_numpy(bases.view(np.int64).reshape(-1)).pin_memory()
    hs = torch.from_numpy(s.view(np.int64).reshape(-1)).pin_memory()
    side = torch.cuda.Stream()
    a = torch.randn(4096, 4096, device="cuda")
    for trial in range(2):
        bd = torch.zeros(hb.numel(), dtype=torch.int64, device="cuda")
        sd = torch.zeros(hs.numel(), dtype=torch.int64, device="cuda")
        out = torch.zeros(2 * C.limbs, dtype=torch.int64, device="cuda")
        inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            for _ in range(20):  # keep the side stream busy
                a = (a @ a).clamp_(-1, 1)
            bd.copy_(hb, non_blocking=True)
            sd.copy_(hs, non_blocking=True)
            out.fill_(-1)
            eccmi.ecc_msm(ctx, C.cid, bd, sd, n, out, inf)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64), want), trial
        assert bool(inf.cpu()[0]) == want_inf


def test_async_calls_and_sync(ctx):
    """ECC_ASYNC calls only enqueue; after ecc_ctx_sync every output equals the
    oracle's.  An asynchronous call whose scalar is out of range reports
    ECC_ERR_RANGE at the sync and leaves its output untouched."""
    n = 1500
    k, bases = seeded_bases(C.name, n, 0xA51)
    s = seeded_scalars(C.name, n, 0xA52, kind="bits")
    bd, sd = dev(bases), dev(s)
    sizes = [1500, 0, 700, 1]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    want1 = co.msm(C.cid, C.limbs, bases, s)[0]
    wantb = oracle_rows(C, np.concatenate([bases, bases[:701]]), np.concatenate([s, s[:701]]), offs)
    bd2, sd2 = dev(np.concatenate([bases, bases[:701]])), dev(np.concatenate([s, s[:701]]))
    stream = torch.cuda.Stream()
    outs = [torch.full((2 * C.limbs,), 5, dtype=torch.int64, device="cuda") for _ in range(3)]
    infs = [torch.zeros(1, dtype=torch.uint8, device="cuda") for _ in range(3)]
    outb = torch.zeros(len(sizes) * 2 * C.limbs, dtype=torch.int64, device="cuda")
    infb = torch.zeros(len(sizes), dtype=torch.uint8, device="cuda")
    for i in range(3):
        eccmi.ecc_msm(ctx, C.cid, bd, sd, n, outs[i], infs[i], flags=eccmi.ECC_ASYNC, stream=stream)
    eccmi.ecc_msm_batch(ctx, C.cid, bd2, sd2, offs, outb, infb, flags=eccmi.ECC_ASYNC, stream=stream)
    ctx.sync()
    for i in range(3):
        assert np.array_equal(outs[i].cpu().numpy().view(np.uint64), want1), i
    got = outb.cpu().numpy().view(np.uint64).reshape(len(sizes), -1)
    assert np.array_equal(got, wantb)
    assert infb.cpu().tolist() == [int(not r.any()) for r in wantb]
    # an input error surfaces at the sync; the output keeps its contents
    bad = s.copy()
    bad[17, 3] = np.uint64(1) << np.uint64(63)  # bit 255: >= 2^255
    bdd = dev(bad)
    o = torch.full((2 * C.limbs,), 9, dtype=torch.int64, device="cuda")
    i1 = torch.full((1,), 9, dtype=torch.uint8, device="cuda")
    eccmi.ecc_msm(ctx, C.cid, bd, bdd, n, o, i1, flags=eccmi.ECC_ASYNC, stream=stream)
    with pytest.raises(eccmi.EccError) as e:
        ctx.sync()
    assert e.value.name == "ECC_ERR_RANGE"
    assert o.cpu().tolist() == [9] * (2 * C.limbs) and i1.cpu().tolist() == [9]
    ctx.sync()  # the error was reported once
    # asynchronous verification
    from tests.common import seeded_signatures
    hashes, pubs, sigs = seeded_signatures(300, 0xA53)
    want_v = co.ecdsa_verify(curves.SECP256R1.cid, hashes, pubs, sigs)
    v = torch.full((300,), 7, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch(ctx, curves.SECP256R1.cid, torch.from_numpy(hashes).cuda(),
                           torch.from_numpy(pubs.view(np.int64)).cuda(), torch.from_numpy(sigs.view(np.int64)).cuda(),
                           300, v, flags=eccmi.ECC_ASYNC, stream=stream)
    ctx.sync()
    assert np.array_equal(v.cpu().numpy().astype(bool), want_v)
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_msm(ctx, C.cid, bases, s, n, np.zeros(2 * C.limbs, dtype=np.uint64), np.zeros(1, dtype=np.uint8),
                      flags=eccmi.ECC_ASYNC)
    assert e.value.name == "ECC_ERR_ARG"  # asynchronous calls take device pointers only


@pytest.mark.parametrize("flags", [0, eccmi.ECC_USE_GRAPH], ids=["eager", "graph"])
def test_bases_per_msm_in_place(ctx, flags):
    """MSMs over ranges of one resident base set, named by per-MSM pointers
    (overlapping, repeated and empty ranges), equal the oracle's MSMs of the
    same ranges; a second call with other ranges of the same sizes reuses a
    captured graph and still reads the new ranges."""
    n = 5000
    k, bases = seeded_bases(C.name, n, 0xB0B)
    bd = dev(bases)
    stride = 2 * C.limbs
    for trial, ranges in enumerate([[(0, 1200), (1000, 1), (4000, 1000), (7, 0), (1000, 1)],
                                    [(3000, 1200), (0, 1), (2000, 1000), (9, 0), (4999, 1)]]):
        sizes = [ln for _, ln in ranges]
        offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
        offs[1:] = np.cumsum(sizes)
        total = int(offs[-1])
        s = seeded_scalars(C.name, total, 0xB0C + trial, kind="bits")
        cat = np.concatenate([bases[a:a + ln] for a, ln in ranges])
        want = oracle_rows(C, cat, s, offs)
        flat = bd.reshape(-1)
        ptrs = [flat[a * stride:].data_ptr() for a, _ in ranges]
        out = torch.zeros(len(sizes) * stride, dtype=torch.int64, device="cuda")
        inf = torch.zeros(len(sizes), dtype=torch.uint8, device="cuda")
        eccmi.ecc_msm_batch(ctx, C.cid, ptrs, dev(s), offs, out, inf, flags=flags)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint64).reshape(len(sizes), -1), want), trial
        assert inf.cpu().tolist() == [int(not r.any()) for r in want]


def test_scratch_plan_matches_budget(ctx):
    """A context whose HBM budget is exactly the planned scratch of a batch runs
    that batch (results equal the oracle's); a budget 64 KiB below the plan
    fails with ECC_ERR_NOMEM and leaves the outputs untouched."""
    sizes = [2000, 33, 700]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    total = int(offs[-1])
    k, bases = seeded_bases(C.name, total, 0x5C4)
    s = seeded_scalars(C.name, total, 0x5C5, kind="bits")
    want = oracle_rows(C, bases, s, offs)
    plan = eccmi.ecc_msm_batch_scratch_bytes(ctx, C.cid, offs)
    assert plan > 0
    stride = 2 * C.limbs
    for budget, ok in ((plan, True), (plan - (64 << 10), False)):
        with eccmi.Context(0, hbm_budget_bytes=budget) as c2:
            out = torch.full((len(sizes) * stride,), 3, dtype=torch.int64, device="cuda")
            inf = torch.full((len(sizes),), 3, dtype=torch.uint8, device="cuda")
            if ok:
                eccmi.ecc_msm_batch(c2, C.cid, dev(bases), dev(s), offs, out, inf)
                assert np.array_equal(out.cpu().numpy().view(np.uint64).reshape(len(sizes), -1), want)
                assert c2.scratch_bytes() <= budget
            else:
                with pytest.raises(eccmi.EccError) as e:
                    eccmi.ecc_msm_batch(c2, C.cid, dev(bases), dev(s), offs, out, inf)
                assert e.value.name == "ECC_ERR_NOMEM"
                assert out.cpu().tolist() == [3] * (len(sizes) * stride)
