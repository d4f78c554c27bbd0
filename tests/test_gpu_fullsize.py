"""MSM parity at the full workload sizes, in the configuration the benchmark
times: bases P_i = k_i G made by the GPU fixed-base kernel (sampled rows
checked against the oracle), results checked exactly through the identity
sum_i s_i (k_i G) = (sum_i s_i k_i mod r) G, whose right side the oracle
computes as one scalar multiplication."""

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves, ref
from tests.common import rows_to_points

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.close()


def dlog_expected(c, k: np.ndarray, s: np.ndarray):
    """(sum_i s_i k_i mod r) G, with the products summed in Python integers."""
    from tests.common import limbs_to_objects
    acc = int((limbs_to_objects(k) * limbs_to_objects(s)).sum())
    return ref.scalar_mul(c, acc % c.r, ref.generator(c))


def full_size_case(ctx, c, log2n, window, seed, kind):
    n = 1 << log2n
    k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, n, 1, c.r, 4)
    if kind == "bits":
        s = syn.uniform_bits(seed, syn.TAG_SCALARS, n, c.scalar_bits, 4)
    else:
        s = syn.uniform_below(seed, syn.TAG_SCALARS, n, c.r, 4)
    kd = torch.from_numpy(k.view(np.int64)).cuda()
    bases = torch.empty(n * 2 * c.limbs, dtype=torch.int64, device="cuda")
    eccmi.ecc_fixed_base_mul(ctx, c.cid, kd, n, bases)
    del kd
    idx = syn.choice_indices(seed + 1, syn.TAG_MISC, n, 32)
    hb = bases.view(-1, 2 * c.limbs)[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
    assert np.array_equal(hb, co.fixed_base(c.cid, c.limbs, k[idx]))
    out = torch.zeros(2 * c.limbs, dtype=torch.int64, device="cuda")
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
    sd = torch.from_numpy(s.view(np.int64)).cuda()
    eccmi.ecc_msm(ctx, c.cid, bases, sd, n, out, inf, window_c=window)
    got = rows_to_points(c, out.cpu().numpy().view(np.uint64).reshape(1, -1), inf.cpu().numpy())[0]
    del bases, sd
    assert got == dlog_expected(c, k, s)


@pytest.mark.parametrize("log2n", [16, 20, 22])
def test_bn254_plain_window16(ctx, log2n):
    full_size_case(ctx, curves.BN254, log2n, 16, 0xB254 + log2n, "mod_r")


@pytest.mark.parametrize("log2n", [16, 24])
def test_bls12_381_library_window(ctx, log2n):
    full_size_case(ctx, curves.BLS12_381, log2n, 0, 0xB15 + log2n, "bits")


def test_batch_uneven_4096_full_size(ctx):
    """The benchmark's uneven batch exactly as bench.py draws it (4096 BLS12-381
    MSMs, sizes log-uniform in [2, 2^14], seed 0xBA7C, bases k_i G from the GPU
    fixed-base kernel, uniform 255-bit scalars), as one captured launch
    sequence: every one of the 4096 results, on capture and on replay, equals
    (sum over the MSM of s_i k_i mod r) G from the oracle."""
    from tests.common import dlog_batch_expected
    c = curves.BLS12_381
    seed, m = 0xBA7C, 4096
    sizes = syn.log_uniform_sizes(seed, syn.TAG_SIZES, m, 1.0, 14.0)
    offs = np.zeros(m + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    total = int(offs[-1])
    assert sizes.min() >= 2 and sizes.max() <= 1 << 14 and total > 6_000_000
    k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, total, 1, c.r, 4)
    s = syn.uniform_bits(seed, syn.TAG_SCALARS, total, c.scalar_bits, 4)
    kd = torch.from_numpy(k.view(np.int64)).cuda()
    bases = torch.empty(total * 2 * c.limbs, dtype=torch.int64, device="cuda")
    eccmi.ecc_fixed_base_mul(ctx, c.cid, kd, total, bases)
    del kd
    idx = syn.choice_indices(seed + 1, syn.TAG_MISC, total, 32)
    hb = bases.view(-1, 2 * c.limbs)[torch.from_numpy(idx.astype(np.int64)).cuda()].cpu().numpy().view(np.uint64)
    assert np.array_equal(hb, co.fixed_base(c.cid, c.limbs, k[idx]))
    want = dlog_batch_expected(c, k, s, offs)
    want_inf = ~want.any(axis=1)
    sd = torch.from_numpy(s.view(np.int64)).cuda()
    out = torch.zeros(m * 2 * c.limbs, dtype=torch.int64, device="cuda")
    inf = torch.zeros(m, dtype=torch.uint8, device="cuda")
    for rep in range(2):  # capture, then replay
        out.fill_(7)
        inf.fill_(7)
        eccmi.ecc_msm_batch(ctx, c.cid, bases, sd, offs, out, inf, flags=eccmi.ECC_USE_GRAPH)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64).reshape(m, 2 * c.limbs)
        gi = inf.cpu().numpy().astype(bool)
        bad = np.nonzero((got != want).any(axis=1) | (gi != want_inf))[0]
        assert bad.size == 0, f"replay {rep}: {bad.size} MSMs differ, first {bad[:8].tolist()}"
    del bases, sd


@pytest.mark.parametrize("form", [eccmi.ECC_VERIFY_PER_LANE, eccmi.ECC_VERIFY_BATCHED], ids=["per_lane", "batched"])
def test_verify_across_launch_chunk(ctx, form):
    """2^16 + 257 secp256r1 verifications in one call: the per-lane form splits
    them at 2^16 requests per launch.  Requests are drawn (seeded, with
    repetition) from the oracle-made request file, whose verdicts the oracle
    computed, so every verdict is known; the draw makes a misplaced chunk
    offset visible."""
    import os
    req = np.load(os.path.join(os.path.dirname(__file__), "golden", "p256_requests.npz"))
    H, Q, S, V = req["hashes"], req["pubkeys"], req["sigs"], req["valid"]
    m = (1 << 16) + 257
    pick = (syn.u64(0xC4A, syn.TAG_MISC, m) % np.uint64(H.shape[0])).astype(np.int64)
    h = torch.from_numpy(np.ascontiguousarray(H[pick])).cuda()
    q = torch.from_numpy(np.ascontiguousarray(Q[pick]).view(np.int64)).cuda()
    sg = torch.from_numpy(np.ascontiguousarray(S[pick]).view(np.int64)).cuda()
    v = torch.full((m,), 7, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch(ctx, curves.SECP256R1.cid, h, q, sg, m, v, flags=form)
    got = v.cpu().numpy()
    want = V[pick].astype(np.uint8)
    assert 0 < want.sum() < m
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} verdicts differ, first {bad[:8].tolist()}"
