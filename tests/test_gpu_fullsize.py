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
    kb = np.ascontiguousarray(k).view(np.uint8).reshape(-1, 32)
    sb = np.ascontiguousarray(s).view(np.uint8).reshape(-1, 32)
    acc = 0
    frm = int.from_bytes
    for i in range(kb.shape[0]):
        acc += frm(kb[i].tobytes(), "little") * frm(sb[i].tobytes(), "little")
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
