"""Parity of batched ECDSA signing (secp256r1 and SM2) with the CPU oracle.

Each signature (r, s) is compared word for word with the oracle's for the
same key, nonce and hash; out-of-range keys and nonces give all-zero rows on
both sides.  The signatures also pass the library's own verification."""

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")

SIGN_CURVES = [curves.SECP256R1, curves.SM2]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.close()


def seeded_sign_requests(c, m: int, seed: int):
    d = syn.uniform_range(seed, syn.TAG_KEYS, m, 1, c.r, 4)
    k = syn.uniform_range(seed, syn.TAG_NONCES, m, 1, c.r, 4)
    h = syn.random_bytes(seed, syn.TAG_HASH, m, 32)
    return h, d, k


def gpu_sign(ctx, c, h, d, k):
    m = h.shape[0]
    ht = torch.from_numpy(np.ascontiguousarray(h)).cuda()
    dt = torch.from_numpy(np.ascontiguousarray(d, dtype=np.uint64).view(np.int64)).cuda()
    kt = torch.from_numpy(np.ascontiguousarray(k, dtype=np.uint64).view(np.int64)).cuda()
    out = torch.full((max(1, m) * 8,), -1, dtype=torch.int64, device="cuda")
    eccmi.ecc_sign_batch(ctx, c.cid, ht, dt, kt, m, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64).reshape(-1, 8)[:m]


@pytest.mark.parametrize("c", SIGN_CURVES, ids=lambda c: c.name)
@pytest.mark.parametrize("m", [1, 255, 257, 2000])
def test_sign_seeded_requests(ctx, c, m):
    h, d, k = seeded_sign_requests(c, m, 1200 + m)
    want = co.ecdsa_sign(c.cid, h, d, k)
    got = gpu_sign(ctx, c, h, d, k)
    assert np.array_equal(got, want)
    # the signatures verify under Q = d G, in the library and in the oracle
    Q = co.fixed_base(c.cid, c.limbs, d)
    assert co.ecdsa_verify(c.cid, h, Q, got).all()
    v = torch.zeros(m, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch(ctx, c.cid, torch.from_numpy(np.ascontiguousarray(h)).cuda(),
                           torch.from_numpy(Q.view(np.int64)).cuda(), torch.from_numpy(got.view(np.int64)).cuda(),
                           m, v)
    torch.cuda.synchronize()
    assert v.cpu().numpy().all()


@pytest.mark.parametrize("c", SIGN_CURVES, ids=lambda c: c.name)
def test_sign_edge_requests(ctx, c):
    """Keys and nonces at and beyond the ends of [1, n), and hashes 0 and
    2^256 - 1 (e >= n)."""
    n = c.r
    keys = [0, 1, 2, n - 1, n, n + 1, (1 << 256) - 1, 0x1234567890ABCDEF]
    nonces = [0, 1, 2, n - 1, n, (1 << 256) - 1, 0xFEDCBA9876543210]
    hashes = [bytes(32), b"\xff" * 32, bytes(range(32))]
    rows = [(h, dd, kk) for h in hashes for dd in keys for kk in nonces]
    H = np.array([list(r[0]) for r in rows], dtype=np.uint8)
    D = syn.ints_to_limbs([r[1] for r in rows], 4)
    K = syn.ints_to_limbs([r[2] for r in rows], 4)
    want = co.ecdsa_sign(c.cid, H, D, K)
    ok = np.array([1 <= r[1] < n and 1 <= r[2] < n for r in rows])
    assert (want[~ok] == 0).all() and (want[ok] != 0).any(axis=1).all()
    assert np.array_equal(gpu_sign(ctx, c, H, D, K), want)


def test_sign_host_pointers_empty_and_errors(ctx):
    c = curves.SECP256R1
    h, d, k = seeded_sign_requests(c, 300, 1290)
    out = np.zeros((300, 8), dtype=np.uint64)
    eccmi.ecc_sign_batch(ctx, c.cid, np.ascontiguousarray(h), np.ascontiguousarray(d), np.ascontiguousarray(k),
                         300, out)
    assert np.array_equal(out, co.ecdsa_sign(c.cid, h, d, k))
    eccmi.ecc_sign_batch(ctx, c.cid, None, None, None, 0, None)
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_sign_batch(ctx, curves.BN254.cid, h[:4], d[:4], k[:4], 4, out[:4])
    assert e.value.name == "ECC_ERR_UNSUPPORTED"
