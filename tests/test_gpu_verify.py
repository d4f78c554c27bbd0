"""Parity of batched ECDSA verification (secp256r1) with the CPU oracle.

The result is one byte per request, compared exactly with the oracle's
verification of the same request."""

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves, ref
from tests.common import points_to_rows, seeded_signatures

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")

C = curves.SECP256R1


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.close()


def gpu_verify(ctx, hashes, pubs, sigs):
    m = hashes.shape[0]
    h = torch.from_numpy(np.ascontiguousarray(hashes)).cuda()
    q = torch.from_numpy(np.ascontiguousarray(pubs).view(np.int64)).cuda()
    s = torch.from_numpy(np.ascontiguousarray(sigs).view(np.int64)).cuda()
    v = torch.full((max(1, m),), 7, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch(ctx, C.cid, h, q, s, m, v)
    torch.cuda.synchronize()
    return v.cpu().numpy()[:m].astype(bool)


def oracle_verify(hashes, pubs, sigs):
    return co.ecdsa_verify(C.cid, hashes, pubs, sigs)


@pytest.mark.parametrize("m", [1, 255, 257, 3000])
def test_verify_seeded_requests(ctx, m):
    hashes, pubs, sigs = seeded_signatures(m, 900 + m)
    want = oracle_verify(hashes, pubs, sigs)
    assert want.sum() >= m - (m + 15) // 16  # the uncorrupted ones verify
    assert np.array_equal(gpu_verify(ctx, hashes, pubs, sigs), want)


def test_verify_malformed_requests(ctx):
    hashes, pubs, sigs = seeded_signatures(40, 950, corrupt_every=0)
    n, p = C.r, C.p
    rows = []

    def add(h, q, r, s):
        rows.append((np.array(h, dtype=np.uint8), np.array(q, dtype=np.uint64),
                     np.concatenate([syn.ints_to_limbs([r], 4)[0], syn.ints_to_limbs([s], 4)[0]])))

    for i in range(10):
        h, q = hashes[i], pubs[i]
        r, s = syn.limbs_to_int(sigs[i, :4]), syn.limbs_to_int(sigs[i, 4:])
        add(h, q, r, s)  # valid
        add(h, q, 0, s)
        add(h, q, r, 0)
        add(h, q, r + n if r + n < 1 << 256 else n, s)
        add(h, q, r, n)
        add(h, q, r, n - s)  # (r, -s) also verifies
        add(h, np.zeros(8, dtype=np.uint64), r, s)  # Q = O
        off = q.copy()
        off[4] ^= np.uint64(1)
        add(h, off, r, s)  # off the curve
        big = q.copy()
        big[:4] = syn.ints_to_limbs([p + 1], 4)[0] if p + 1 < 1 << 256 else big[:4]
        add(h, big, r, s)  # coordinate >= p
    # e = 0 and e >= n (hash all ones): signatures made for those hashes
    for hv in (bytes(32), b"\xff" * 32):
        d, kk = 12345678901234567, 98765432123456789
        Q = ref.scalar_mul(C, d, ref.generator(C))
        sig = ref.ecdsa_sign(C, d, kk, hv)
        add(list(hv), points_to_rows(C, [Q])[0], sig[0], sig[1])
    H = np.stack([r[0] for r in rows])
    Qs = np.stack([r[1] for r in rows])
    S = np.stack([r[2] for r in rows])
    want = oracle_verify(H, Qs, S)
    assert want[0] and not want[1] and want[5]
    assert np.array_equal(gpu_verify(ctx, H, Qs, S), want)


def test_verify_host_pointers_and_empty(ctx):
    hashes, pubs, sigs = seeded_signatures(300, 960)
    v = np.zeros(300, dtype=np.uint8)
    eccmi.ecc_verify_batch(ctx, C.cid, np.ascontiguousarray(hashes), np.ascontiguousarray(pubs),
                           np.ascontiguousarray(sigs), 300, v)
    assert np.array_equal(v.astype(bool), oracle_verify(hashes, pubs, sigs))
    eccmi.ecc_verify_batch(ctx, C.cid, None, None, None, 0, None)


def test_verify_wrong_curve(ctx):
    hashes, pubs, sigs = seeded_signatures(4, 970)
    v = np.zeros(4, dtype=np.uint8)
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_verify_batch(ctx, curves.BN254.cid, hashes, pubs, sigs, 4, v)
    assert e.value.name == "ECC_ERR_UNSUPPORTED"
