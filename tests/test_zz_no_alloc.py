"""The allocation-free verification entry point (ecc_verify_batch_noalloc)
against ecc_verify_batch's per-lane form on the same requests: two calls in a
row, the second smaller, on both signing curves; plus its size limit and the
curves without ECDSA keys."""

import numpy as np
import pytest

from oracle import curves
from tests.common import seeded_signatures

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")


def _dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    if dtype is not None:
        a = a.view(dtype)
    return torch.from_numpy(a).cuda()


def _requests(m, seed, c):
    hashes, pubs, sigs = seeded_signatures(m, seed, c=c)
    return _dev(hashes), _dev(pubs, np.int64), _dev(sigs, np.int64)


def _with_context(c, h, q, s, m):
    v = torch.full((m,), 7, dtype=torch.uint8, device="cuda")
    with eccmi.Context(0) as ctx:
        eccmi.ecc_verify_batch(ctx, c.cid, h, q, s, m, v, flags=eccmi.ECC_VERIFY_PER_LANE)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def _no_alloc(c, h, q, s, m):
    v = torch.full((m,), 7, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch_noalloc(c.cid, h, q, s, m, v)
    torch.cuda.synchronize()
    return v.cpu().numpy()


@pytest.mark.parametrize("c", [curves.SECP256R1, curves.SM2], ids=lambda c: c.name)
def test_no_alloc_matches_the_context_call_twice(c):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mmax = eccmi.ecc_verify_batch_noalloc_max()
    for m, seed in ((mmax, 7100), (1000, 7101)):  # second call smaller
        h, q, s = _requests(m, seed, c)
        got = _no_alloc(c, h, q, s, m)
        want = _with_context(c, h, q, s, m)
        assert set(np.unique(got)) <= {0, 1}
        assert want.sum() >= m - (m + 15) // 16  # the uncorrupted requests verify
        assert np.array_equal(got, want)


def test_no_alloc_limits_and_other_curves():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = curves.SECP256R1
    mmax = eccmi.ecc_verify_batch_noalloc_max()
    h, q, s = _requests(3, 7102, c)
    # above the maximum: rejected on the host, before any launch
    big = torch.zeros(mmax + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_verify_batch_noalloc(c.cid, torch.zeros((mmax + 1) * 32, dtype=torch.uint8, device="cuda"),
                                       torch.zeros((mmax + 1) * 8, dtype=torch.int64, device="cuda"),
                                       torch.zeros((mmax + 1) * 8, dtype=torch.int64, device="cuda"), mmax + 1, big)
    assert e.value.name == "ECC_ERR_ARG"
    # empty batch: nothing written
    v = torch.full((1,), 7, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch_noalloc(c.cid, h, q, s, 0, v)
    torch.cuda.synchronize()
    assert int(v.cpu()[0]) == 7
    # curves without ECDSA keys: every request invalid
    v = torch.full((3,), 7, dtype=torch.uint8, device="cuda")
    eccmi.ecc_verify_batch_noalloc(curves.BLS12_381.cid, h, q, s, 3, v)
    torch.cuda.synchronize()
    assert v.cpu().numpy().tolist() == [0, 0, 0]
