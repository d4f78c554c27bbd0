"""Parity of the batched MSM entry point (ecc_msm_batch) with the CPU oracle.

Each MSM of a batch must equal the oracle's MSM of its own slice, bit for
bit, whatever the sizes of its neighbours, in eager mode and when the launch
sequence is captured as a graph and replayed."""

import numpy as np
import pytest

import synthetic as syn
from oracle import c_oracle as co
from oracle import curves
from tests.common import rows_to_points, seeded_bases, seeded_scalars

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
eccmi = pytest.importorskip("paper_2501_03245_amd")

MSM_CURVES = [curves.BN254, curves.BLS12_381]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = eccmi.Context(0)
    yield c
    c.close()


def dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64).copy()).cuda()


def uneven_sizes(seed: int, m: int, hi_exp: float) -> np.ndarray:
    sizes = syn.log_uniform_sizes(seed, syn.TAG_MISC, m, 1.0, hi_exp)
    sizes[::7] = 0  # empty MSMs among the others
    sizes[1::11] = 1
    return sizes


def batch_inputs(c, sizes, seed):
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    total = int(offs[-1])
    k, bases = seeded_bases(c.name, max(total, 1), seed)
    s = seeded_scalars(c.name, max(total, 1), seed + 1, kind="bits")
    return offs, bases[:total], s[:total]


def run_batch(ctx, c, bases, scalars, offs, flags=0, window_c=0, bd=None, sd=None):
    m = len(offs) - 1
    out = torch.zeros(max(1, m) * 2 * c.limbs, dtype=torch.int64, device="cuda")
    inf = torch.zeros(max(1, m), dtype=torch.uint8, device="cuda")
    if bd is None:
        bd = dev(bases) if len(bases) else None
        sd = dev(scalars) if len(scalars) else None
    eccmi.ecc_msm_batch(ctx, c.cid, bd, sd, offs, out, inf, flags=flags, window_c=window_c)
    torch.cuda.synchronize()
    rows = out.cpu().numpy().view(np.uint64).reshape(-1, 2 * c.limbs)[:m]
    return rows_to_points(c, rows, inf.cpu().numpy()[:m])


def oracle_batch(c, bases, scalars, offs):
    out, inf = co.msm_batch(c.cid, c.limbs, bases, scalars, offs)
    return rows_to_points(c, out, inf)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_batch_uneven_sizes(ctx, c):
    sizes = uneven_sizes(3, 60, 11.0)
    offs, bases, s = batch_inputs(c, sizes, 300)
    assert run_batch(ctx, c, bases, s, offs) == oracle_batch(c, bases, s, offs)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_batch_matches_single_calls(ctx, c):
    sizes = np.array([5, 0, 1000, 1, 77, 4096, 3], dtype=np.int64)
    offs, bases, s = batch_inputs(c, sizes, 310)
    got = run_batch(ctx, c, bases, s, offs)
    for j in range(len(sizes)):
        lo, hi = int(offs[j]), int(offs[j + 1])
        out = torch.zeros(2 * c.limbs, dtype=torch.int64, device="cuda")
        inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
        n = hi - lo
        eccmi.ecc_msm(ctx, c.cid, dev(bases[lo:hi]) if n else None, dev(s[lo:hi]) if n else None, n, out, inf)
        single = rows_to_points(c, out.cpu().numpy().view(np.uint64).reshape(1, -1), inf.cpu().numpy())[0]
        assert got[j] == single


def test_batch_many_small_msms(ctx):
    """More MSMs (16,500) than the one-wave-per-MSM combine takes: one lane each."""
    c = curves.BN254
    sizes = syn.log_uniform_sizes(4, syn.TAG_MISC, 16500, 0.0, 3.0)
    offs, bases, s = batch_inputs(c, sizes, 320)
    assert run_batch(ctx, c, bases, s, offs) == oracle_batch(c, bases, s, offs)


@pytest.mark.parametrize("wc", [3, 9, 16])
def test_batch_fixed_window(ctx, wc):
    c = curves.BLS12_381
    sizes = uneven_sizes(5, 12, 10.0)
    offs, bases, s = batch_inputs(c, sizes, 330)
    assert run_batch(ctx, c, bases, s, offs, window_c=wc) == oracle_batch(c, bases, s, offs)


def test_batch_reduction_work_bound(ctx):
    """600 MSMs at window 9: 4.5 M buckets, so every reduction job gets fewer
    lanes with longer chains (four lanes of 64 buckets, sixteen jobs per
    wave) than a lone MSM would."""
    c = curves.BN254
    sizes = syn.log_uniform_sizes(8, syn.TAG_MISC, 600, 5.0, 7.0)
    offs, bases, s = batch_inputs(c, sizes, 360)
    assert run_batch(ctx, c, bases, s, offs, window_c=9) == oracle_batch(c, bases, s, offs)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_batch_graph_replay(ctx, c):
    """The captured sequence is replayed: each replay reads the buffers' current
    contents, with eager calls in between."""
    sizes = uneven_sizes(6, 30, 10.0)
    offs, bases, s = batch_inputs(c, sizes, 340)
    bd, sd = dev(bases), dev(s)
    want = oracle_batch(c, bases, s, offs)
    for rep in range(3):
        assert run_batch(ctx, c, bases, s, offs, flags=eccmi.ECC_USE_GRAPH, bd=bd, sd=sd) == want
        # eager work between replays
        assert run_batch(ctx, c, bases[:100], s[:100], np.array([0, 40, 100], dtype=np.uint64)) == \
            oracle_batch(c, bases[:100], s[:100], np.array([0, 40, 100], dtype=np.uint64))
    # new scalars in the same buffer: the replay follows them
    s2 = seeded_scalars(c.name, len(s), 341, kind="bits")
    sd.copy_(dev(s2))
    assert run_batch(ctx, c, bases, s2, offs, flags=eccmi.ECC_USE_GRAPH, bd=bd, sd=sd) == \
        oracle_batch(c, bases, s2, offs)


@pytest.mark.parametrize("c", MSM_CURVES, ids=lambda c: c.name)
def test_batch_errors_leave_outputs_untouched(ctx, c):
    sizes = np.array([10, 20, 30], dtype=np.int64)
    offs, bases, s = batch_inputs(c, sizes, 350)
    out = torch.full((3 * 2 * c.limbs,), 55, dtype=torch.int64, device="cuda")
    inf = torch.full((3,), 4, dtype=torch.uint8, device="cuda")
    big = s.copy()
    big[25] = syn.ints_to_limbs([1 << c.scalar_bits], 4)[0]
    for flags in (0, eccmi.ECC_USE_GRAPH):
        with pytest.raises(eccmi.EccError) as e:
            eccmi.ecc_msm_batch(ctx, c.cid, dev(bases), dev(big), offs, out, inf, flags=flags)
        assert e.value.name == "ECC_ERR_RANGE"
        assert torch.all(out == 55) and torch.all(inf == 4)
    bad = offs.copy()
    bad[2] = bad[1] - 1
    with pytest.raises(eccmi.EccError) as e:
        eccmi.ecc_msm_batch(ctx, c.cid, dev(bases), dev(s), bad, out, inf)
    assert e.value.name == "ECC_ERR_ARG"
    assert torch.all(out == 55) and torch.all(inf == 4)


def test_batch_host_pointers(ctx):
    c = curves.BLS12_381
    sizes = np.array([3, 0, 50, 1], dtype=np.int64)
    offs, bases, s = batch_inputs(c, sizes, 360)
    out = np.zeros((4, 2 * c.limbs), dtype=np.uint64)
    inf = np.zeros(4, dtype=np.uint8)
    eccmi.ecc_msm_batch(ctx, c.cid, np.ascontiguousarray(bases), np.ascontiguousarray(s), offs, out, inf)
    assert rows_to_points(c, out, inf) == oracle_batch(c, bases, s, offs)


def test_tuner_table_and_results(ctx, tmp_path):
    """The tuner picks a window per size class; MSMs of that class use it and
    stay exact; the table survives a save/load round trip."""
    c = curves.BN254
    eccmi.ecc_tune(ctx, c.cid, 9, 10, reps=1)
    w9, k9 = eccmi.ecc_tuned_params(ctx, c.cid, 700)
    assert 2 <= w9 <= 20 and k9 >= 1
    k, bases = seeded_bases(c.name, 700, 370)
    s = seeded_scalars(c.name, 700, 371, kind="bits")
    out = torch.zeros(2 * c.limbs, dtype=torch.int64, device="cuda")
    inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
    eccmi.ecc_msm(ctx, c.cid, dev(bases), dev(s), 700, out, inf)
    got = rows_to_points(c, out.cpu().numpy().view(np.uint64).reshape(1, -1), inf.cpu().numpy())[0]
    want, winf = co.msm(c.cid, c.limbs, bases, s)
    assert got == rows_to_points(c, want.reshape(1, -1), np.array([winf]))[0]
    path = str(tmp_path / "tune.txt")
    eccmi.ecc_tune_save(ctx, path)
    fresh = eccmi.Context(0)
    try:
        assert eccmi.ecc_tune_load(fresh, path) == 2
        assert eccmi.ecc_tuned_params(fresh, c.cid, 700) == (w9, k9)
    finally:
        fresh.close()


@pytest.mark.parametrize("wc", [0, 4], ids=["library_window", "window4"])
def test_batch_mixed_grouping_paths(ctx, wc):
    """One batch whose MSMs are grouped by both bucket-grouping paths: MSMs whose
    buckets fit LDS counters (and that have at most 2^16 points) by one
    workgroup each, the others by the per-point kernels, in one counts and
    offsets array.  At window 4 every MSM's buckets fit LDS, so the 70,000-point
    MSM goes to the per-point kernels by its size alone."""
    c = curves.BLS12_381
    sizes = np.array([4096, 40000, 3, 70000, 0, 129], dtype=np.int64)
    offs, bases, s = batch_inputs(c, sizes, 380)
    k, _ = seeded_bases(c.name, int(offs[-1]), 380)
    from tests.common import dlog_batch_expected
    want = dlog_batch_expected(c, k, s, offs)
    got = run_batch(ctx, c, bases, s, offs, window_c=wc)
    assert got == rows_to_points(c, want, ~want.any(axis=1))


def test_batch_split_and_bases_outside_g1(ctx):
    """Batches take the endomorphism split too (points 2i, 2i + 1 of the doubled
    index space).  BLS12-381 bases outside G1 need ECC_NO_ENDOMORPHISM in a
    batch as in a single call; with bases in G1 the flag changes nothing, and
    edge scalars (0, r - 1, r, 2^255 - 1, lambda) split correctly."""
    from tests.test_gpu_parity import bls_points_outside_g1
    from tests.common import points_to_rows
    c = curves.BLS12_381
    sizes = np.array([40, 0, 1, 17], dtype=np.int64)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    total = int(offs[-1])
    rows = points_to_rows(c, bls_points_outside_g1(total, 5))
    s = seeded_scalars(c.name, total, 391, kind="bits")
    want = oracle_batch(c, rows, s, offs)
    assert run_batch(ctx, c, rows, s, offs, flags=eccmi.ECC_NO_ENDOMORPHISM) == want
    got = run_batch(ctx, c, rows, s, offs)
    assert got[0] != want[0]  # the split assumes the order-r subgroup
    lam = 0xac45a4010001a40200000000ffffffff
    s[:5] = syn.ints_to_limbs([0, c.r - 1, c.r, (1 << 255) - 1, lam], 4)
    k, g1 = seeded_bases(c.name, total, 392)
    exp = oracle_batch(c, g1, s, offs)
    assert run_batch(ctx, c, g1, s, offs) == exp
    assert run_batch(ctx, c, g1, s, offs, flags=eccmi.ECC_NO_ENDOMORPHISM) == exp
