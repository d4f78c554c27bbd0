#!/usr/bin/env python3
"""Benchmark: multi-scalar multiplication throughput on one MI355X.

Workload (default): BLS12-381 G1 MSM of N = 2^20 points, uniform 255-bit
scalars, seeded bases P_i = k_i G (k_i uniform in [1, r)), Pippenger window
c = 16.  Bases and scalars are generated on the device before the timed
region; one step is one ecc_msm call over the resident inputs (which splits
every scalar with the curve endomorphism and buckets 2N points of 127-bit
half-scalars).

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 compute units at 2.4 GHz; v_mad_u64_u32 (one 32x32+64 multiply-add
# per lane) issues at one per lane per clock on each SIMD's 16 lanes, i.e.
# 4 x 16 = 64 lane-ops per CU per clock, the fp64-FMA rate class.
CUS = 256
CLOCK_HZ = 2.4e9
MAD32_PER_CU_CLK = 64
PEAK_MAD32 = CUS * CLOCK_HZ * MAD32_PER_CU_CLK  # 3.93e13 /s

# per batch-affine addition: 6 field multiplications (Section 3.1) of
# 2m^2 + m = 300 word multiply-adds each for m = 12 (381-bit field, D = 2^32)
MAD32_PER_MUL = {1: 2 * 8 * 8 + 8, 2: 2 * 12 * 12 + 12}
MULS_PER_AFFINE_ADD = 6


def adds_per_point(n: int, bits: int, c: int) -> float:
    """Textbook unsigned-digit Pippenger additions per point at window c."""
    W = -(-bits // c)
    return (n * W + W * 2 * (2 ** c - 1) + bits + W) / n


def algorithmic_mad32_per_point(n: int, bits: int, curve: int) -> float:
    best = min(adds_per_point(n, bits, c) for c in range(1, 25))
    return best * MULS_PER_AFFINE_ADD * MAD32_PER_MUL[curve]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bucket_round_traffic_bls12_381_n2p20.json")
KERNEL_SOURCES = ["constants.h", "curves.h", "field.h", "inverse.h", "point.h", "kernels.h"]


def kernel_source_digest() -> str:
    """sha256 over the device sources the bucket-round kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_03245_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per bucket-round launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != kernel_source_digest():
        return None
    return t.get("bytes_per_launch")


def batched_vs_plain(eccmi, syn, torch, np, ctx, cid: int, m: int, plain_m: int, seed: int) -> dict:
    """Uneven batch: m BLS12-381 MSMs with sizes log-uniform in [2, 2^14],
    seeded bases k_i G (made on the GPU) and uniform scalars.  The whole batch
    runs as one captured launch sequence (ecc_msm_batch with ECC_USE_GRAPH);
    the first plain_m MSMs also run as one ecc_msm call each, and batched, for
    a like-for-like ratio."""
    L = eccmi.LIMBS[cid]
    bits = eccmi.SCALAR_BITS[cid]
    order = 0x73EDA753299D7D483339D80809A1D80553BDA402FFFE5BFEFFFFFFFF00000001
    sizes = syn.log_uniform_sizes(seed, syn.TAG_SIZES, m, 1.0, 14.0)
    offs = np.zeros(m + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    total = int(offs[-1])
    dev = torch.device("cuda:0")
    k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, total, 1, order, 4)
    s = syn.uniform_bits(seed, syn.TAG_SCALARS, total, bits, 4)
    kd = torch.from_numpy(k.view(np.int64)).to(dev)
    sd = torch.from_numpy(s.view(np.int64)).to(dev)
    bases = torch.empty(total * 2 * L, dtype=torch.int64, device=dev)
    eccmi.ecc_fixed_base_mul(ctx, cid, kd, total, bases)
    del kd
    out = torch.zeros(m * 2 * L, dtype=torch.int64, device=dev)
    inf = torch.zeros(m, dtype=torch.uint8, device=dev)

    def run_batch(o, nm, reps):
        eccmi.ecc_msm_batch(ctx, cid, bases, sd, o, out, inf, flags=eccmi.ECC_USE_GRAPH)  # capture + warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            eccmi.ecc_msm_batch(ctx, cid, bases, sd, o, out, inf, flags=eccmi.ECC_USE_GRAPH)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_all = run_batch(offs, m, 2)
    sub = offs[: plain_m + 1]
    pts_sub = int(sub[-1])
    t_sub_batched = run_batch(sub, plain_m, 2)
    o1 = torch.zeros(2 * L, dtype=torch.int64, device=dev)
    i1 = torch.zeros(1, dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    for j in range(plain_m):
        lo, hi = int(offs[j]), int(offs[j + 1])
        eccmi.ecc_msm(ctx, cid, bases[lo * 2 * L: hi * 2 * L], sd[lo * 4: hi * 4], hi - lo, o1, i1)
    torch.cuda.synchronize()
    t_sub_plain = time.perf_counter() - t0
    del bases, sd
    return {"workload": f"{m} BLS12-381 MSMs, sizes log-uniform in [2, 2^14], {total} points; "
                        f"one captured launch sequence",
            "batched_points_per_s": total / t_all, "batched_ms": t_all * 1e3,
            "subset": f"first {plain_m} MSMs ({pts_sub} points)",
            "subset_batched_points_per_s": pts_sub / t_sub_batched,
            "subset_plain_points_per_s": pts_sub / t_sub_plain,
            "batched_over_plain": t_sub_plain / t_sub_batched}


ORDERS = {1: 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001,
          2: 0x73EDA753299D7D483339D80809A1D80553BDA402FFFE5BFEFFFFFFFF00000001}


def config_sweep(eccmi, syn, torch, np, ctx, budget_s: float) -> list:
    """The other MSM workloads: BN254 at 2^12 with bases given in Montgomery
    form; BN254 plain at 2^16, 2^20 and 2^22 with c = 16; BLS12-381 at 2^16
    and 2^24, plain (c = 16) against the autotuned window (ecc_tune run in
    this process for that size).  Seeded bases k_i G (k_i uniform in [1, r),
    the products made on the GPU) and uniform scalars ([0, r) for the 2^12
    case, full bit length otherwise).  Each row: host clock around `reps`
    synchronous calls after one warm-up, reps chosen for about 0.3 s."""
    rows = []
    t_start = time.perf_counter()
    cases = [(1, 12, "mont", 0), (1, 16, "plain", 16), (1, 20, "plain", 16), (1, 22, "plain", 16),
             (2, 16, "plain", 16), (2, 16, "tuned", 0), (2, 24, "plain", 16), (2, 24, "tuned", 0)]
    inputs = {}
    for cid, lg, kind, c in cases:
        if time.perf_counter() - t_start > budget_s:
            rows.append({"curve": cid, "log2n": lg, "kind": kind, "skipped": "time budget of the sweep spent"})
            continue
        n = 1 << lg
        L = eccmi.LIMBS[cid]
        bits = eccmi.SCALAR_BITS[cid]
        key = (cid, lg, kind == "mont")
        if key not in inputs:
            inputs.clear()
            torch.cuda.empty_cache()
            seed = 0xC0F0 + 64 * cid + lg
            k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, n, 1, ORDERS[cid], 4)
            if kind == "mont":
                s = syn.uniform_below(seed, syn.TAG_SCALARS, n, ORDERS[cid], 4)
            else:
                s = syn.uniform_bits(seed, syn.TAG_SCALARS, n, bits, 4)
            kd = torch.from_numpy(k.view(np.int64)).cuda()
            b = torch.empty(n * 2 * L, dtype=torch.int64, device="cuda")
            eccmi.ecc_fixed_base_mul(ctx, cid, kd, n, b, flags=eccmi.ECC_IN_MONTGOMERY if kind == "mont" else 0)
            del kd
            inputs[key] = (b, torch.from_numpy(s.view(np.int64)).cuda())
        b, sd = inputs[key]
        out = torch.zeros(2 * L, dtype=torch.int64, device="cuda")
        inf = torch.zeros(1, dtype=torch.uint8, device="cuda")
        flags = eccmi.ECC_IN_MONTGOMERY if kind == "mont" else 0
        tune_s = None
        if kind == "tuned":
            t0 = time.perf_counter()
            eccmi.ecc_tune(ctx, cid, lg, lg, reps=2)
            tune_s = time.perf_counter() - t0
        eccmi.ecc_msm(ctx, cid, b, sd, n, out, inf, flags=flags, window_c=c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eccmi.ecc_msm(ctx, cid, b, sd, n, out, inf, flags=flags, window_c=c)
        torch.cuda.synchronize()
        one = time.perf_counter() - t0
        reps = max(2, min(50, int(0.3 / max(one, 1e-4))))
        t0 = time.perf_counter()
        for _ in range(reps):
            eccmi.ecc_msm(ctx, cid, b, sd, n, out, inf, flags=flags, window_c=c)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        used_c = c if c else eccmi.ecc_tuned_params(ctx, cid, n)[0]
        row = {"curve": {1: "bn254", 2: "bls12_381"}[cid], "n": n, "log2n": lg,
               "kind": {"mont": "library window, bases in Montgomery form", "plain": "window c fixed at 16",
                        "tuned": "autotuned window"}[kind],
               "window_c": used_c, "reps": reps, "ms_per_msm": dt * 1e3, "points_per_s": n / dt,
               "msm_frac": (n / dt) * algorithmic_mad32_per_point(n, bits, cid) / PEAK_MAD32}
        if tune_s is not None:
            row["tune_s"] = tune_s
        rows.append(row)
        print(f"[bench] config: {json.dumps(row)}", file=sys.stderr, flush=True)
    inputs.clear()
    torch.cuda.empty_cache()
    return rows


# the paper's Table 5 (one NVIDIA A100, SM2): operations per second at
# batches of 432 streaming processors x 2^11 .. 2^16 requests
PAPER_TABLE5_A100 = {
    "fpmul": [11723016, 13005468, 13755865, 14389168, 14385871, 14299320],
    "upmul": [6270010, 6561449, 6689186, 6766892, 6837619, 6732287],
}


def table5_sweep(eccmi, syn, torch, np, ctx, lgs=(11, 12, 13, 14, 15, 16)) -> dict:
    """The paper's Table 5 workload on SM2: fixed-point (FPMUL, k_i G) and
    unknown-point (UPMUL, k_i P_i) multiplication throughput against the batch
    size, at the table's per-processor batches scaled to MI355X's 256 compute
    units (256 x 2^11 .. 256 x 2^16 requests).  UPMUL runs in both forms: the
    paper's batched-affine Algorithm 3 (ECC_PMUL_BATCHED) and the per-lane
    XYZZ form.  Requests: 2^20 distinct seeded (k_i, P_i = a_i G) pairs, tiled
    up to the batch size; device-resident; host clock around one synchronous
    call after one warm-up call of the same size."""
    cid = eccmi.CURVES["sm2"]
    order = 0xFFFFFFFEFFFFFFFFFFFFFFFFFFFFFFFF7203DF6B21C6052B53BBF40939D54123
    base_n = 1 << 20
    seed = 0x7AB5
    a = torch.from_numpy(syn.uniform_range(seed, syn.TAG_BASE_DLOG, base_n, 1, order, 4).view(np.int64)).cuda()
    k = torch.from_numpy(syn.uniform_bits(seed, syn.TAG_SCALARS, base_n, 256, 4).view(np.int64).reshape(-1)).cuda()
    pts = torch.empty(base_n * 8, dtype=torch.int64, device="cuda")
    eccmi.ecc_fixed_base_mul(ctx, cid, a, base_n, pts)
    del a
    rows = []
    for j, lg in enumerate(lgs):
        n = 256 << lg
        reps = -(-n // base_n)
        kk = k.repeat(reps)[: n * 4]
        pp = pts.repeat(reps)[: n * 8]
        out = torch.empty(n * 8, dtype=torch.int64, device="cuda")

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        t_fp = timed(lambda: eccmi.ecc_fixed_base_mul(ctx, cid, kk, n, out))
        t_up = timed(lambda: eccmi.ecc_pmul_batch(ctx, cid, pp, kk, n, out, flags=eccmi.ECC_PMUL_BATCHED))
        t_pl = timed(lambda: eccmi.ecc_pmul_batch(ctx, cid, pp, kk, n, out))
        row = {"batch": n, "per_cu": 1 << lg,
               "fpmul_per_s": n / t_fp, "upmul_batched_affine_per_s": n / t_up, "upmul_per_lane_per_s": n / t_pl,
               "paper_a100_batch": 432 << lg,
               "paper_a100_fpmul_per_s": PAPER_TABLE5_A100["fpmul"][j],
               "paper_a100_upmul_per_s": PAPER_TABLE5_A100["upmul"][j]}
        rows.append(row)
        print(f"[bench] table5: {json.dumps(row)}", file=sys.stderr, flush=True)
        del kk, pp, out
    del k, pts
    torch.cuda.empty_cache()
    return {"workload": "SM2 fixed- and unknown-point multiplication, batches of 256 x 2^11 .. 256 x 2^16 "
                        "requests (the paper's Table 5 per-processor batches on 256 compute units)",
            "paper_hardware": "one NVIDIA A100 (the paper's Table 5, SM2); batches of 432 x 2^11 .. 2^16",
            "rows": rows}


def serve_mix(eccmi, syn, torch, np, ctx, seconds: float, seed: int) -> dict:
    """Served mixed stream on one GPU: secp256r1 verifications (the oracle-made
    requests of tests/golden/p256_requests.npz, every 16th corrupted, tiled)
    with one BLS12-381 MSM request (size round(2^U), U uniform in [10, 18],
    over a resident set of 2^18 bases) after every 256 verifications; two
    slots, and an HBM budget of about two 2^18-point MSM batches per slot so
    that admission cuts large batches.  First the saturated capacity: one
    burst of 2^17 verifications and their 512 MSMs, verifications per second
    over the burst's span.  Then Poisson arrivals (seeded exponential gaps) at
    rho = 0.5 and 0.8 of that capacity, for 2^20 verifications or `seconds`,
    whichever is shorter; requests are offered by a host loop at their
    arrival times (in groups of those due, every ~100 us).  Latency is from
    submission to the end of the request's batch.  Every verdict is checked
    against the oracle's in the request file, and a sample of the served MSM
    results against the same MSM run alone by ecc_msm."""
    req = np.load(os.path.join(ROOT, "tests", "golden", "p256_requests.npz"))
    H, Q, S, V = req["hashes"], req["pubkeys"], req["sigs"], req["valid"]
    nreq = H.shape[0]
    cid = eccmi.CURVES["bls12_381"]
    L = eccmi.LIMBS[cid]
    nb = 1 << 18
    order = ORDERS[2]
    k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, nb, 1, order, 4)
    kd = torch.from_numpy(k.view(np.int64).reshape(-1)).cuda()
    bases = torch.empty(nb * 2 * L, dtype=torch.int64, device="cuda")
    eccmi.ecc_fixed_base_mul(ctx, cid, kd, nb, bases)
    del kd
    bh = bases.cpu().numpy().view(np.uint64).reshape(nb, 2 * L)
    pool = syn.uniform_bits(seed, syn.TAG_SCALARS, nb, 255, 4)
    n_msm_max = (1 << 20) // 256 + 1
    msz = syn.log_uniform_sizes(seed, syn.TAG_SIZES, n_msm_max, 10.0, 18.0)
    mfirst = (syn.u64(seed, syn.TAG_MISC, n_msm_max) % np.uint64(nb)).astype(np.int64)
    mfirst = np.minimum(mfirst, nb - msz)
    plan2 = eccmi.ecc_msm_batch_scratch_bytes(ctx, cid, [0, nb, 2 * nb], flags=eccmi.ECC_BASES_PER_MSM)
    budget = 2 * plan2

    def run_phase(rate, total_v, burst):
        """Offer total_v verifications (and one MSM per 256) at `rate`/s, or all
        at once (burst); returns the phase's measurements."""
        srv = eccmi.Server(0, slots=2, hbm_budget_bytes=budget, max_batch_points=1 << 20,
                           max_batch_verify=1 << 16)
        try:
            bid = srv.add_bases(cid, bh)
            n_m = total_v // 256
            arrive = np.zeros(total_v) if burst else np.cumsum(
                syn.exponential_gaps(seed + int(rate), syn.TAG_ARRIVALS, total_v, 1.0 / rate))
            tv, tm = [], []
            idx = 0
            mi = 0
            t0 = time.perf_counter()
            while idx < total_v:
                now = time.perf_counter() - t0
                due = int(np.searchsorted(arrive, now, side="right"))
                if due <= idx:
                    time.sleep(5e-5)
                    continue
                while idx < due:
                    hi = min(due, (idx // 256 + 1) * 256)
                    sel = np.arange(idx, hi) % nreq
                    tv += srv.submit_verify_many(H[sel], Q[sel], S[sel])
                    idx = hi
                    if idx % 256 == 0 and mi < n_m:
                        n = int(msz[mi])
                        a = int(mfirst[mi])
                        tm.append((mi, srv.submit_msm(bid, a, pool[a:a + n])))
                        mi += 1
            t_offered = time.perf_counter() - t0
            flags, lat_v, stv = srv.wait_many(tv)
            res_m = [(j, srv.wait(t)) for j, t in tm]
            st = srv.stats()
        finally:
            srv.close()
        sel = np.arange(total_v) % nreq
        wrong = int(np.count_nonzero(flags != V[sel])) + int(np.count_nonzero(stv != 0))
        lat_m = np.array([r[2] for _, r in res_m]) if res_m else np.zeros(1)
        out = {"verifications": total_v, "msms": len(res_m), "msm_points": int(st["msm_points"]),
               "offered_s": t_offered, "span_s": st["span_ms"] * 1e-3,
               "verify_per_s": total_v / (st["span_ms"] * 1e-3) if st["span_ms"] else 0.0,
               "p50_verify_ms": float(np.percentile(lat_v, 50)), "p99_verify_ms": float(np.percentile(lat_v, 99)),
               "p50_msm_ms": float(np.percentile(lat_m, 50)), "p99_msm_ms": float(np.percentile(lat_m, 99)),
               "batches": int(st["batches"]), "budget_cuts": int(st["budget_cuts"]),
               "nomem_splits": int(st["nomem_splits"]), "max_queue": int(st["max_queue"]),
               "verdicts_differing_from_oracle_file": wrong}
        if not burst:
            out["offered_verify_per_s"] = rate
        return out, res_m

    cap, _ = run_phase(0.0, 1 << 17, True)
    capacity = cap["verify_per_s"]
    phases = {"saturated": cap}
    checked = 0
    mismatched = 0
    for rho in (0.5, 0.8):
        rate = rho * capacity
        total_v = int(min(1 << 20, rate * seconds)) // 256 * 256
        ph, res_m = run_phase(rate, max(256, total_v), False)
        phases[f"rho_{rho}"] = ph
        # the same MSM alone, by the plain call over the same resident bases
        for j, (xy, flag, _) in res_m[:: max(1, len(res_m) // 6)][:6]:
            n, a = int(msz[j]), int(mfirst[j])
            o = torch.zeros(2 * L, dtype=torch.int64, device="cuda")
            f = torch.zeros(1, dtype=torch.uint8, device="cuda")
            sd = torch.from_numpy(pool[a:a + n].view(np.int64).reshape(-1)).cuda()
            eccmi.ecc_msm(ctx, cid, bases[a * 2 * L:(a + n) * 2 * L], sd, n, o, f)
            checked += 1
            mismatched += int(not (np.array_equal(o.cpu().numpy().view(np.uint64), xy) and int(f.item()) == flag))
        print(f"[bench] served rho={rho}: {json.dumps(ph)}", file=sys.stderr, flush=True)
    del bases
    return {"workload": "secp256r1 verifications (oracle-made, 1/16 corrupted) with one BLS12-381 MSM of "
                        "round(2^U) points, U in [10, 18], per 256 verifications, over 2^18 resident bases; "
                        f"2 slots, HBM budget {budget} bytes (two 2^18-point MSM batches per slot)",
            "capacity_verify_per_s": capacity, "phases": phases,
            "msm_results_checked_against_alone": checked, "msm_results_differing": mismatched}


def ablations(eccmi, torch, ctx, cid, bases, sd, n, out, inf, args) -> int:
    """The benchmark MSM with one design choice changed at a time, each on the
    same resident inputs: the default; the endomorphism split off
    (ECC_NO_ENDOMORPHISM: 16 windows over N points instead of 8 over 2N); the
    window width c in {12, 14, 18}; the launch sequence replayed as one
    captured graph (ECC_USE_GRAPH); and, on BLS12-381, the round kernel's
    design variants (stored denominators, per-lane chain layout, both: the
    paper's memory management off; decompress and additions in two kernels;
    all three: memory management and fusion off; per-lane inversion instead
    of GAS).  Each variant's result must equal the
    default's.  Host clock over `steps` synchronous calls after `warmup`."""
    variants = [("default", 0, args.window, 0),
                ("no_endomorphism_split", eccmi.ECC_NO_ENDOMORPHISM, args.window, 0),
                ("window_c12", 0, 12, 0), ("window_c14", 0, 14, 0), ("window_c18", 0, 18, 0),
                ("graph_replay", eccmi.ECC_USE_GRAPH, args.window, 0)]
    if cid == 2:
        # the round kernel's own design choices (Sections 3.2 and 3.3), one at a
        # time and the paper's two compound variants
        variants += [("round_store_denominators", 0, args.window, eccmi.RV_STORE_DENOM),
                     ("round_chain_per_lane_layout", 0, args.window, eccmi.RV_AOS_CHAIN),
                     ("round_memory_management_off", 0, args.window, eccmi.RV_STORE_DENOM | eccmi.RV_AOS_CHAIN),
                     ("round_unfused_decompress_and_add", 0, args.window, eccmi.RV_SPLIT_APPLY),
                     ("round_memory_management_and_fusion_off", 0, args.window,
                      eccmi.RV_STORE_DENOM | eccmi.RV_AOS_CHAIN | eccmi.RV_SPLIT_APPLY),
                     ("round_per_lane_inversion", 0, args.window, eccmi.RV_LANE_INV),
                     ("round_half_prefix_recompute", 0, args.window, eccmi.RV_HALF_PREFIX),
                     ("rounds_to_the_end", 0, args.window, eccmi.RV_ROUNDS_ONLY)]
    ref_xy = None
    bad = 0
    for name, flags, c, variant in variants:
        ctx.set_round_variant(variant)
        for _ in range(max(1, args.warmup)):
            eccmi.ecc_msm(ctx, cid, bases, sd, n, out, inf, flags=flags, window_c=c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            eccmi.ecc_msm(ctx, cid, bases, sd, n, out, inf, flags=flags, window_c=c)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        # one more call with phase timing, outside the timed loop
        ctx.set_profiling(True)
        eccmi.ecc_msm(ctx, cid, bases, sd, n, out, inf, flags=flags, window_c=c)
        st = ctx.stats()
        ctx.set_profiling(False)
        phases = {k: round(st[k + "_ms"], 3) for k in ("prepare", "round", "finish", "reduce", "combine")}
        phases["round_launches"] = st["round_launches"]
        phases["round_adds"] = st["round_adds"]
        xy = out.cpu().tolist() + inf.cpu().tolist()
        if ref_xy is None:
            ref_xy = xy
        same = xy == ref_xy
        bad += not same
        ctx.set_round_variant(0)
        print(json.dumps({"ablation": name, "flags": flags, "window_c": c, "round_variant": variant, "n": n,
                          "ms_per_msm": dt * 1e3,
                          "points_per_s": n / dt, "result_equals_default": same, "phases_ms": phases}), flush=True)
    ctx.close()
    return 1 if bad else 0


def ecdsa_sweep(eccmi, syn, torch, np, log2s) -> int:
    """ECDSA signing and verification, and fixed- and unknown-point
    multiplication (the paper's FPMUL and UPMUL), on secp256r1 and SM2 at each
    batch size 2^lg, device-resident: seeded keys d, nonces k and hashes; the signatures
    come from ecc_sign_batch and the keys Q = d G from ecc_fixed_base_mul, and
    every 16th hash is then flipped in one bit, so the expected verdicts are
    known without the oracle.  Host clock around one synchronous call, median
    of five (two above 2^16); verification in both kernel forms."""
    bad = 0
    ctx = eccmi.Context(0)
    try:
        for name in ("secp256r1", "sm2"):
            cid = eccmi.CURVES[name]
            n_order = {"secp256r1": 0xFFFFFFFF00000000FFFFFFFFFFFFFFFFBCE6FAADA7179E84F3B9CAC2FC632551,
                       "sm2": 0xFFFFFFFEFFFFFFFFFFFFFFFFFFFFFFFF7203DF6B21C6052B53BBF40939D54123}[name]
            for lg in log2s:
                m = 1 << lg
                seed = 0xEC5A + lg
                d = torch.from_numpy(syn.uniform_range(seed, syn.TAG_KEYS, m, 1, n_order, 4).view(np.int64)).cuda()
                k = torch.from_numpy(syn.uniform_range(seed, syn.TAG_NONCES, m, 1, n_order, 4).view(np.int64)).cuda()
                hh = syn.random_bytes(seed, syn.TAG_HASH, m, 32)
                h = torch.from_numpy(np.ascontiguousarray(hh)).cuda()
                sig = torch.zeros(m * 8, dtype=torch.int64, device="cuda")
                q = torch.zeros(m * 8, dtype=torch.int64, device="cuda")
                reps = 5 if lg <= 16 else 2

                def timed(fn):
                    fn()
                    torch.cuda.synchronize()
                    ts = []
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        fn()
                        torch.cuda.synchronize()
                        ts.append(time.perf_counter() - t0)
                    return sorted(ts)[len(ts) // 2]

                t_sign = timed(lambda: eccmi.ecc_sign_batch(ctx, cid, h, d, k, m, sig))
                t_fp = timed(lambda: eccmi.ecc_fixed_base_mul(ctx, cid, d, m, q))
                kq = torch.zeros(m * 8, dtype=torch.int64, device="cuda")
                t_up = timed(lambda: eccmi.ecc_pmul_batch(ctx, cid, q, k, m, kq))
                hh[::16, 0] ^= 1
                h.copy_(torch.from_numpy(hh))
                want = np.ones(m, dtype=np.uint8)
                want[::16] = 0
                row = {"curve": name, "requests": m,
                       "sign": {"ms": t_sign * 1e3, "per_s": m / t_sign,
                                "all_nonzero": bool(sig.view(m, 8).ne(0).any(dim=1).all().item())},
                       "fixed_point_mul": {"ms": t_fp * 1e3, "per_s": m / t_fp},
                       "unknown_point_mul": {"ms": t_up * 1e3, "per_s": m / t_up,
                                             "all_finite": bool(kq.view(m, 8).ne(0).any(dim=1).all().item())}}
                v = torch.zeros(m, dtype=torch.uint8, device="cuda")
                for form, fl in (("verify_batched", eccmi.ECC_VERIFY_BATCHED),
                                 ("verify_per_lane", eccmi.ECC_VERIFY_PER_LANE)):
                    t = timed(lambda: eccmi.ecc_verify_batch(ctx, cid, h, q, sig, m, v, flags=fl))
                    ok = bool(np.array_equal(v.cpu().numpy(), want))
                    bad += not ok
                    row[form] = {"ms": t * 1e3, "per_s": m / t, "verdicts_as_expected": ok}
                bad += not row["sign"]["all_nonzero"]
                bad += not row["unknown_point_mul"]["all_finite"]
                print(json.dumps(row), flush=True)
    finally:
        ctx.close()
    return 1 if bad else 0


def issue_rate(eccmi, ctx) -> int:
    """Issue-rate probe (the paper's Table 2 method): every lane runs 1 or 8
    interleaved dependency chains of one instruction class at 1, 2 and 4 waves
    per SIMD; reports lane-operations per compute unit and clock at the
    2.4 GHz spec clock and at the shader clock measured in the kernel."""
    for op in ("v_mad_u64_u32", "v_mul_lo_u32", "v_fma_f64"):
        for chains in (1, 8):
            for waves in (1, 2, 4):
                r = eccmi.ecc_probe_issue_rate(ctx, op, chains, waves, iters=2048 if chains == 8 else 8192)
                per_cu_s = r["lane_ops"] / (r["ms"] * 1e-3) / CUS
                row = {"probe": op, "chains": chains, "waves_per_simd": waves, "ms": r["ms"],
                       "lane_ops_per_cu_clk_at_2400mhz": per_cu_s / CLOCK_HZ,
                       "shader_mhz": r["shader_mhz"],
                       "lane_ops_per_cu_clk_at_shader_clock": per_cu_s / (r["shader_mhz"] * 1e6)
                       if r["shader_mhz"] > 0 else None,
                       "chip_lane_ops_per_s": per_cu_s * CUS}
                print(json.dumps(row), flush=True)
    ctx.close()
    return 0


def cpu_baseline(bases_host, scalars_host, curve_cid: int, limbs: int, sample: int) -> dict:
    """The plain oracle (naive sum of scalar multiples, C, all host threads)
    on the first `sample` points of the same workload."""
    from oracle import c_oracle as co
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    b = bases_host[:sample]
    s = scalars_host[:sample]
    t0 = time.perf_counter()
    co.msm(curve_cid, limbs, b, s, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": f"naive sum of {sample} scalar multiples (double-and-add, Jacobian), "
                      f"the first {sample} points of the benchmark workload; {dt:.1f} s wall"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--window", type=int, default=16)
    ap.add_argument("--curve", default="bls12_381", choices=["bls12_381", "bn254"])
    ap.add_argument("--cpu-sample", type=int, default=1 << 19)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and served measurements")
    ap.add_argument("--batch-m", type=int, default=4096)
    ap.add_argument("--no-configs", action="store_true", help="skip the sweep over the other MSM workloads")
    ap.add_argument("--table5-only", action="store_true", help="only the SM2 FPMUL/UPMUL batch sweep")
    ap.add_argument("--configs-only", action="store_true", help="only the sweep over the other MSM workloads")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-only", action="store_true", help="only the served mixed stream")
    ap.add_argument("--batched-only", action="store_true", help="only the uneven 4096-MSM batch")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (the reference "
                         "for scaling HBM byte counters), then exit")
    ap.add_argument("--ablations", action="store_true",
                    help="only time the MSM of the benchmark workload with one design choice changed at a time "
                         "(endomorphism split off, window width, graph capture), print one JSON line per variant, "
                         "then exit")
    ap.add_argument("--ecdsa-sweep", type=str, default="", metavar="LOG2S",
                    help="only time ECDSA signing and verification (both forms) on secp256r1 and SM2 at the "
                         "comma-separated log2 batch sizes, print one JSON line per curve and size, then exit")
    ap.add_argument("--issue-rate", action="store_true",
                    help="only run the instruction issue-rate probe (v_mad_u64_u32, v_mul_lo_u32, v_fma_f64; "
                         "dependent and interleaved chains at 1, 2 and 4 waves per SIMD), print one JSON line "
                         "per case, then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}), flush=True)
        return 0

    import paper_2501_03245_amd as eccmi
    import synthetic as syn

    if args.ecdsa_sweep:
        return ecdsa_sweep(eccmi, syn, torch, np, [int(x) for x in args.ecdsa_sweep.split(",")])
    if args.issue_rate:
        return issue_rate(eccmi, eccmi.Context(0))

    if args.batched_only:
        ctx = eccmi.Context(0)
        ctx.set_profiling(True)
        r = batched_vs_plain(eccmi, syn, torch, np, ctx, 2, args.batch_m, min(512, args.batch_m), 0xBA7C)
        r["phases_ms_all_calls"] = ctx.stats()
        print(json.dumps(r), flush=True)
        ctx.close()
        return 0

    if args.serve_only:
        ctx = eccmi.Context(0)
        print(json.dumps(serve_mix(eccmi, syn, torch, np, ctx, args.serve_seconds, 0x5E4E)), flush=True)
        ctx.close()
        return 0

    if args.table5_only:
        ctx = eccmi.Context(0)
        print(json.dumps(table5_sweep(eccmi, syn, torch, np, ctx)), flush=True)
        ctx.close()
        return 0

    if args.configs_only:
        ctx = eccmi.Context(0)
        rows = config_sweep(eccmi, syn, torch, np, ctx, 1e9)
        for r in rows:
            print(json.dumps(r), flush=True)
        ctx.close()
        return 0

    cid = eccmi.CURVES[args.curve]
    L = eccmi.LIMBS[cid]
    bits = eccmi.SCALAR_BITS[cid]
    n = 1 << args.log2n
    order = {1: 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001,
             2: 0x73EDA753299D7D483339D80809A1D80553BDA402FFFE5BFEFFFFFFFF00000001}[cid]
    seed = 0xECC2

    t0 = time.perf_counter()
    k = syn.uniform_range(seed, syn.TAG_BASE_DLOG, n, 1, order, 4)
    s = syn.uniform_bits(seed, syn.TAG_SCALARS, n, bits, 4)
    print(f"[bench] inputs drawn in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    ctx = eccmi.Context(0)
    kd = torch.from_numpy(k.view(np.int64)).to(dev)
    sd = torch.from_numpy(s.view(np.int64)).to(dev)
    bases = torch.empty(n * 2 * L, dtype=torch.int64, device=dev)
    eccmi.ecc_fixed_base_mul(ctx, cid, kd, n, bases)
    out = torch.zeros(2 * L, dtype=torch.int64, device=dev)
    inf = torch.zeros(1, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print(f"[bench] bases k_i G generated on the GPU", file=sys.stderr, flush=True)

    if args.ablations:
        return ablations(eccmi, torch, ctx, cid, bases, sd, n, out, inf, args)

    for _ in range(args.warmup):
        eccmi.ecc_msm(ctx, cid, bases, sd, n, out, inf, window_c=args.window)
    torch.cuda.synchronize()
    print(f"[bench] warmup done", file=sys.stderr, flush=True)

    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eccmi.ecc_msm(ctx, cid, bases, sd, n, out, inf, window_c=args.window)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ctx.stats()
    ctx.set_profiling(False)
    print(f"[bench] timed {args.steps} steps in {dt:.3f}s; phases (ms/step): "
          f"prepare {st['prepare_ms'] / args.steps:.3f} rounds {st['round_ms'] / args.steps:.3f} "
          f"finish {st['finish_ms'] / args.steps:.3f} "
          f"reduce {st['reduce_ms'] / args.steps:.3f} combine {st['combine_ms'] / args.steps:.3f} "
          f"total {st['total_ms'] / args.steps:.3f}", file=sys.stderr, flush=True)

    value = n * args.steps / dt
    per_add = MULS_PER_AFFINE_ADD * MAD32_PER_MUL[cid]
    achieved = st["round_adds"] * per_add / (st["round_ms"] * 1e-3) if st["round_ms"] > 0 else 0.0
    roofline = {
        "bound": "alu",
        "kernel": "k_bucket_round (batch-affine bucket accumulation)",
        "achieved": achieved / 1e12,
        "peak": PEAK_MAD32 / 1e12,
        "unit": "TOP/s",
        "frac": achieved / PEAK_MAD32,
        "traffic": measured_traffic(),
        "per_unit": f"{per_add} MAD32 per batch-affine addition",
        "units_per_launch": st["round_adds"] / max(1, st["round_launches"]),
        "avg_launch_ms": st["round_ms"] / max(1, st["round_launches"]),
        "finishing_pass_ms": st["finish_ms"] / args.steps,
        "msm_frac": value * algorithmic_mad32_per_point(n, bits, cid) / PEAK_MAD32,
    }

    batched = served = configs = table5 = None
    if not args.no_extras and not args.no_configs and cid == 2:
        configs = config_sweep(eccmi, syn, torch, np, ctx, 150.0)
        table5 = table5_sweep(eccmi, syn, torch, np, ctx)
    if not args.no_extras and cid == 2:
        batched = batched_vs_plain(eccmi, syn, torch, np, ctx, cid, args.batch_m, min(512, args.batch_m), 0xBA7C)
        print(f"[bench] batched: {json.dumps(batched)}", file=sys.stderr, flush=True)
        served = serve_mix(eccmi, syn, torch, np, ctx, args.serve_seconds, 0x5E4E)
        print(f"[bench] served: {json.dumps(served)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, n)
        bh = bases[: sample * 2 * L].cpu().numpy().view(np.uint64).reshape(sample, 2 * L)
        cpu = cpu_baseline(bh, s[:sample], cid, L, sample)

    line = {
        "metric": ("MSM points/s (BLS12-381 G1, N=2^20); batched vs plain; p99 verify latency" if cid == 2
                   else "MSM points/s (BN254 G1)"),
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.curve} G1 MSM, N=2^{args.log2n}, uniform {bits}-bit scalars, "
                               f"bases k_i*G, plain (one ecc_msm per MSM), window c={args.window}; "
                               f"inside the call the endomorphism split runs the buckets over 2N points "
                               f"of half-length scalars",
                   "curve": args.curve, "n": n, "window_c": args.window, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "served": served,
        "configs": configs,
        "table5": table5,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
