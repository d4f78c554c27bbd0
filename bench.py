#!/usr/bin/env python3
"""Benchmark: multi-scalar multiplication throughput on one MI355X.

Workload (default): BLS12-381 G1 MSM of N = 2^20 points, uniform 255-bit
scalars, seeded bases P_i = k_i G (k_i uniform in [1, r)), Pippenger window
c = 16.  Bases and scalars are generated on the device before the timed
region; one step is one ecc_msm call over the resident inputs.

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
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (the reference "
                         "for scaling HBM byte counters), then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
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
        "traffic": None,
        "per_unit": f"{per_add} MAD32 per batch-affine addition",
        "units_per_launch": st["round_adds"] / max(1, st["round_launches"]),
        "avg_launch_ms": st["round_ms"] / max(1, st["round_launches"]),
        "msm_frac": value * algorithmic_mad32_per_point(n, bits, cid) / PEAK_MAD32,
    }

    cpu = None
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, n)
        bh = bases[: sample * 2 * L].cpu().numpy().view(np.uint64).reshape(sample, 2 * L)
        cpu = cpu_baseline(bh, s[:sample], cid, L, sample)

    line = {
        "metric": "MSM points/s (BLS12-381 G1, N=2^20)" if cid == 2 else "MSM points/s (BN254 G1)",
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
                               f"bases k_i*G, plain (one ecc_msm per MSM), window c={args.window}",
                   "curve": args.curve, "n": n, "window_c": args.window, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
