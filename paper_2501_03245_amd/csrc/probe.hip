// Issue-rate probe of the instructions a field product is built from: the
// 32x32+64 -> 64 integer multiply-add (v_mad_u64_u32, one per limb product of
// Algorithm 2), the 32-bit low multiply (v_mul_lo_u32, the q_inv step of each
// reduction row) and, for comparison, the double-precision fused multiply-add
// (v_fma_f64).  It is a measurement, not a step of the path: the rate it
// reports is the attainable ceiling that the ALU-bound kernels are judged
// against, next to the nominal 64 lane-operations per compute unit and clock.
//
// Every lane runs CHAINS interleaved dependency chains of one instruction;
// one chain exposes the instruction's latency, several expose its issue rate.
// The number of waves per SIMD is set by the grid (one 256-lane workgroup,
// four waves, per compute unit and wave slot).
#include "host.h"

namespace {

enum : int { PROBE_MAD_U64_U32 = 0, PROBE_FMA_F64 = 1, PROBE_MUL_LO_U32 = 2 };
constexpr int PROBE_WG = 256;
constexpr int PROBE_UNROLL = 16;

template <int OP, int CHAINS>
__global__ void __launch_bounds__(PROBE_WG) k_probe_issue(uint32_t iters, uint64_t* __restrict__ sink,
                                                          long long* __restrict__ clocks) {
  const uint32_t seed = blockIdx.x * PROBE_WG + threadIdx.x;
  const uint32_t a = seed * 2654435761u | 1u, b = seed ^ 0x9e3779b9u;
  const double fa = 1.0 + 1e-12 * double(seed & 255), fb = 1e-9;
  uint64_t acc[CHAINS];
  double facc[CHAINS];
  uint32_t macc[CHAINS];
#pragma unroll
  for (int j = 0; j < CHAINS; j++) {
    acc[j] = seed + j;
    facc[j] = double(j);
    macc[j] = seed + 3u * j;
  }
  const long long c0 = clock64(), w0 = wall_clock64();
  for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; u++) {
#pragma unroll
      for (int j = 0; j < CHAINS; j++) {
        if constexpr (OP == PROBE_MAD_U64_U32) {
          uint64_t cy;
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[j]), "=s"(cy) : "v"(a), "v"(b));
        } else if constexpr (OP == PROBE_FMA_F64) {
          asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(facc[j]) : "v"(fa), "v"(fb));
        } else {
          asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(macc[j]) : "v"(a));
        }
      }
    }
  }
  const long long c1 = clock64(), w1 = wall_clock64();
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < CHAINS; j++) s += acc[j] + uint64_t(facc[j]) + macc[j];
  sink[seed] = s;
  if (threadIdx.x == 0) {
    clocks[2 * blockIdx.x] = c1 - c0;
    clocks[2 * blockIdx.x + 1] = w1 - w0;
  }
}

template <int OP>
void launch_probe(int chains, uint32_t blocks, uint32_t iters, uint64_t* sink, long long* clocks, hipStream_t st) {
  switch (chains) {
    case 1: k_probe_issue<OP, 1><<<blocks, PROBE_WG, 0, st>>>(iters, sink, clocks); break;
    case 2: k_probe_issue<OP, 2><<<blocks, PROBE_WG, 0, st>>>(iters, sink, clocks); break;
    case 4: k_probe_issue<OP, 4><<<blocks, PROBE_WG, 0, st>>>(iters, sink, clocks); break;
    default: k_probe_issue<OP, 8><<<blocks, PROBE_WG, 0, st>>>(iters, sink, clocks); break;
  }
}

}  // namespace

extern "C" {

ecc_status ecc_probe_issue_rate(ecc_ctx* ctx, int op, int chains, int waves_per_simd, uint32_t iters, double* ms,
                                double* lane_ops, double* shader_mhz) {
  ECC_TRY(enter(ctx));
  if (op < 0 || op > 2) return fail(ctx, ECC_ERR_ARG, "op %d outside [0, 2]", op);
  if (chains != 1 && chains != 2 && chains != 4 && chains != 8)
    return fail(ctx, ECC_ERR_ARG, "chains %d not 1, 2, 4 or 8", chains);
  if (waves_per_simd < 1 || waves_per_simd > 8) return fail(ctx, ECC_ERR_ARG, "waves per SIMD %d outside [1, 8]", waves_per_simd);
  if (iters < 1 || iters > (1u << 20)) return fail(ctx, ECC_ERR_ARG, "iters %u outside [1, 2^20]", iters);
  if (!ms || !lane_ops || !shader_mhz) return fail(ctx, ECC_ERR_ARG, "null pointer");
  const uint32_t blocks = uint32_t(ctx->cu_count) * uint32_t(waves_per_simd);
  const size_t lanes = size_t(blocks) * PROBE_WG;
  ECC_TRY(ensure(ctx, ctx->stage_a, lanes * 8));
  ECC_TRY(ensure(ctx, ctx->stage_b, size_t(blocks) * 16));
  hipStream_t st = ctx->stream;
  uint64_t* sink = P<uint64_t>(ctx->stage_a);
  long long* clocks = P<long long>(ctx->stage_b);
  hipEvent_t e0, e1;
  ECC_TRY(ev(ctx, 0, &e0));
  ECC_TRY(ev(ctx, 1, &e1));
  for (int rep = 0; rep < 2; rep++) {  // the first launch warms up
    HIP_TRY(hipEventRecord(e0, st));
    switch (op) {
      case PROBE_MAD_U64_U32: launch_probe<PROBE_MAD_U64_U32>(chains, blocks, iters, sink, clocks, st); break;
      case PROBE_FMA_F64: launch_probe<PROBE_FMA_F64>(chains, blocks, iters, sink, clocks, st); break;
      default: launch_probe<PROBE_MUL_LO_U32>(chains, blocks, iters, sink, clocks, st); break;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e1, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  std::vector<long long> cl(2 * size_t(blocks));
  HIP_TRY(hipMemcpy(cl.data(), clocks, cl.size() * sizeof(long long), hipMemcpyDeviceToHost));
  int wall_khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ctx->device));
  double cyc = 0.0, wall = 0.0;
  for (uint32_t i = 0; i < blocks; i++) {
    cyc += double(cl[2 * i]);
    wall += double(cl[2 * i + 1]);
  }
  *ms = double(t);
  *lane_ops = double(lanes) * double(iters) * PROBE_UNROLL * chains;
  *shader_mhz = wall > 0.0 ? cyc / wall * (double(wall_khz) * 1e-3) : 0.0;
  return ECC_OK;
}

}  // extern "C"
