// Elementwise entry points of the C ABI (include/ecc_mi.h) that expose single
// steps of the path to the parity tests: field product and inverse, the
// lane-parallel field of the window combination, and the batch-affine
// addition of the bucket rounds.  They take device pointers only.
#include "host.h"

namespace {

template <class C>
ecc_status test_fp_mul_impl(ecc_ctx* ctx, const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n) {
  if (n == 0) return ECC_OK;
  k_test_fp_mul<C><<<ceil_div(n, 256), 256, 0, ctx->stream>>>(reinterpret_cast<const uint32_t*>(a),
                                                               reinterpret_cast<const uint32_t*>(b),
                                                               reinterpret_cast<uint32_t*>(out), n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ECC_OK;
}

template <class C>
ecc_status test_lane_field_impl(ecc_ctx* ctx, int op, const uint64_t* a, const uint64_t* b, uint64_t* out,
                                size_t n) {
  if (op < 0 || op > 7) return fail(ctx, ECC_ERR_ARG, "op %d outside [0, 7]", op);
  if (n == 0) return ECC_OK;
  k_test_lane_field<C><<<ceil_div(n, 4), 64, 0, ctx->stream>>>(reinterpret_cast<const uint32_t*>(a),
                                                                reinterpret_cast<const uint32_t*>(b),
                                                                reinterpret_cast<uint32_t*>(out), n, op);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ECC_OK;
}

template <class C>
ecc_status test_fp_inv_impl(ecc_ctx* ctx, const uint64_t* a, uint64_t* out, size_t n) {
  if (n == 0) return ECC_OK;
  k_test_fp_inv<C, 256><<<ceil_div(n, 256), 256, 0, ctx->stream>>>(reinterpret_cast<const uint32_t*>(a),
                                                                    reinterpret_cast<uint32_t*>(out), n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ECC_OK;
}

template <class C>
ecc_status test_batch_add_impl(ecc_ctx* ctx, const uint64_t* p, const uint64_t* q, uint64_t* out, size_t n) {
  constexpr int NL = C::F::NL;
  constexpr int PW = affine_words<C>();
  if (n == 0) return ECC_OK;
  if (n > (1u << 30)) return fail(ctx, ECC_ERR_ARG, "n too large");
  hipStream_t st = ctx->stream;
  // the round kernel at its default occupancy target, on the lanes that fit at once
  int bpc = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_bucket_round<C, ROUND_WG, ROUND_OCC>, ROUND_WG, 0));
  const uint32_t lanes_max = uint32_t(std::max(1, bpc)) * uint32_t(ctx->cu_count) * ROUND_WG;
  const size_t cap = 2 * n;
  ECC_TRY(ensure(ctx, ctx->slots, cap * PW * 4));
  ECC_TRY(ensure(ctx, ctx->slots2, cap * PW * 4));
  ECC_TRY(ensure(ctx, ctx->desc, n * 8));
  ECC_TRY(ensure(ctx, ctx->mscr, (n + lanes_max + ROUND_WG) * NL * 4));
  ECC_TRY(ensure(ctx, ctx->flags, (2 + 2 * MAX_ROUNDS) * 4));
  ECC_TRY(ensure(ctx, ctx->rparams, (MAX_ROUNDS + 1) * sizeof(uint4)));
  uint32_t* in_x = P<uint32_t>(ctx->slots);
  uint32_t* in_y = in_x + cap * C::F::CW;
  uint32_t* out_x = P<uint32_t>(ctx->slots2);
  uint32_t* out_y = out_x + cap * C::F::CW;
  k_test_pairs_in<C><<<ceil_div(n, 256), 256, 0, st>>>(reinterpret_cast<const uint32_t*>(p),
                                                        reinterpret_cast<const uint32_t*>(q), in_x, in_y,
                                                        P<uint2>(ctx->desc), n);
  HIP_TRY(hipGetLastError());
  uint32_t* d_na = P<uint32_t>(ctx->flags) + 1;
  ECC_TRY(fill_u32(ctx, d_na, 2 * MAX_ROUNDS + 1, 0u, st));
  ECC_TRY(fill_u32(ctx, d_na, 1, uint32_t(n), st));
  k_round_params<<<1, 64, 0, st>>>(d_na, lanes_max, ROUND_WG, KMIN, P<uint4>(ctx->rparams), d_na + 2 * MAX_ROUNDS, 0u);
  HIP_TRY(hipGetLastError());
  uint32_t blocks = round_lane_count(uint32_t(n), lanes_max, ROUND_WG, KMIN) / ROUND_WG;
  k_bucket_round<C, ROUND_WG, ROUND_OCC><<<blocks, ROUND_WG, 0, st>>>(
      nullptr, nullptr, in_x, in_y, out_x, out_y, P<uint2>(ctx->desc), P<uint4>(ctx->rparams), 0,
      P<uint32_t>(ctx->mscr), nullptr, d_na + MAX_ROUNDS);
  HIP_TRY(hipGetLastError());
  k_test_pairs_out<C><<<ceil_div(n, 256), 256, 0, st>>>(out_x, out_y, reinterpret_cast<uint32_t*>(out), n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

}  // namespace

extern "C" {

ecc_status ecc_test_fp_mul(ecc_ctx* ctx, ecc_curve curve, const uint64_t* a, const uint64_t* b, uint64_t* out,
                           size_t n) {
  ECC_TRY(enter(ctx));
  if (n && (!a || !b || !out)) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1: return test_fp_mul_impl<BN254>(ctx, a, b, out, n);
    case ECC_BLS12_381_G1: return test_fp_mul_impl<BLS12_381>(ctx, a, b, out, n);
    case ECC_SECP256R1: return test_fp_mul_impl<P256>(ctx, a, b, out, n);
    case ECC_SM2: return test_fp_mul_impl<SM2>(ctx, a, b, out, n);
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_test_lane_field(ecc_ctx* ctx, ecc_curve curve, int op, const uint64_t* a, const uint64_t* b,
                               uint64_t* out, size_t n) {
  ECC_TRY(enter(ctx));
  if (n && (!a || !b || !out)) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1: return test_lane_field_impl<BN254>(ctx, op, a, b, out, n);
    case ECC_BLS12_381_G1: return test_lane_field_impl<BLS12_381>(ctx, op, a, b, out, n);
    case ECC_SECP256R1: return test_lane_field_impl<P256>(ctx, op, a, b, out, n);
    case ECC_SM2: return test_lane_field_impl<SM2>(ctx, op, a, b, out, n);
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_test_fp_inv(ecc_ctx* ctx, ecc_curve curve, const uint64_t* a, uint64_t* out, size_t n) {
  ECC_TRY(enter(ctx));
  if (n && (!a || !out)) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1: return test_fp_inv_impl<BN254>(ctx, a, out, n);
    case ECC_BLS12_381_G1: return test_fp_inv_impl<BLS12_381>(ctx, a, out, n);
    case ECC_SECP256R1: return test_fp_inv_impl<P256>(ctx, a, out, n);
    case ECC_SM2: return test_fp_inv_impl<SM2>(ctx, a, out, n);
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_test_batch_add(ecc_ctx* ctx, ecc_curve curve, const uint64_t* p, const uint64_t* q, uint64_t* out,
                              size_t n) {
  ECC_TRY(enter(ctx));
  if (n && (!p || !q || !out)) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1: return test_batch_add_impl<BN254>(ctx, p, q, out, n);
    case ECC_BLS12_381_G1: return test_batch_add_impl<BLS12_381>(ctx, p, q, out, n);
    case ECC_SECP256R1: return test_batch_add_impl<P256>(ctx, p, q, out, n);
    case ECC_SM2: return test_batch_add_impl<SM2>(ctx, p, q, out, n);
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

}  // extern "C"
