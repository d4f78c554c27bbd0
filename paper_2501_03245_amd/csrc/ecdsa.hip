// Host side of the signing, verification and point-multiplication calls of
// the C ABI declared in include/ecc_mi.h (secp256r1 and SM2 signatures; point
// multiplication on every curve), and the elementwise field tests.
#include "host.h"

namespace {

template <class C>
ecc_status ensure_gcomb(ecc_ctx* ctx, hipStream_t st);

template <class C>
ecc_status fixed_base_impl(ecc_ctx* ctx, const uint64_t* ks, size_t n, uint64_t* out, const ecc_opts* opts) {
  constexpr int PW = 2 * C::F::N32;  // boundary point words
  const uint32_t flags = opts ? opts->flags : 0u;
  const bool host = flags & ECC_HOST_PTRS;
  hipStream_t st = pick_stream(ctx, opts);
  if (n == 0) return ECC_OK;
  const uint32_t* d_k = reinterpret_cast<const uint32_t*>(ks);
  uint32_t* d_out = reinterpret_cast<uint32_t*>(out);
  if (host) {
    ECC_TRY(ensure(ctx, ctx->stage_a, n * 32));
    ECC_TRY(ensure(ctx, ctx->stage_b, n * PW * 4));
    HIP_TRY(hipMemcpyAsync(ctx->stage_a.p, ks, n * 32, hipMemcpyHostToDevice, st));
    d_k = P<uint32_t>(ctx->stage_a);
    d_out = P<uint32_t>(ctx->stage_b);
  }
  // one mixed addition per scalar byte from the comb table (made by the
  // double-and-add kernel on the first call)
  ECC_TRY(ensure_gcomb<C>(ctx, st));
  k_fixed_base_comb<C, 256><<<ceil_div(n, 256), 256, 0, st>>>(d_k, n, P<uint32_t>(ctx->gcomb[C::ID]), d_out,
                                                              (flags & ECC_IN_MONTGOMERY) ? 1 : 0);
  HIP_TRY(hipGetLastError());
  if (host) HIP_TRY(hipMemcpyAsync(out, d_out, n * PW * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

// 2^j G for j < 256, in the working form the batched-affine verification
// kernel reads (made once per context and curve by the fixed-base kernel)
template <class C>
ecc_status ensure_gtab(ecc_ctx* ctx, hipStream_t st) {
  if (ctx->gtab_ready[C::ID]) return ECC_OK;
  constexpr int IOW = 2 * C::F::N32;
  ECC_TRY(ensure(ctx, ctx->gtab[C::ID], 256 * affine_words<C>() * 4));
  ECC_TRY(ensure(ctx, ctx->stage_d, 256 * 32 + 256 * IOW * 4 + 256));
  std::vector<uint64_t> ks(256 * 4, 0);
  for (int j = 0; j < 256; j++) ks[size_t(j) * 4 + j / 64] = uint64_t(1) << (j % 64);
  uint32_t* d_k = P<uint32_t>(ctx->stage_d);
  uint32_t* d_pts = d_k + 256 * 8;
  uint32_t* d_err = d_pts + 256 * IOW;
  HIP_TRY(hipMemcpyAsync(d_k, ks.data(), ks.size() * 8, hipMemcpyHostToDevice, st));
  ECC_TRY(fill_u32(ctx, d_err, 1, 0u, st));
  k_fixed_base<C, 256><<<1, 256, 0, st>>>(d_k, 256, d_pts, 0);
  HIP_TRY(hipGetLastError());
  k_ingest_points<C><<<1, 256, 0, st>>>(d_pts, P<uint32_t>(ctx->gtab[C::ID]), nullptr, 256, 0, 0, d_err);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  ctx->gtab_ready[C::ID] = true;
  return ECC_OK;
}

// the comb table of the per-lane verification and of signing: d 2^(8 j) G
// for j < 32 and d < 256 in the working form, entry (j, d) at j 256 + d
// (entry d = 0 holds 2^(8 j) G and is never read); made once per context and
// curve by the fixed-base kernel
template <class C>
ecc_status ensure_gcomb(ecc_ctx* ctx, hipStream_t st) {
  if (ctx->gcomb_ready[C::ID]) return ECC_OK;
  constexpr int IOW = 2 * C::F::N32;
  constexpr size_t NE = size_t(VCOMB_WINDOWS) * VCOMB_ENTRIES;
  ECC_TRY(ensure(ctx, ctx->gcomb[C::ID], NE * affine_words<C>() * 4));
  ECC_TRY(ensure(ctx, ctx->stage_d, NE * 32 + NE * IOW * 4 + 256));
  std::vector<uint64_t> ks(NE * 4, 0);
  for (int j = 0; j < VCOMB_WINDOWS; j++)
    for (int d = 0; d < VCOMB_ENTRIES; d++)
      ks[(size_t(j) * VCOMB_ENTRIES + d) * 4 + (8 * j) / 64] = uint64_t(d == 0 ? 1 : d) << ((8 * j) % 64);
  uint32_t* d_k = P<uint32_t>(ctx->stage_d);
  uint32_t* d_pts = d_k + NE * 8;
  uint32_t* d_err = d_pts + NE * IOW;
  HIP_TRY(hipMemcpyAsync(d_k, ks.data(), ks.size() * 8, hipMemcpyHostToDevice, st));
  ECC_TRY(fill_u32(ctx, d_err, 1, 0u, st));
  k_fixed_base<C, 256><<<unsigned(ceil_div(NE, 256)), 256, 0, st>>>(d_k, NE, d_pts, 0);
  HIP_TRY(hipGetLastError());
  k_ingest_points<C><<<unsigned(ceil_div(NE, 256)), 256, 0, st>>>(d_pts, P<uint32_t>(ctx->gcomb[C::ID]), nullptr, NE,
                                                                  0, 0, d_err);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  ctx->gcomb_ready[C::ID] = true;
  return ECC_OK;
}

template <class C>
ecc_status verify_impl(ecc_ctx* ctx, const uint8_t* hashes, const uint64_t* pubkeys, const uint64_t* sigs, size_t m,
                       uint8_t* valid, const ecc_opts* opts) {
  const uint32_t flags = opts ? opts->flags : 0u;
  const bool host = flags & ECC_HOST_PTRS;
  const bool async = flags & ECC_ASYNC;
  hipStream_t st = pick_stream(ctx, opts);
  if (async && host) return fail(ctx, ECC_ERR_ARG, "ECC_ASYNC needs device pointers");
  if (m == 0) return ECC_OK;
  // the per-lane form is faster at every measured batch size (2^8 .. 2^18)
  const bool per_lane = !(flags & ECC_VERIFY_BATCHED);
  if (per_lane) {
    ECC_TRY(ensure_gcomb<C>(ctx, st));
    const size_t lanes = ceil_div(std::min(m, VERIFY_LANE_CHUNK), VERIFY_LANE_WG) * VERIFY_LANE_WG;
    ECC_TRY(ensure(ctx, ctx->vscr, lanes * VT_N * vt_slot<typename C::F>() * 4));
  } else {
    ECC_TRY(ensure_gtab<C>(ctx, st));
  }
  const uint8_t* d_h = hashes;
  const uint32_t* d_q = reinterpret_cast<const uint32_t*>(pubkeys);
  const uint32_t* d_s = reinterpret_cast<const uint32_t*>(sigs);
  uint8_t* d_v = valid;
  if (host) {
    ECC_TRY(ensure(ctx, ctx->stage_a, m * 64));
    ECC_TRY(ensure(ctx, ctx->stage_b, m * 64));
    ECC_TRY(ensure(ctx, ctx->stage_c, m * 32 + m + 64));
    HIP_TRY(hipMemcpyAsync(ctx->stage_a.p, pubkeys, m * 64, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ctx->stage_b.p, sigs, m * 64, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ctx->stage_c.p, hashes, m * 32, hipMemcpyHostToDevice, st));
    d_q = P<uint32_t>(ctx->stage_a);
    d_s = P<uint32_t>(ctx->stage_b);
    d_h = P<uint8_t>(ctx->stage_c);
    d_v = P<uint8_t>(ctx->stage_c) + m * 32;
  }
  if (per_lane) {
    for (size_t off = 0; off < m; off += VERIFY_LANE_CHUNK) {
      const size_t c = std::min(VERIFY_LANE_CHUNK, m - off);
      k_verify_xyzz<C, VERIFY_LANE_WG><<<ceil_div(c, VERIFY_LANE_WG), VERIFY_LANE_WG, 0, st>>>(
          d_h + off * 32, d_q + off * 16, d_s + off * 16, c, P<uint32_t>(ctx->gcomb[C::ID]), P<uint32_t>(ctx->vscr),
          d_v + off);
      HIP_TRY(hipGetLastError());
    }
  } else {
    k_verify<C, VERIFY_WG><<<ceil_div(m, VERIFY_WG), VERIFY_WG, 0, st>>>(d_h, d_q, d_s, m,
                                                                        P<uint32_t>(ctx->gtab[C::ID]), d_v);
    HIP_TRY(hipGetLastError());
  }
  if (async) {
    if (std::find(ctx->pending.begin(), ctx->pending.end(), st) == ctx->pending.end()) ctx->pending.push_back(st);
    return ECC_OK;
  }
  if (host) HIP_TRY(hipMemcpyAsync(valid, d_v, m, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

template <class C>
ecc_status sign_impl(ecc_ctx* ctx, const uint8_t* hashes, const uint64_t* privkeys, const uint64_t* nonces, size_t m,
                     uint64_t* sigs, const ecc_opts* opts) {
  const uint32_t flags = opts ? opts->flags : 0u;
  const bool host = flags & ECC_HOST_PTRS;
  hipStream_t st = pick_stream(ctx, opts);
  if (m == 0) return ECC_OK;
  ECC_TRY(ensure_gcomb<C>(ctx, st));
  const uint8_t* d_h = hashes;
  const uint32_t* d_d = reinterpret_cast<const uint32_t*>(privkeys);
  const uint32_t* d_k = reinterpret_cast<const uint32_t*>(nonces);
  uint32_t* d_s = reinterpret_cast<uint32_t*>(sigs);
  if (host) {
    ECC_TRY(ensure(ctx, ctx->stage_a, m * 32));
    ECC_TRY(ensure(ctx, ctx->stage_b, m * 32));
    ECC_TRY(ensure(ctx, ctx->stage_c, m * 32 + m * 64));
    HIP_TRY(hipMemcpyAsync(ctx->stage_a.p, privkeys, m * 32, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ctx->stage_b.p, nonces, m * 32, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ctx->stage_c.p, hashes, m * 32, hipMemcpyHostToDevice, st));
    d_d = P<uint32_t>(ctx->stage_a);
    d_k = P<uint32_t>(ctx->stage_b);
    d_h = P<uint8_t>(ctx->stage_c);
    d_s = reinterpret_cast<uint32_t*>(P<uint8_t>(ctx->stage_c) + m * 32);
  }
  k_sign<C, SIGN_WG><<<ceil_div(m, SIGN_WG), SIGN_WG, 0, st>>>(d_h, d_d, d_k, m, P<uint32_t>(ctx->gcomb[C::ID]), d_s);
  HIP_TRY(hipGetLastError());
  if (host) HIP_TRY(hipMemcpyAsync(sigs, d_s, m * 64, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

template <class C>
ecc_status pmul_impl(ecc_ctx* ctx, const uint64_t* pts, const uint64_t* ks, size_t n, uint64_t* out,
                     const ecc_opts* opts) {
  using F = typename C::F;
  constexpr int IOW = 2 * F::N32;  // boundary point words
  constexpr int PW = affine_words<C>();
  const uint32_t flags = opts ? opts->flags : 0u;
  const bool host = flags & ECC_HOST_PTRS;
  const int mont = (flags & ECC_IN_MONTGOMERY) ? 1 : 0;
  hipStream_t st = pick_stream(ctx, opts);
  if (n == 0) return ECC_OK;
  const uint32_t* d_p = reinterpret_cast<const uint32_t*>(pts);
  const uint32_t* d_k = reinterpret_cast<const uint32_t*>(ks);
  uint32_t* d_out = reinterpret_cast<uint32_t*>(out);
  if (host) {
    ECC_TRY(ensure(ctx, ctx->stage_a, n * IOW * 4));
    ECC_TRY(ensure(ctx, ctx->stage_b, n * 32));
    ECC_TRY(ensure(ctx, ctx->stage_c, n * IOW * 4));
    HIP_TRY(hipMemcpyAsync(ctx->stage_a.p, pts, n * IOW * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ctx->stage_b.p, ks, n * 32, hipMemcpyHostToDevice, st));
    d_p = P<uint32_t>(ctx->stage_a);
    d_k = P<uint32_t>(ctx->stage_b);
    d_out = P<uint32_t>(ctx->stage_c);
  }
  const size_t lanes = ceil_div(std::min(n, VERIFY_LANE_CHUNK), PMUL_WG) * PMUL_WG;
  ECC_TRY(ensure(ctx, ctx->upts, n * PW * 4));
  if (!(flags & ECC_PMUL_BATCHED)) ECC_TRY(ensure(ctx, ctx->vscr, lanes * VT_N * vt_slot<F>() * 4));
  ECC_TRY(ensure(ctx, ctx->flags, 256));
  uint32_t* d_err = P<uint32_t>(ctx->flags);
  ECC_TRY(fill_u32(ctx, d_err, 1, 0u, st));
  // range and curve checks of every point before any output is written
  k_ingest_points<C><<<ceil_div(n, 256), 256, 0, st>>>(d_p, P<uint32_t>(ctx->upts), nullptr, n, mont, 1, d_err);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(ctx->host_small, d_err, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->host_small[0] & ERRF_RANGE) return fail(ctx, ECC_ERR_RANGE, "a point coordinate is >= p");
  if (ctx->host_small[0] & ERRF_NOT_ON_CURVE) return fail(ctx, ECC_ERR_NOT_ON_CURVE, "a point is not on the curve");
  if (flags & ECC_PMUL_BATCHED) {
    // Algorithm 3: about UPMUL_KPER requests per lane on at most the lanes
    // that are resident at once
    int& blocks = ctx->upmul_blocks[C::ID];
    if (blocks == 0) {
      int b = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_upmul_affine<C, UPMUL_WG>, UPMUL_WG, 0));
      blocks = std::max(1, b);
    }
    const size_t cap = size_t(blocks) * size_t(ctx->cu_count) * UPMUL_WG;
    size_t T = size_t(ceil_div(ceil_div(n, UPMUL_KPER), UPMUL_WG)) * UPMUL_WG;
    T = std::max<size_t>(UPMUL_WG, std::min(T, cap));
    const size_t kper = (n + T - 1) / T;
    ECC_TRY(ensure(ctx, ctx->vscr, T * kper * upmul_state_words<F>() * 4));
    k_upmul_affine<C, UPMUL_WG><<<unsigned(T / UPMUL_WG), UPMUL_WG, 0, st>>>(
        P<uint32_t>(ctx->upts), d_k, n, uint32_t(kper), P<uint32_t>(ctx->vscr), d_out, mont);
    HIP_TRY(hipGetLastError());
  }
  for (size_t off = 0; off < n && !(flags & ECC_PMUL_BATCHED); off += VERIFY_LANE_CHUNK) {
    const size_t c = std::min(VERIFY_LANE_CHUNK, n - off);
    k_pmul<C, PMUL_WG><<<ceil_div(c, PMUL_WG), PMUL_WG, 0, st>>>(P<uint32_t>(ctx->upts) + off * PW, d_k + off * 8, c,
                                                                 P<uint32_t>(ctx->vscr), d_out + off * IOW, mont);
    HIP_TRY(hipGetLastError());
  }
  if (host) HIP_TRY(hipMemcpyAsync(out, d_out, n * IOW * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

}  // namespace

extern "C" {

ecc_status ecc_verify_batch(ecc_ctx* ctx, ecc_curve curve, const uint8_t* hashes, const uint64_t* pubkeys,
                            const uint64_t* sigs, size_t m, uint8_t* valid, const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (m == 0) return ECC_OK;
  if (!hashes || !pubkeys || !sigs || !valid) return fail(ctx, ECC_ERR_ARG, "null pointer with m > 0");
  if (m > (size_t(1) << 30)) return fail(ctx, ECC_ERR_ARG, "m = %zu exceeds 2^30", m);
  if (opts && (opts->flags & ~uint32_t(ECC_HOST_PTRS | ECC_VERIFY_BATCHED | ECC_VERIFY_PER_LANE | ECC_ASYNC)))
    return fail(ctx, ECC_ERR_ARG, "unsupported flag bits 0x%x", opts->flags);
  if (opts && (opts->flags & ECC_VERIFY_BATCHED) && (opts->flags & ECC_VERIFY_PER_LANE))
    return fail(ctx, ECC_ERR_ARG, "ECC_VERIFY_BATCHED and ECC_VERIFY_PER_LANE together");
  switch (curve) {
    case ECC_SECP256R1: return verify_impl<P256>(ctx, hashes, pubkeys, sigs, m, valid, opts);
    case ECC_SM2: return verify_impl<SM2>(ctx, hashes, pubkeys, sigs, m, valid, opts);
    case ECC_BN254_G1:
    case ECC_BLS12_381_G1: {
      // no ECDSA keys live on these curves: every request is invalid
      if (opts && (opts->flags & ECC_HOST_PTRS)) {
        memset(valid, 0, m);
        return ECC_OK;
      }
      hipStream_t st = pick_stream(ctx, opts);
      k_fill_u8<<<ceil_div(m, 256), 256, 0, st>>>(valid, m, 0);
      HIP_TRY(hipGetLastError());
      if (opts && (opts->flags & ECC_ASYNC)) {
        if (std::find(ctx->pending.begin(), ctx->pending.end(), st) == ctx->pending.end()) ctx->pending.push_back(st);
        return ECC_OK;
      }
      HIP_TRY(hipStreamSynchronize(st));
      return ECC_OK;
    }
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_sign_batch(ecc_ctx* ctx, ecc_curve curve, const uint8_t* hashes, const uint64_t* privkeys,
                          const uint64_t* nonces, size_t m, uint64_t* sigs, const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (m == 0) return ECC_OK;
  if (!hashes || !privkeys || !nonces || !sigs) return fail(ctx, ECC_ERR_ARG, "null pointer with m > 0");
  if (m > (size_t(1) << 30)) return fail(ctx, ECC_ERR_ARG, "m = %zu exceeds 2^30", m);
  if (opts && (opts->flags & ~uint32_t(ECC_HOST_PTRS)))
    return fail(ctx, ECC_ERR_ARG, "unsupported flag bits 0x%x", opts->flags);
  switch (curve) {
    case ECC_SECP256R1: return sign_impl<P256>(ctx, hashes, privkeys, nonces, m, sigs, opts);
    case ECC_SM2: return sign_impl<SM2>(ctx, hashes, privkeys, nonces, m, sigs, opts);
    default: return fail(ctx, ECC_ERR_UNSUPPORTED, "signing is provided for secp256r1 and SM2");
  }
}

ecc_status ecc_pmul_batch(ecc_ctx* ctx, ecc_curve curve, const uint64_t* points, const uint64_t* scalars, size_t n,
                          uint64_t* out_xy, const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (n == 0) return ECC_OK;
  if (!points || !scalars || !out_xy) return fail(ctx, ECC_ERR_ARG, "null pointer with n > 0");
  if (n > (size_t(1) << 30)) return fail(ctx, ECC_ERR_ARG, "n = %zu exceeds 2^30", n);
  if (opts && (opts->flags & ~uint32_t(ECC_IN_MONTGOMERY | ECC_HOST_PTRS | ECC_PMUL_BATCHED)))
    return fail(ctx, ECC_ERR_ARG, "unsupported flag bits 0x%x", opts->flags);
  switch (curve) {
    case ECC_BN254_G1: return pmul_impl<BN254>(ctx, points, scalars, n, out_xy, opts);
    case ECC_BLS12_381_G1: return pmul_impl<BLS12_381>(ctx, points, scalars, n, out_xy, opts);
    case ECC_SECP256R1: return pmul_impl<P256>(ctx, points, scalars, n, out_xy, opts);
    case ECC_SM2: return pmul_impl<SM2>(ctx, points, scalars, n, out_xy, opts);
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_fixed_base_mul(ecc_ctx* ctx, ecc_curve curve, const uint64_t* ks, size_t n, uint64_t* out_xy,
                              const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (n && (!ks || !out_xy)) return fail(ctx, ECC_ERR_ARG, "null pointer with n > 0");
  if (opts && (opts->flags & ~uint32_t(ECC_IN_MONTGOMERY | ECC_HOST_PTRS)))
    return fail(ctx, ECC_ERR_ARG, "unsupported flag bits 0x%x", opts->flags);
  switch (curve) {
    case ECC_BN254_G1: return fixed_base_impl<BN254>(ctx, ks, n, out_xy, opts);
    case ECC_BLS12_381_G1: return fixed_base_impl<BLS12_381>(ctx, ks, n, out_xy, opts);
    case ECC_SECP256R1: return fixed_base_impl<P256>(ctx, ks, n, out_xy, opts);
    case ECC_SM2: return fixed_base_impl<SM2>(ctx, ks, n, out_xy, opts);
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

}  // extern "C"
