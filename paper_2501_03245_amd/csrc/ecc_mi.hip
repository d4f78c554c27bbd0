// Host side of the C ABI declared in include/ecc_mi.h: argument checks,
// device scratch management and the launch sequence of the MSM path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ecc_mi.h"
#include "kernels.h"

using namespace eccmi;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

constexpr int ROUND_WG = 256;
constexpr int PLAN_WG = 256;
constexpr int REDUCE_WG = 256;
constexpr int KMIN = 8;  // target additions per lane in a round

}  // namespace

struct ecc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t held = 0;
  std::string err;
  DevBuf bases, skip, counts, offsets, cursor, sorted, slots, desc, desc_base, mscr, segS, segT, winsum, flags,
      scan_tmp, stage_a, stage_b, stage_c, stage_d;
  uint32_t* host_small = nullptr;  // pinned readback area
  int cu_count = 256;
  int round_blocks[4] = {0, 0, 0, 0};  // resident round workgroups per CU, by curve id
  bool profiling = false;
  ecc_stats stats{};
  std::vector<hipEvent_t> events;  // pool for per-phase timing
};

namespace {

ecc_status fail(ecc_ctx* ctx, ecc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  ctx->err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(ctx, ECC_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define ECC_TRY(expr)              \
  do {                             \
    ecc_status s_ = (expr);        \
    if (s_ != ECC_OK) return s_;   \
  } while (0)

ecc_status ensure(ecc_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return ECC_OK;
  size_t want = std::max(bytes, b.cap + b.cap / 4);
  want = (want + 4095) & ~size_t(4095);
  if (ctx->budget && ctx->held - b.cap + want > ctx->budget) {
    want = (bytes + 4095) & ~size_t(4095);
    if (ctx->held - b.cap + want > ctx->budget)
      return fail(ctx, ECC_ERR_NOMEM, "HBM budget of %zu bytes exceeded (need %zu more)", ctx->budget,
                  want - b.cap);
  }
  if (b.p) {
    HIP_TRY(hipFree(b.p));
    ctx->held -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, ECC_ERR_NOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
  }
  b.cap = want;
  ctx->held += want;
  return ECC_OK;
}

// event pool: ev(ctx, i) returns the i-th event, creating it on first use
ecc_status ev(ecc_ctx* ctx, size_t i, hipEvent_t* out) {
  while (ctx->events.size() <= i) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    ctx->events.push_back(e);
  }
  *out = ctx->events[i];
  return ECC_OK;
}

ecc_status record(ecc_ctx* ctx, size_t i, hipStream_t st) {
  if (!ctx->profiling) return ECC_OK;
  hipEvent_t e;
  ECC_TRY(ev(ctx, i, &e));
  HIP_TRY(hipEventRecord(e, st));
  return ECC_OK;
}

double elapsed(ecc_ctx* ctx, size_t a, size_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->events[a], ctx->events[b]) != hipSuccess) return 0.0;
  return double(ms);
}

// lanes of the bucket-round kernel that fit on the device at once: a round's
// additions are spread over exactly these lanes so each lane runs one chain
template <class C>
ecc_status round_lanes(ecc_ctx* ctx, uint32_t* lanes) {
  int& blocks = ctx->round_blocks[C::ID];
  if (blocks == 0) {
    int b = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_bucket_round<C, ROUND_WG>, ROUND_WG, 0));
    blocks = std::max(1, b);
  }
  *lanes = uint32_t(blocks) * uint32_t(ctx->cu_count) * ROUND_WG;
  return ECC_OK;
}

template <class T>
T* P(DevBuf& b) {
  return static_cast<T*>(b.p);
}

inline uint32_t ceil_div(size_t a, size_t b) { return uint32_t((a + b - 1) / b); }

hipStream_t pick_stream(ecc_ctx* ctx, const ecc_opts* o) {
  return (o && o->stream) ? static_cast<hipStream_t>(o->stream) : ctx->stream;
}

int bit_length(uint64_t v) {
  int b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}

// exclusive scan of n u32 (in and out may not alias)
ecc_status scan_u32(ecc_ctx* ctx, const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp, size_t tmp_words,
                    hipStream_t st) {
  uint32_t tiles = ceil_div(n, SCAN_TILE);
  if (tmp_words < 2 * size_t(tiles)) return fail(ctx, ECC_ERR_ARG, "scan scratch too small");
  uint32_t* sums = tmp;
  uint32_t* sums_scan = tmp + tiles;
  k_scan_tiles<<<tiles, SCAN_WG, 0, st>>>(in, out, sums, n);
  HIP_TRY(hipGetLastError());
  if (tiles > 1) {
    ECC_TRY(scan_u32(ctx, sums, sums_scan, tiles, tmp + 2 * size_t(tiles), tmp_words - 2 * size_t(tiles), st));
    k_scan_add<<<ceil_div(n, 256), 256, 0, st>>>(out, sums_scan, n);
    HIP_TRY(hipGetLastError());
  }
  return ECC_OK;
}

size_t scan_tmp_words(size_t n) {
  size_t w = 0;
  while (true) {
    size_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    w += 2 * tiles;
    if (tiles <= 1) break;
    n = tiles;
  }
  return w + 16;
}

int default_window(int curve, size_t n) {
  // fewer buckets than points per window keeps the reduction small; the
  // tuned table replaces this rule of thumb where one exists
  int lg = bit_length(n ? n : 1) - 1;
  int c = lg - 4;
  if (curve == ECC_BLS12_381_G1 && n >= (1u << 18)) c = lg - 4;
  return std::max(4, std::min(16, c));
}

struct Plan {
  int c, W, bits;
  uint32_t D, B;
  size_t E_max;
  int rounds_bound;
  size_t desc_base[MAX_ROUNDS];
  size_t desc_total;
};

template <class C>
Plan make_plan(size_t n, int c) {
  Plan p{};
  p.c = c;
  p.bits = C::SCALAR_BITS;
  p.W = (p.bits + 1 + c - 1) / c;
  p.D = 1u << (c - 1);
  p.B = uint32_t(p.W) * p.D;
  p.E_max = n * size_t(p.W);
  p.rounds_bound = std::min(MAX_ROUNDS, bit_length(n));
  size_t acc = 0;
  size_t nonempty = std::min<size_t>(p.B, p.E_max);
  for (int r = 0; r < MAX_ROUNDS; r++) {
    p.desc_base[r] = acc;
    if (r < p.rounds_bound) acc += (p.E_max >> (r + 1)) + nonempty / 2 + 1;
  }
  p.desc_total = acc;
  return p;
}

// ---------------------------------------------------------------------------

template <class C>
ecc_status msm_impl(ecc_ctx* ctx, const uint64_t* bases_in, const uint64_t* scalars_in, size_t n, uint64_t* out_xy,
                    uint8_t* out_inf, const ecc_opts* opts) {
  using F = typename C::F;
  constexpr int NL = F::NL;
  constexpr int IOW = 2 * F::N32;            // words of a boundary point
  constexpr int PW = affine_words<C>();      // words of a stored working-form point
  constexpr int XW = xyzz_words<C>();
  const uint32_t flags = opts ? opts->flags : 0u;
  const bool host = flags & ECC_HOST_PTRS;
  hipStream_t st = pick_stream(ctx, opts);
  int c = (opts && opts->window_c) ? opts->window_c : default_window(C::ID, n);
  if (c < 2 || c > 20) return fail(ctx, ECC_ERR_ARG, "window_c %d outside [2, 20]", c);

  uint32_t* d_out = reinterpret_cast<uint32_t*>(out_xy);
  uint8_t* d_inf = out_inf;
  if (host) {
    ECC_TRY(ensure(ctx, ctx->stage_c, IOW * 4 + 64));
    d_out = P<uint32_t>(ctx->stage_c);
    d_inf = reinterpret_cast<uint8_t*>(d_out + IOW);
  }
  if (n == 0) {
    k_write_inf<C><<<1, 64, 0, st>>>(d_out, d_inf, 1);
    HIP_TRY(hipGetLastError());
  } else {
    const uint32_t* d_bases_in = reinterpret_cast<const uint32_t*>(bases_in);
    const uint32_t* d_scalars = reinterpret_cast<const uint32_t*>(scalars_in);
    if (host) {
      ECC_TRY(ensure(ctx, ctx->stage_a, n * IOW * 4));
      ECC_TRY(ensure(ctx, ctx->stage_b, n * 32));
      HIP_TRY(hipMemcpyAsync(ctx->stage_a.p, bases_in, n * IOW * 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(ctx->stage_b.p, scalars_in, n * 32, hipMemcpyHostToDevice, st));
      d_bases_in = P<uint32_t>(ctx->stage_a);
      d_scalars = P<uint32_t>(ctx->stage_b);
    }
    Plan pl = make_plan<C>(n, c);
    const uint32_t nred = uint32_t(pl.W) * reduce_waves(pl.c);  // level-A waves
    const size_t adds_max = pl.E_max / 2 + 1;
    uint32_t lanes_max = 0;
    ECC_TRY(round_lanes<C>(ctx, &lanes_max));
    ECC_TRY(ensure(ctx, ctx->bases, n * PW * 4));
    ECC_TRY(ensure(ctx, ctx->skip, n));
    ECC_TRY(ensure(ctx, ctx->counts, (size_t(pl.B) + 1) * 4));
    ECC_TRY(ensure(ctx, ctx->offsets, (size_t(pl.B) + 1) * 4));
    ECC_TRY(ensure(ctx, ctx->cursor, size_t(pl.B) * 4));
    ECC_TRY(ensure(ctx, ctx->sorted, pl.E_max * 4));
    ECC_TRY(ensure(ctx, ctx->slots, pl.E_max * PW * 4));
    ECC_TRY(ensure(ctx, ctx->desc, pl.desc_total * 4));
    ECC_TRY(ensure(ctx, ctx->desc_base, sizeof(pl.desc_base)));
    ECC_TRY(ensure(ctx, ctx->mscr, (adds_max + lanes_max + ROUND_WG) * NL * 4));
    ECC_TRY(ensure(ctx, ctx->segS, size_t(nred) * XW * 4));
    ECC_TRY(ensure(ctx, ctx->segT, size_t(nred) * XW * 4));
    ECC_TRY(ensure(ctx, ctx->winsum, size_t(pl.W) * XW * 4));
    ECC_TRY(ensure(ctx, ctx->flags, (1 + MAX_ROUNDS) * 4));
    size_t stw = scan_tmp_words(size_t(pl.B) + 1);
    ECC_TRY(ensure(ctx, ctx->scan_tmp, stw * 4));

    uint32_t* d_flags = P<uint32_t>(ctx->flags);  // [0] error bits, [1..] round counts
    HIP_TRY(hipMemsetAsync(d_flags, 0, (1 + MAX_ROUNDS) * 4, st));
    HIP_TRY(hipMemsetAsync(ctx->counts.p, 0, (size_t(pl.B) + 1) * 4, st));
    HIP_TRY(hipMemsetAsync(ctx->cursor.p, 0, size_t(pl.B) * 4, st));
    HIP_TRY(hipMemcpyAsync(ctx->desc_base.p, pl.desc_base, sizeof(pl.desc_base), hipMemcpyHostToDevice, st));

    ECC_TRY(record(ctx, 0, st));
    k_ingest_points<C><<<ceil_div(n, 256), 256, 0, st>>>(d_bases_in, P<uint32_t>(ctx->bases), P<uint8_t>(ctx->skip),
                                                         n, (flags & ECC_IN_MONTGOMERY) ? 1 : 0,
                                                         (flags & ECC_CHECK_ON_CURVE) ? 1 : 0, d_flags);
    HIP_TRY(hipGetLastError());
    k_window_count<<<ceil_div(n, 256), 256, 0, st>>>(d_scalars, P<uint8_t>(ctx->skip), n, pl.c, pl.W, pl.bits,
                                                     P<uint32_t>(ctx->counts), d_flags);
    HIP_TRY(hipGetLastError());
    ECC_TRY(scan_u32(ctx, P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), size_t(pl.B) + 1,
                     P<uint32_t>(ctx->scan_tmp), stw, st));
    k_window_scatter<<<ceil_div(n, 256), 256, 0, st>>>(d_scalars, P<uint8_t>(ctx->skip), n, pl.c, pl.W, pl.bits,
                                                       P<uint32_t>(ctx->offsets), P<uint32_t>(ctx->cursor),
                                                       P<uint32_t>(ctx->sorted));
    HIP_TRY(hipGetLastError());
    k_plan<C, PLAN_WG><<<ceil_div(pl.B, PLAN_WG), PLAN_WG, 0, st>>>(
        P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), pl.B, P<uint32_t>(ctx->sorted), P<uint32_t>(ctx->bases),
        P<uint32_t>(ctx->slots), P<uint32_t>(ctx->desc), P<size_t>(ctx->desc_base), d_flags + 1);
    HIP_TRY(hipGetLastError());
    ECC_TRY(record(ctx, 1, st));
    HIP_TRY(hipMemcpyAsync(ctx->host_small, d_flags, (1 + MAX_ROUNDS) * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    uint32_t errbits = ctx->host_small[0];
    if (errbits & ERRF_SCALAR_RANGE) return fail(ctx, ECC_ERR_RANGE, "a scalar is >= 2^%d", pl.bits);
    if (errbits & ERRF_RANGE) return fail(ctx, ECC_ERR_RANGE, "a base coordinate is >= p");
    if (errbits & ERRF_NOT_ON_CURVE) return fail(ctx, ECC_ERR_NOT_ON_CURVE, "a base is not on the curve");
    uint32_t round_counts[MAX_ROUNDS];
    memcpy(round_counts, ctx->host_small + 1, sizeof(round_counts));

    int nr = 0;
    uint64_t adds = 0;
    for (int r = 0; r < MAX_ROUNDS; r++) {
      uint32_t na = round_counts[r];
      if (na == 0) break;
      uint32_t T = std::max<uint32_t>(ROUND_WG, std::min<uint32_t>(lanes_max, ceil_div(na, KMIN)));
      T = ceil_div(T, ROUND_WG) * ROUND_WG;
      uint32_t k = ceil_div(na, T);
      ECC_TRY(record(ctx, 2 + 2 * r, st));
      k_bucket_round<C, ROUND_WG><<<T / ROUND_WG, ROUND_WG, 0, st>>>(
          P<uint32_t>(ctx->bases), P<uint32_t>(ctx->sorted), P<uint32_t>(ctx->slots),
          P<uint32_t>(ctx->desc) + pl.desc_base[r], na, 1u << r, r == 0 ? 1 : 0, P<uint32_t>(ctx->mscr), k);
      HIP_TRY(hipGetLastError());
      ECC_TRY(record(ctx, 3 + 2 * r, st));
      nr++;
      adds += na;
    }
    const size_t ev_red = 2 + 2 * MAX_ROUNDS, ev_comb = ev_red + 1;
    k_reduce_a<C, REDUCE_WG><<<ceil_div(nred * 64, REDUCE_WG), REDUCE_WG, 0, st>>>(
        P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), P<uint32_t>(ctx->slots), pl.W, pl.c,
        P<uint32_t>(ctx->segS), P<uint32_t>(ctx->segT));
    HIP_TRY(hipGetLastError());
    k_reduce_b<C><<<pl.W, 64, 0, st>>>(P<uint32_t>(ctx->segS), P<uint32_t>(ctx->segT), pl.c,
                                       P<uint32_t>(ctx->winsum));
    HIP_TRY(hipGetLastError());
    ECC_TRY(record(ctx, ev_red, st));
    k_combine<C><<<1, 64, 0, st>>>(P<uint32_t>(ctx->winsum), pl.W, pl.c, d_out, d_inf);
    HIP_TRY(hipGetLastError());
    ECC_TRY(record(ctx, ev_comb, st));
    if (ctx->profiling) {
      HIP_TRY(hipStreamSynchronize(st));
      ecc_stats& S = ctx->stats;
      S.msm_calls += 1;
      S.points += n;
      S.round_launches += nr;
      S.round_adds += adds;
      S.prepare_ms += elapsed(ctx, 0, 1);
      for (int r = 0; r < nr; r++) S.round_ms += elapsed(ctx, 2 + 2 * r, 3 + 2 * r);
      S.reduce_ms += elapsed(ctx, nr ? 3 + 2 * (nr - 1) : 1, ev_red);
      S.combine_ms += elapsed(ctx, ev_red, ev_comb);
      S.total_ms += elapsed(ctx, 0, ev_comb);
    }
  }
  if (host) {
    HIP_TRY(hipMemcpyAsync(out_xy, d_out, IOW * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(out_inf, d_inf, 1, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

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
  k_fixed_base<C, 256><<<ceil_div(n, 256), 256, 0, st>>>(d_k, n, d_out, (flags & ECC_IN_MONTGOMERY) ? 1 : 0);
  HIP_TRY(hipGetLastError());
  if (host) HIP_TRY(hipMemcpyAsync(out, d_out, n * PW * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

// elementwise test entry points operate on device pointers only
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
  uint32_t lanes_max = 0;
  ECC_TRY(round_lanes<C>(ctx, &lanes_max));
  ECC_TRY(ensure(ctx, ctx->slots, 2 * n * PW * 4));
  ECC_TRY(ensure(ctx, ctx->desc, n * 4));
  ECC_TRY(ensure(ctx, ctx->mscr, (n + lanes_max + ROUND_WG) * NL * 4));
  k_test_pairs_in<C><<<ceil_div(n, 256), 256, 0, st>>>(reinterpret_cast<const uint32_t*>(p),
                                                        reinterpret_cast<const uint32_t*>(q), P<uint32_t>(ctx->slots),
                                                        P<uint32_t>(ctx->desc), n);
  HIP_TRY(hipGetLastError());
  uint32_t na = uint32_t(n);
  uint32_t T = std::max<uint32_t>(ROUND_WG, std::min<uint32_t>(lanes_max, ceil_div(na, KMIN)));
  T = ceil_div(T, ROUND_WG) * ROUND_WG;
  uint32_t k = ceil_div(na, T);
  k_bucket_round<C, ROUND_WG><<<T / ROUND_WG, ROUND_WG, 0, st>>>(nullptr, nullptr, P<uint32_t>(ctx->slots),
                                                                 P<uint32_t>(ctx->desc), na, 1u, 0,
                                                                 P<uint32_t>(ctx->mscr), k);
  HIP_TRY(hipGetLastError());
  k_test_pairs_out<C><<<ceil_div(n, 256), 256, 0, st>>>(P<uint32_t>(ctx->slots), reinterpret_cast<uint32_t*>(out), n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return ECC_OK;
}

template <class C>
ecc_status test_bucket_sort_impl(ecc_ctx* ctx, const uint64_t* scalars, size_t n, int c, uint32_t* counts,
                                 uint32_t* offsets, uint32_t* sorted) {
  if (c < 2 || c > 20) return fail(ctx, ECC_ERR_ARG, "window_c %d outside [2, 20]", c);
  hipStream_t st = ctx->stream;
  Plan pl = make_plan<C>(n, c);
  ECC_TRY(ensure(ctx, ctx->cursor, size_t(pl.B) * 4));
  ECC_TRY(ensure(ctx, ctx->flags, (1 + MAX_ROUNDS) * 4));
  size_t stw = scan_tmp_words(size_t(pl.B) + 1);
  ECC_TRY(ensure(ctx, ctx->scan_tmp, stw * 4));
  uint32_t* d_flags = P<uint32_t>(ctx->flags);
  HIP_TRY(hipMemsetAsync(d_flags, 0, 4, st));
  HIP_TRY(hipMemsetAsync(counts, 0, (size_t(pl.B) + 1) * 4, st));
  HIP_TRY(hipMemsetAsync(ctx->cursor.p, 0, size_t(pl.B) * 4, st));
  if (n) {
    k_window_count<<<ceil_div(n, 256), 256, 0, st>>>(reinterpret_cast<const uint32_t*>(scalars), nullptr, n, pl.c,
                                                     pl.W, pl.bits, counts, d_flags);
    HIP_TRY(hipGetLastError());
  }
  ECC_TRY(scan_u32(ctx, counts, offsets, size_t(pl.B) + 1, P<uint32_t>(ctx->scan_tmp), stw, st));
  if (n) {
    k_window_scatter<<<ceil_div(n, 256), 256, 0, st>>>(reinterpret_cast<const uint32_t*>(scalars), nullptr, n, pl.c,
                                                       pl.W, pl.bits, offsets, P<uint32_t>(ctx->cursor), sorted);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipMemcpyAsync(ctx->host_small, d_flags, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->host_small[0] & ERRF_SCALAR_RANGE) return fail(ctx, ECC_ERR_RANGE, "a scalar is >= 2^%d", pl.bits);
  return ECC_OK;
}

ecc_status enter(ecc_ctx* ctx) {
  if (!ctx) return ECC_ERR_ARG;
  ctx->err.clear();
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
  return ECC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported C ABI

extern "C" {

ecc_status ecc_ctx_create(int hip_device, size_t hbm_budget_bytes, ecc_ctx** out) {
  if (!out) return ECC_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return ECC_ERR_DEVICE;
  if (hip_device < 0 || hip_device >= count) return ECC_ERR_ARG;
  if (hipSetDevice(hip_device) != hipSuccess) return ECC_ERR_DEVICE;
  ecc_ctx* ctx = new ecc_ctx();
  ctx->device = hip_device;
  ctx->budget = hbm_budget_bytes;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->cu_count = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&ctx->host_small), 4096, hipHostMallocDefault) != hipSuccess) {
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return ECC_ERR_DEVICE;
  }
  *out = ctx;
  return ECC_OK;
}

void ecc_ctx_destroy(ecc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  DevBuf* all[] = {&ctx->bases,    &ctx->skip,  &ctx->counts, &ctx->offsets, &ctx->cursor,   &ctx->sorted,
                   &ctx->slots,    &ctx->desc,  &ctx->desc_base, &ctx->mscr, &ctx->segS,     &ctx->segT,
                   &ctx->winsum,   &ctx->flags, &ctx->scan_tmp, &ctx->stage_a, &ctx->stage_b, &ctx->stage_c,
                   &ctx->stage_d};
  for (DevBuf* b : all)
    if (b->p) (void)hipFree(b->p);
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  if (ctx->host_small) (void)hipHostFree(ctx->host_small);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* ecc_last_error(const ecc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t ecc_ctx_scratch_bytes(const ecc_ctx* ctx) { return ctx ? ctx->held : 0; }

ecc_status ecc_ctx_set_profiling(ecc_ctx* ctx, int enable) {
  if (!ctx) return ECC_ERR_ARG;
  ctx->profiling = enable != 0;
  if (ctx->profiling) ctx->stats = ecc_stats{};
  return ECC_OK;
}

ecc_status ecc_ctx_get_stats(const ecc_ctx* ctx, ecc_stats* out) {
  if (!ctx || !out) return ECC_ERR_ARG;
  *out = ctx->stats;
  return ECC_OK;
}

ecc_status ecc_msm(ecc_ctx* ctx, ecc_curve curve, const uint64_t* bases, const uint64_t* scalars, size_t n,
                   uint64_t* out_xy, uint8_t* out_inf, const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (!out_xy || !out_inf) return fail(ctx, ECC_ERR_ARG, "null output pointer");
  if (n && (!bases || !scalars)) return fail(ctx, ECC_ERR_ARG, "null input pointer with n > 0");
  if (n > (size_t(1) << 28)) return fail(ctx, ECC_ERR_ARG, "n = %zu exceeds 2^28", n);
  if (opts && (opts->flags & ~uint32_t(ECC_IN_MONTGOMERY | ECC_CHECK_ON_CURVE | ECC_HOST_PTRS)))
    return fail(ctx, ECC_ERR_ARG, "unknown flag bits 0x%x", opts->flags);
  switch (curve) {
    case ECC_BN254_G1: return msm_impl<BN254>(ctx, bases, scalars, n, out_xy, out_inf, opts);
    case ECC_BLS12_381_G1: return msm_impl<BLS12_381>(ctx, bases, scalars, n, out_xy, out_inf, opts);
    case ECC_SECP256R1: return fail(ctx, ECC_ERR_UNSUPPORTED, "MSM is provided for BN254 and BLS12-381 G1");
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
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_test_fp_mul(ecc_ctx* ctx, ecc_curve curve, const uint64_t* a, const uint64_t* b, uint64_t* out,
                           size_t n) {
  ECC_TRY(enter(ctx));
  if (n && (!a || !b || !out)) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1: return test_fp_mul_impl<BN254>(ctx, a, b, out, n);
    case ECC_BLS12_381_G1: return test_fp_mul_impl<BLS12_381>(ctx, a, b, out, n);
    case ECC_SECP256R1: return test_fp_mul_impl<P256>(ctx, a, b, out, n);
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
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_test_bucket_sort(ecc_ctx* ctx, ecc_curve curve, const uint64_t* scalars, size_t n, int window_c,
                                uint32_t* counts, uint32_t* offsets, uint32_t* sorted) {
  ECC_TRY(enter(ctx));
  if (!counts || !offsets || (n && (!scalars || !sorted))) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1: return test_bucket_sort_impl<BN254>(ctx, scalars, n, window_c, counts, offsets, sorted);
    case ECC_BLS12_381_G1:
      return test_bucket_sort_impl<BLS12_381>(ctx, scalars, n, window_c, counts, offsets, sorted);
    default: return fail(ctx, ECC_ERR_UNSUPPORTED, "bucket sort is provided for the MSM curves");
  }
}

}  // extern "C"
