// Host-side state and helpers shared by the library's translation units
// (ecc_mi.hip: MSM path; ecdsa.hip: signing, verification and point
// multiplication).  Internal: not part of the C ABI.  Helpers live in an
// unnamed namespace so that each translation unit keeps its own copy.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ecc_mi.h"
#include "kernels.h"
#include "verify.h"

using namespace eccmi;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  uint64_t used = 0;  // the context call that last asked for this buffer
  size_t need = 0;    // the bytes that call asked for
};

constexpr int ROUND_WG = 256;
constexpr int PLAN_WG = 1024;
constexpr int REDUCE_WG = 256;
constexpr int KMIN = 3;  // target additions per lane in a round
// rounds stop once no bucket holds more than this many partial sums; a
// per-lane pass adds the rest (k_bucket_finish); 0 turns it off
constexpr uint32_t FIN_LMAX = 16;
constexpr int FINISH_WG = 256;
constexpr int ROUND_OCC = 3;  // default waves per SIMD of the round kernel
// up to this many MSMs the window combination takes one wave each (the
// lane-parallel field, several waves per SIMD), else one lane each
constexpr uint32_t COMBINE_WAVE_MAX = 16384;
constexpr uint64_t REDUCE_LANE_TARGET = uint64_t(1) << 17;  // two waves per SIMD
constexpr int REDUCE_MAX_SHRINK = 4;
constexpr size_t GRAPH_CACHE = 16;
constexpr int VERIFY_WG = 256;
constexpr int VERIFY_LANE_WG = 64;                       // per-lane verification: one wave per workgroup
constexpr size_t VERIFY_LANE_CHUNK = size_t(1) << 16;    // requests per launch of the per-lane form
constexpr int SIGN_WG = 256;
constexpr int PMUL_WG = 64;
constexpr int UPMUL_WG = 256;       // batch UPMUL (Algorithm 3): lanes per workgroup
constexpr size_t UPMUL_KPER = 8;    // requests per lane it aims at (amortises the per-bit inversion)

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

// A bucket round of BLS12-381 in design variant `variant` (RV_* bits, nonzero),
// with k_round_apply after it for RV_SPLIT_APPLY (ablate.hip).  Returns the
// launch error, hipErrorInvalidValue for a variant that is not built.
hipError_t launch_round_variant_bls(int variant, uint32_t blocks, hipStream_t st, const uint32_t* bases,
                                    const uint32_t* sorted, const uint32_t* in_x, const uint32_t* in_y,
                                    uint32_t* out_x, uint32_t* out_y, const uint2* desc, const uint4* prm,
                                    int from_bases, uint32_t* mscr, const uint2* tails, const uint32_t* n_tails,
                                    uint32_t* dscr);
// the variants launch_round_variant_bls provides
constexpr int ROUND_VARIANTS[] = {RV_STORE_DENOM, RV_AOS_CHAIN, RV_STORE_DENOM | RV_AOS_CHAIN, RV_SPLIT_APPLY,
                                  RV_STORE_DENOM | RV_AOS_CHAIN | RV_SPLIT_APPLY, RV_LANE_INV, RV_HALF_PREFIX};

struct ecc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t held = 0;
  std::string err;
  DevBuf bases, skip, counts, offsets, cursor, sorted, slots, slots2, desc, tails, mscr, segS, segT, winsum, flags,
      scan_tmp, stage_a, stage_b, stage_c, stage_d;
  uint32_t* host_small = nullptr;  // pinned readback area
  int cu_count = 256;
  int round_blocks[5][2] = {};     // resident round workgroups per CU, by curve id and occupancy target
  bool profiling = false;
  ecc_stats stats{};
  std::vector<hipEvent_t> events;  // pool for per-phase timing
  DevBuf rparams;                  // per-round launch parameters (uint4 each)
  DevBuf hist, hist_scan;          // coarse-bin counts per (window, chunk) of the bucket sort, and their scan
  DevBuf dig, part;                // digit codes and coarse-grouped entries of the bucket sort
  DevBuf hscal;                    // half-scalars of a batch with the endomorphism split
  DevBuf fzz;                      // ZZ, ZZZ of the bucket sums the finishing pass leaves in XYZZ form
  DevBuf geo;                      // launch geometry tables of the current call
  // tables of the signing curves (secp256r1, SM2), by curve id, in the working form:
  DevBuf gtab[5];                  // 2^j G, j < 256 (batched-affine verification)
  bool gtab_ready[5] = {};
  DevBuf gcomb[5];                 // d 2^(8 j) G, j < 32, d < 256 (fixed-base products, per-lane verification, signing)
  bool gcomb_ready[5] = {};
  DevBuf vscr;                     // per-lane verification and point multiplication: each lane's table of d Q
  DevBuf upts;                     // point multiplication: the points in the working form
  int upmul_blocks[5] = {};        // resident batch-UPMUL workgroups per CU, by curve id
  void* host_geo = nullptr;        // pinned staging for them
  size_t host_geo_cap = 0;
  uint64_t generation = 0;         // bumped whenever a device buffer moves
  int tuned[5][32] = {};           // window width by curve and log2 n (0: model)
  int tuned_kmin[5][32] = {};      // additions per lane in a round (0: default)
  int kmin_override = 0;           // set while tuning
  int occ_override = 0;
  int round_variant = 0;           // RV_* design variant of the rounds (ablations; 0 = library form)
  uint32_t fin_lmax = FIN_LMAX;    // partial sums per bucket at which the rounds hand over to k_bucket_finish
  int tuned_occ[5][32] = {};       // occupancy target of the round kernel (0: default)
  std::string device_key;          // architecture and CU count, for the tuning file
  std::vector<GraphEntry> graphs;  // captured launch sequences, most recent last
  hipEvent_t geo_copied = nullptr; // recorded after the geometry upload leaves host_geo
  DevBuf sticky;                   // error bits of asynchronous calls, OR-ed until ecc_ctx_sync
  std::vector<hipStream_t> pending;  // streams with asynchronous calls not yet synchronised
  uint64_t call = 0;               // counts entries into the C ABI
  bool planning = false;           // ensure() only adds up sizes into plan_bytes
  size_t plan_bytes = 0;
  bool reserving = false;          // the call has enqueued nothing yet: its buffers hold no data
};

namespace {

// the context's per-call scratch (every device buffer but the tables of G and
// the sticky error word), which a call may release to fit the HBM budget
std::vector<DevBuf*> scratch_bufs(ecc_ctx* ctx) {
  return {&ctx->bases,   &ctx->skip,    &ctx->counts,  &ctx->offsets, &ctx->cursor,    &ctx->sorted,
          &ctx->slots,   &ctx->slots2,  &ctx->desc,    &ctx->tails,   &ctx->mscr,      &ctx->segS,
          &ctx->segT,    &ctx->winsum,  &ctx->flags,   &ctx->scan_tmp, &ctx->stage_a,  &ctx->stage_b,
          &ctx->stage_c, &ctx->stage_d, &ctx->vscr,    &ctx->upts,    &ctx->rparams,   &ctx->hist,
          &ctx->hist_scan, &ctx->dig,   &ctx->part,    &ctx->geo,     &ctx->hscal,     &ctx->fzz};
}

}  // namespace

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

// Make buffer b hold at least `bytes`.  Under an HBM budget, buffers that
// the current call has not asked for are released first when the budget
// would otherwise be exceeded.  In planning mode only the size is added up.
ecc_status ensure(ecc_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->planning) {
    ctx->plan_bytes += (bytes + 4095) & ~size_t(4095);
    return ECC_OK;
  }
  b.used = ctx->call;
  b.need = bytes;
  if (b.cap >= bytes) return ECC_OK;
  size_t want = std::max(bytes, b.cap + b.cap / 4);
  want = (want + 4095) & ~size_t(4095);
  if (ctx->budget && ctx->held - b.cap + want > ctx->budget) {
    want = (bytes + 4095) & ~size_t(4095);
    if (ctx->held - b.cap + want > ctx->budget) {
      // release what this call does not use, then (while the call has
      // enqueued nothing) trim what it uses to the sizes it asked for
      for (hipStream_t s : ctx->pending) HIP_TRY(hipStreamSynchronize(s));
      for (DevBuf* o : scratch_bufs(ctx)) {
        if (o == &b || !o->p) continue;
        const size_t exact = (o->need + 4095) & ~size_t(4095);
        const bool unused = o->used != ctx->call;
        if (!unused && !(ctx->reserving && o->cap > exact)) continue;
        HIP_TRY(hipFree(o->p));
        ctx->held -= o->cap;
        o->p = nullptr;
        o->cap = 0;
        ctx->generation++;
        if (!unused) {
          hipError_t e = hipMalloc(&o->p, exact);
          if (e != hipSuccess) {
            o->p = nullptr;
            (void)hipGetLastError();
            return fail(ctx, ECC_ERR_NOMEM, "hipMalloc(%zu): %s", exact, hipGetErrorString(e));
          }
          o->cap = exact;
          ctx->held += exact;
        }
      }
    }
    if (ctx->held - b.cap + want > ctx->budget)
      return fail(ctx, ECC_ERR_NOMEM, "HBM budget of %zu bytes exceeded (need %zu more)", ctx->budget,
                  want - b.cap);
  }
  if (b.p) {
    // asynchronous calls may still read the old buffer
    for (hipStream_t s : ctx->pending) HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(b.p));
    ctx->held -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  ctx->generation++;
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

template <class T>
const T* GP(ecc_ctx* ctx, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(ctx->geo.p) + off);
}

ecc_status fill_u32(ecc_ctx* ctx, uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return ECC_OK;
  k_fill_u32<<<ceil_div(n, 256), 256, 0, st>>>(p, n, v);
  HIP_TRY(hipGetLastError());
  return ECC_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

ecc_status enter(ecc_ctx* ctx) {
  if (!ctx) return ECC_ERR_ARG;
  ctx->err.clear();
  ctx->call++;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
  return ECC_OK;
}

}  // namespace
