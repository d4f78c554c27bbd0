// Host side of the MSM calls of the C ABI declared in include/ecc_mi.h:
// argument checks, device scratch management and the launch sequence of the
// MSM path; context creation and the window tuner.
#include "host.h"

namespace {

// lanes of the bucket-round kernel that fit on the device at once: a round's
// additions are spread over at most these lanes so each lane runs one chain
template <class C>
ecc_status round_lanes(ecc_ctx* ctx, int occ, uint32_t* lanes) {
  int& blocks = ctx->round_blocks[C::ID][occ == 2 ? 0 : 1];
  if (blocks == 0) {
    int b = 0;
    if (occ == 2) {
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_bucket_round<C, ROUND_WG, 2>, ROUND_WG, 0));
    } else {
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_bucket_round<C, ROUND_WG, 3>, ROUND_WG, 0));
    }
    blocks = std::max(1, b);
  }
  *lanes = uint32_t(blocks) * uint32_t(ctx->cu_count) * ROUND_WG;
  return ECC_OK;
}

// one bucket-accumulation round at the chosen occupancy target
template <class C>
void launch_round(int occ, uint32_t blocks, hipStream_t st, const uint32_t* bases, const uint32_t* sorted,
                  const uint32_t* in_x, const uint32_t* in_y, uint32_t* out_x, uint32_t* out_y, const uint2* desc,
                  const uint4* prm, int from_bases, uint32_t* mscr, const uint2* tails, const uint32_t* n_tails) {
  if (occ == 2)
    k_bucket_round<C, ROUND_WG, 2><<<blocks, ROUND_WG, 0, st>>>(bases, sorted, in_x, in_y, out_x, out_y, desc, prm,
                                                               from_bases, mscr, tails, n_tails);
  else
    k_bucket_round<C, ROUND_WG, 3><<<blocks, ROUND_WG, 0, st>>>(bases, sorted, in_x, in_y, out_x, out_y, desc, prm,
                                                               from_bases, mscr, tails, n_tails);
}

// x and y planes of a slot buffer with `cap` entries
template <class C>
struct Planes {
  uint32_t* x;
  uint32_t* y;
};
template <class C>
Planes<C> planes(DevBuf& b, size_t cap) {
  uint32_t* p = static_cast<uint32_t*>(b.p);
  return Planes<C>{p, p + cap * C::F::CW};
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

// Window width for an MSM of n points when the caller gives none.  The cost
// model weighs the W (n + alpha D) bucket work of W = ceil((bits + 1) / c)
// windows of D = 2^(c-1) buckets: each point is added once per window, and
// the reduction costs about alpha batch additions per bucket (two chained
// XYZZ additions, each about 2.5 batch additions' worth of products).  A
// tuned table from ecc_tune replaces the rule where one exists.
// bound on the half-scalars of the endomorphism split (0: no split on this curve)
template <class C>
constexpr int glv_bits_of() {
  if constexpr (Glv<C>::HAS) return Glv<C>::BITS;
  else return 0;
}

int model_window(int bits, size_t n, double alpha) {
  int best = 2;
  double best_cost = 1e300;
  // up to 16: the widest window whose buckets the LDS grouping and the
  // reduction waves handle without long per-lane chains (wider only if tuned)
  for (int c = 2; c <= 16; c++) {
    double W = double((bits + 1 + c - 1) / c);
    double cost = W * (double(n) + alpha * double(1u << (c - 1)));
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
  }
  return best;
}

// n_in: points given by the caller (the tuned table's index); bits and n_eff:
// scalar bits and points of the bucket work (2 n_in points of half-length
// scalars after the endomorphism split)
int default_window(ecc_ctx* ctx, int curve, int bits, size_t n_in, size_t n_eff) {
  int lg = bit_length(n_in ? n_in : 1) - 1;
  if (lg < 32 && ctx->tuned[curve][lg] > 0) return ctx->tuned[curve][lg];
  return model_window(bits, n_eff, 5.0);
}

// Launch geometry of a batch of MSMs (a single MSM is a batch of one).
struct Geometry {
  std::vector<MsmDesc> msms;
  std::vector<RedJob> jobs;
  std::vector<RedWave> waves;
  std::vector<uint32_t> big;  // jobs spread over more than one wave
  size_t n = 0;               // points given by the caller
  bool glv = false;           // single MSM over 2 n points after the endomorphism split (fused ingest)
  bool glv_batch = false;     // the split for any batch: point i -> points 2i, 2i + 1 (k_ingest_glv_batch)
  size_t B = 0;               // buckets
  size_t E = 0;               // bound on bucket entries
  uint32_t nseg = 0;          // level-A results of the big jobs
  uint32_t max_n = 0;
  uint32_t kmin = KMIN;       // target additions per lane in a round
  int occ = ROUND_OCC;        // occupancy target of the round kernel
  int rounds = 0;             // bound on the number of rounds
  size_t desc_base[MAX_ROUNDS];  // per round, first descriptor (uint2 units)
  size_t desc_total = 0;
  size_t tail_base[MAX_ROUNDS];  // per round, first tail descriptor
  size_t tail_total = 0;
  size_t slot_cap = 0;           // entries of each slot buffer
  // byte offsets of the tables inside the uploaded block
  std::vector<uint64_t> ptrs;  // per-MSM base pointers (bases read in place), or empty
  size_t off_msms = 0, off_jobs = 0, off_waves = 0, off_big = 0, off_desc_base = 0, off_tail_base = 0, off_ptrs = 0,
         bytes = 0;
};

constexpr int RADIX_SORT_MAX_C = 16;
constexpr uint64_t GLV_MAX_POINTS = uint64_t(1) << 26;  // 2n within the sort's 27-bit entry indices

// sizes[i] points per MSM; c_fixed > 0 forces the window width.  glv_bits > 0
// (a curve with the endomorphism split, halves below 2^glv_bits): the MSMs
// run over 2 n points of half-length scalars.  A single MSM over one array
// takes the fused ingest of k_ingest_glv (points i and n + i) when its
// window fits the two-level sort, and no split otherwise; batches and calls
// with per-MSM base pointers take k_ingest_glv_batch (points 2i and 2i + 1,
// MSM ranges doubled).
ecc_status build_geometry(ecc_ctx* ctx, int curve, int bits, const uint64_t* sizes, size_t m, int c_fixed,
                          Geometry& g, int glv_bits = 0, bool per_msm = false) {
  g = Geometry{};
  g.msms.resize(m);
  uint64_t first = 0;
  if (glv_bits > 0) {
    if (!per_msm && m == 1) {
      // a single MSM over one array: the fused ingest when its window fits
      // the two-level sort; a wider window runs without the split, since its
      // top window over the 128-bit halves would hold only a few bits of every
      // scalar and pile most entries into a handful of buckets
      if (sizes[0] > 0 && sizes[0] <= GLV_MAX_POINTS) {
        const int c = c_fixed ? c_fixed : default_window(ctx, curve, glv_bits, sizes[0], 2 * sizes[0]);
        g.glv = c <= RADIX_SORT_MAX_C;
      }
    } else {
      g.glv_batch = true;
    }
  }
  const bool split = g.glv || g.glv_batch;
  for (size_t i = 0; i < m; i++) {
    const uint64_t n_in = sizes[i];
    const uint64_t n = split ? 2 * n_in : n_in;
    const int sbits = split ? glv_bits : bits;
    MsmDesc& d = g.msms[i];
    d.first = uint32_t(g.glv_batch ? 2 * first : first);
    d.n = uint32_t(n);
    int c = c_fixed ? c_fixed : default_window(ctx, curve, sbits, n_in, n);
    d.c = uint32_t(c);
    d.W = n ? uint32_t((sbits + 1 + c - 1) / c) : 0u;
    d.bucket_base = uint32_t(g.B);
    d.job_base = uint32_t(g.jobs.size());
    const uint32_t D = 1u << (c - 1);
    for (uint32_t w = 0; w < d.W; w++) {
      RedJob j{uint32_t(g.B) + w * D, uint32_t(c - 1), 0u, 0u};
      g.jobs.push_back(j);
    }
    g.B += size_t(d.W) * D;
    g.E += size_t(n) * d.W;
    g.max_n = std::max<uint32_t>(g.max_n, uint32_t(n));
    first += n_in;
    if (g.B > (size_t(1) << 31) || first > (uint64_t(1) << 31))
      return fail(ctx, ECC_ERR_ARG, "batch too large: %zu buckets, %llu points", g.B, (unsigned long long)first);
  }
  g.n = size_t(first);
  // lanes of each reduction job: reduce_lg_lanes, unless that spreads the
  // batch's buckets over more than REDUCE_LANE_TARGET lanes.  The reduction
  // is then bound by its total work, and every lane's segment scan costs
  // about 2 log2(64) + 1 point operations on top of its buckets, so every
  // job's lanes are halved (up to REDUCE_MAX_SHRINK times, and never to more
  // than 64 buckets per lane) until the total fits.
  {
    auto lanes_of = [](const RedJob& j, int shrink) {
      const int def = reduce_lg_lanes(int(j.lgD));
      const int floor_lg = std::min(def, std::max(0, int(j.lgD) - 6));  // at most 64 buckets per lane
      return std::max(def - shrink, floor_lg);
    };
    int shrink = 0;
    for (;; shrink++) {
      uint64_t lanes = 0;
      for (const RedJob& j : g.jobs) lanes += uint64_t(1) << lanes_of(j, shrink);
      if (lanes <= REDUCE_LANE_TARGET || shrink == REDUCE_MAX_SHRINK) break;
    }
    for (RedJob& j : g.jobs) j.lgLam = uint32_t(lanes_of(j, shrink));
  }
  // level-A waves: jobs of more than 64 lanes get whole waves; smaller jobs
  // with the same segment size share waves (consecutive job indices)
  RedWave cur{0, 0, 0, 0};
  bool open = false;
  for (uint32_t j = 0; j < uint32_t(g.jobs.size()); j++) {
    int lgLam = int(g.jobs[j].lgLam);
    if (lgLam > 6) {
      if (open) {
        g.waves.push_back(cur);
        open = false;
      }
      g.jobs[j].seg_base = g.nseg;
      uint32_t G = 1u << (lgLam - 6);
      for (uint32_t k = 0; k < G; k++) g.waves.push_back(RedWave{j, 6u, 1u, k});
      g.nseg += G;
      g.big.push_back(j);
      continue;
    }
    uint32_t lgS = uint32_t(lgLam);
    if (open && cur.lgS == lgS && cur.njobs < (64u >> lgS)) {
      cur.njobs++;
    } else {
      if (open) g.waves.push_back(cur);
      cur = RedWave{j, lgS, 1u, 0u};
      open = true;
    }
  }
  if (open) g.waves.push_back(cur);
  // rounds: a bucket never holds more entries than its MSM has points
  g.rounds = std::min(MAX_ROUNDS, bit_length(g.max_n));
  {
    // tuned tables are indexed by the caller's point count
    uint64_t max_in = 0;
    for (size_t i = 0; i < m; i++) max_in = std::max<uint64_t>(max_in, sizes[i]);
    int lg = bit_length(max_in ? max_in : 1) - 1;
    if (ctx->kmin_override > 0) g.kmin = uint32_t(ctx->kmin_override);
    else if (lg < 32 && ctx->tuned_kmin[curve][lg] > 0) g.kmin = uint32_t(ctx->tuned_kmin[curve][lg]);
    if (ctx->occ_override > 0) g.occ = ctx->occ_override;
    else if (lg < 32 && ctx->tuned_occ[curve][lg] > 0) g.occ = ctx->tuned_occ[curve][lg];
  }
  size_t acc = 0;
  size_t nonempty = std::min(g.B, g.E);
  size_t tacc = 0;
  for (int r = 0; r < MAX_ROUNDS; r++) {
    g.desc_base[r] = acc;
    g.tail_base[r] = tacc;
    if (r < std::max(1, g.rounds)) {
      acc += (g.E >> (r + 1)) + nonempty / 2 + 1;
      tacc += std::min(nonempty, (g.E >> r) + 1) + 1;
    }
  }
  g.desc_total = acc;
  g.tail_total = tacc;
  g.slot_cap = g.E + g.B + 2;
  auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
  size_t o = 0;
  g.off_msms = o;
  o = align(o + sizeof(MsmDesc) * std::max<size_t>(1, m));
  g.off_jobs = o;
  o = align(o + sizeof(RedJob) * std::max<size_t>(1, g.jobs.size()));
  g.off_waves = o;
  o = align(o + sizeof(RedWave) * std::max<size_t>(1, g.waves.size()));
  g.off_big = o;
  o = align(o + sizeof(uint32_t) * std::max<size_t>(1, g.big.size()));
  g.off_desc_base = o;
  o = align(o + sizeof(g.desc_base));
  g.off_tail_base = o;
  o = align(o + sizeof(g.tail_base));
  g.off_ptrs = o;
  o = align(o + sizeof(uint64_t) * m);
  g.bytes = o;
  return ECC_OK;
}

// copy the geometry tables into the context's device block (through pinned
// host memory, on the stream)
ecc_status upload_geometry(ecc_ctx* ctx, const Geometry& g, hipStream_t st) {
  ECC_TRY(ensure(ctx, ctx->geo, g.bytes));
  if (!ctx->geo_copied) HIP_TRY(hipEventCreateWithFlags(&ctx->geo_copied, hipEventDisableTiming));
  // the previous upload must have left the staging area (a wait for that copy
  // only, not for the kernels queued behind it)
  HIP_TRY(hipEventSynchronize(ctx->geo_copied));
  if (ctx->host_geo_cap < g.bytes) {
    if (ctx->host_geo) HIP_TRY(hipHostFree(ctx->host_geo));
    ctx->host_geo = nullptr;
    ctx->host_geo_cap = 0;
    HIP_TRY(hipHostMalloc(&ctx->host_geo, g.bytes, hipHostMallocDefault));
    ctx->host_geo_cap = g.bytes;
  }
  char* h = static_cast<char*>(ctx->host_geo);
  memcpy(h + g.off_msms, g.msms.data(), sizeof(MsmDesc) * g.msms.size());
  memcpy(h + g.off_jobs, g.jobs.data(), sizeof(RedJob) * g.jobs.size());
  memcpy(h + g.off_waves, g.waves.data(), sizeof(RedWave) * g.waves.size());
  memcpy(h + g.off_big, g.big.data(), sizeof(uint32_t) * g.big.size());
  memcpy(h + g.off_desc_base, g.desc_base, sizeof(g.desc_base));
  memcpy(h + g.off_tail_base, g.tail_base, sizeof(g.tail_base));
  if (!g.ptrs.empty()) memcpy(h + g.off_ptrs, g.ptrs.data(), sizeof(uint64_t) * g.ptrs.size());
  HIP_TRY(hipMemcpyAsync(ctx->geo.p, h, g.bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(ctx->geo_copied, st));
  return ECC_OK;
}


// Bucket grouping of a single MSM by the two-level counting sort (window
// widths up to 16, whose signed digits fit 16 bits, and point indices of at
// most 27 bits); otherwise, and for batches, by device-wide atomics.
bool sort_geometry(const Geometry& g, SortGeom& s) {
  if (g.msms.size() != 1 || g.msms[0].n == 0) return false;
  const MsmDesc& d = g.msms[0];
  if (int(d.c) > RADIX_SORT_MAX_C) return false;
  s.n = d.n;
  s.np = (d.n + 7u) & ~7u;
  s.c = d.c;
  s.W = d.W;
  s.vb = uint32_t(std::max(1, bit_length(d.n - 1)));
  if (s.vb > 27) return false;
  const uint32_t cm1 = d.c - 1;
  // fine bits: about SORT_FINE_CAP / 2 entries per coarse bin on average
  uint32_t fb = 0;
  while (fb < cm1 && (uint64_t(d.n) << (fb + 1)) <= (uint64_t(SORT_FINE_CAP / 2) << cm1)) fb++;
  fb = std::min(fb, uint32_t(bit_length(SORT_FINE_MAXB) - 1));
  while ((1u << (cm1 - fb)) > SORT_COARSE_MAX) fb++;
  if (s.vb + 1 + fb > 32) return false;
  s.fb = fb;
  s.ncw = 1u << (cm1 - fb);
  // chunks of at least 16384 points, at most 64 per window (the coarse table
  // has W ncw nch words)
  const uint32_t nch = std::min<uint32_t>(64, (s.np + 16383) / 16384);
  s.chunk = ((s.np + nch - 1) / nch + 7u) & ~7u;
  s.nch = (s.np + s.chunk - 1) / s.chunk;
  return true;
}

size_t sort_hist_words(const SortGeom& s) { return size_t(s.W) * s.ncw * s.nch + 1; }

ecc_status reserve_radix_sort(ecc_ctx* ctx, const SortGeom& s) {
  const size_t hw = sort_hist_words(s);
  ECC_TRY(ensure(ctx, ctx->hist, hw * 4));
  ECC_TRY(ensure(ctx, ctx->hist_scan, hw * 4));
  ECC_TRY(ensure(ctx, ctx->dig, size_t(s.W) * s.np * 2));
  ECC_TRY(ensure(ctx, ctx->part, size_t(s.W) * s.n * 4));
  ECC_TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_words(hw) * 4));
  return ECC_OK;
}

// counts, offsets (B + 1 words) and sorted entries of one MSM; error bits
// into err.  Without d_scalars the digit table is already written (by the
// ingest of the endomorphism split).
ecc_status enqueue_radix_sort(ecc_ctx* ctx, const SortGeom& s, const uint32_t* d_scalars, const uint8_t* d_skip,
                              int bits, uint32_t* counts, uint32_t* offsets, uint32_t* sorted, uint32_t* err,
                              hipStream_t st) {
  const size_t hw = sort_hist_words(s);
  uint16_t* dig = P<uint16_t>(ctx->dig);
  uint32_t* H = P<uint32_t>(ctx->hist);
  uint32_t* Hs = P<uint32_t>(ctx->hist_scan);
  if (d_scalars) {
    k_sort_digits<<<ceil_div(s.np, 256), 256, 0, st>>>(d_scalars, d_skip, s, bits, dig, err);
    HIP_TRY(hipGetLastError());
  }
  k_sort_count<<<s.W * s.nch, SORTC_WG, 0, st>>>(dig, s, H);
  HIP_TRY(hipGetLastError());
  ECC_TRY(scan_u32(ctx, H, Hs, hw, P<uint32_t>(ctx->scan_tmp), scan_tmp_words(hw), st));
  const size_t lds = sort_coarse_lds_bytes(s.ncw);  // at most 3 x 32 KB of bin tables and 48 KB of tile
  if (lds > 65536)
    HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sort_coarse),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
  k_sort_coarse<<<s.W * s.nch, SORTC_WG, lds, st>>>(dig, s, Hs, P<uint32_t>(ctx->part));
  HIP_TRY(hipGetLastError());
  k_sort_fine<<<s.W * s.ncw, SORTF_WG, 0, st>>>(P<uint32_t>(ctx->part), s, Hs, counts, offsets, sorted);
  HIP_TRY(hipGetLastError());
  return ECC_OK;
}

// whether the rounds of a call of m MSMs may hand over to the finishing pass
// (single MSMs by default; batches too with RV_FINISH; never with RV_ROUNDS_ONLY)
bool finish_enabled(const ecc_ctx* ctx, size_t m) {
  return (ctx->round_variant & RV_FINISH) || (m == 1 && !(ctx->round_variant & RV_ROUNDS_ONLY));
}

// Scratch for a geometry (all device buffers of the context).
template <class C>
ecc_status reserve_msm(ecc_ctx* ctx, const Geometry& g, uint32_t lanes_max) {
  constexpr int NL = C::F::NL;
  constexpr int PW = affine_words<C>();
  constexpr int XW = xyzz_words<C>();
  size_t adds_max = g.E / 2 + 1;
  ECC_TRY(ensure(ctx, ctx->bases, (g.glv || g.glv_batch ? 2 : 1) * g.n * PW * 4));
  ECC_TRY(ensure(ctx, ctx->skip, (g.glv_batch ? 2 : 1) * g.n));
  if (g.glv_batch) ECC_TRY(ensure(ctx, ctx->hscal, 2 * g.n * 32));
  ECC_TRY(ensure(ctx, ctx->counts, (g.B + 1) * 4));
  ECC_TRY(ensure(ctx, ctx->offsets, (g.B + 1) * 4));
  ECC_TRY(ensure(ctx, ctx->cursor, g.B * 4));
  ECC_TRY(ensure(ctx, ctx->sorted, g.E * 4));
  ECC_TRY(ensure(ctx, ctx->slots, g.slot_cap * PW * 4));
  ECC_TRY(ensure(ctx, ctx->slots2, g.slot_cap * PW * 4));
  ECC_TRY(ensure(ctx, ctx->desc, g.desc_total * 8));
  ECC_TRY(ensure(ctx, ctx->tails, g.tail_total * 8));
  // prefix products (and, for the stored-denominator variant, the denominators
  // in a second area of the same size)
  const size_t chain_words = (adds_max + lanes_max + ROUND_WG) * NL;
  ECC_TRY(ensure(ctx, ctx->mscr, ((ctx->round_variant & RV_STORE_DENOM) ? 2 : 1) * chain_words * 4));
  ECC_TRY(ensure(ctx, ctx->segS, size_t(g.nseg) * XW * 4));
  ECC_TRY(ensure(ctx, ctx->segT, size_t(g.nseg) * XW * 4));
  ECC_TRY(ensure(ctx, ctx->winsum, g.jobs.size() * XW * 4));
  ECC_TRY(ensure(ctx, ctx->flags, (2 + 2 * MAX_ROUNDS) * 4));
  ECC_TRY(ensure(ctx, ctx->rparams, (MAX_ROUNDS + 1) * sizeof(uint4)));
  ECC_TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_words(g.B + 1) * 4));
  if (finish_enabled(ctx, g.msms.size())) ECC_TRY(ensure(ctx, ctx->fzz, g.B * 2 * C::F::CW * 4));
  SortGeom sg;
  if (sort_geometry(g, sg)) ECC_TRY(reserve_radix_sort(ctx, sg));
  return ECC_OK;
}

// The launch sequence of a batch of MSMs over device inputs and outputs.
// With `exact_rounds` the per-round addition counts are read back once after
// planning, so only rounds with work are launched, each on the lanes it
// needs; otherwise (inside a captured graph) the bound number of rounds is
// launched and each round reads its count on the device.
template <class C>
ecc_status enqueue_msm(ecc_ctx* ctx, const Geometry& g, const uint32_t* d_bases_in, const uint32_t* d_scalars,
                       uint32_t flags, uint32_t* d_out, uint8_t* d_inf, hipStream_t st, bool exact_rounds,
                       int* rounds_run, uint64_t* adds_run, bool* finished = nullptr) {
  uint32_t lanes_max = 0;
  ECC_TRY(round_lanes<C>(ctx, g.occ, &lanes_max));
  const uint32_t m = uint32_t(g.msms.size());
  const MsmDesc* d_msms = GP<MsmDesc>(ctx, g.off_msms);
  // flags: [0] error bits, [1 + r] additions of round r, [1 + MAX_ROUNDS + r] tail copies of round r,
  // [1 + 2 MAX_ROUNDS] the largest bucket
  uint32_t* d_flags = P<uint32_t>(ctx->flags);
  uint32_t* d_maxn = d_flags + 1 + 2 * MAX_ROUNDS;
  const bool prof = exact_rounds && ctx->profiling;
  SortGeom sg;
  const bool radix = sort_geometry(g, sg);
  if (g.glv && !radix) return fail(ctx, ECC_ERR_ARG, "internal: endomorphism split without the two-level sort");
  ECC_TRY(fill_u32(ctx, d_flags, 2 + 2 * MAX_ROUNDS, 0u, st));
  if (!radix) {
    ECC_TRY(fill_u32(ctx, P<uint32_t>(ctx->counts), g.B + 1, 0u, st));
    ECC_TRY(fill_u32(ctx, P<uint32_t>(ctx->cursor), g.B, 0u, st));
  }
  if (prof) ECC_TRY(record(ctx, 0, st));
  if (g.glv) {
    if constexpr (Glv<C>::HAS) {
      const uint32_t n = uint32_t(g.n);
      const uint32_t threads = std::max(n, sg.np - n);
      k_ingest_glv<C><<<ceil_div(threads, 256), 256, 0, st>>>(
          d_bases_in, d_scalars, n, (flags & ECC_IN_MONTGOMERY) ? 1 : 0, (flags & ECC_CHECK_ON_CURVE) ? 1 : 0, sg,
          C::SCALAR_BITS, P<uint32_t>(ctx->bases), P<uint16_t>(ctx->dig), d_flags);
      HIP_TRY(hipGetLastError());
    } else {
      return fail(ctx, ECC_ERR_ARG, "no endomorphism split on this curve");
    }
  } else if (g.glv_batch && g.n) {
    if constexpr (Glv<C>::HAS) {
      k_ingest_glv_batch<C><<<ceil_div(g.n, 256), 256, 0, st>>>(
          d_bases_in, d_scalars, uint32_t(g.n), (flags & ECC_IN_MONTGOMERY) ? 1 : 0,
          (flags & ECC_CHECK_ON_CURVE) ? 1 : 0, C::SCALAR_BITS, P<uint32_t>(ctx->bases), P<uint32_t>(ctx->hscal),
          P<uint8_t>(ctx->skip), d_flags, g.ptrs.empty() ? nullptr : GP<uint64_t>(ctx, g.off_ptrs), d_msms, m);
      HIP_TRY(hipGetLastError());
    } else {
      return fail(ctx, ECC_ERR_ARG, "no endomorphism split on this curve");
    }
  } else if (g.n) {
    k_ingest_points<C><<<ceil_div(g.n, 256), 256, 0, st>>>(
        d_bases_in, P<uint32_t>(ctx->bases), P<uint8_t>(ctx->skip), g.n, (flags & ECC_IN_MONTGOMERY) ? 1 : 0,
        (flags & ECC_CHECK_ON_CURVE) ? 1 : 0, d_flags, g.ptrs.empty() ? nullptr : GP<uint64_t>(ctx, g.off_ptrs),
        d_msms, m);
    HIP_TRY(hipGetLastError());
  }
  // the grouping's scalars: the callers', or the half-scalars of the batch split
  const uint32_t* g_scal = g.glv_batch ? P<uint32_t>(ctx->hscal) : d_scalars;
  const int g_bits = g.glv_batch ? glv_bits_of<C>() : C::SCALAR_BITS;
  const size_t g_np = g.glv_batch ? 2 * g.n : g.n;
  if (radix) {
    ECC_TRY(enqueue_radix_sort(ctx, sg, g.glv ? nullptr : g_scal, P<uint8_t>(ctx->skip), g_bits,
                               P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), P<uint32_t>(ctx->sorted),
                               d_flags, st));
  } else {
    // MSMs whose buckets fit in LDS are grouped one workgroup each; the
    // per-point kernels take the rest
    if (g.n) {
      k_window_group_lds<false><<<m, GROUP_LDS_WG, 0, st>>>(g_scal, P<uint8_t>(ctx->skip), d_msms, g_bits,
                                                             P<uint32_t>(ctx->counts), nullptr, nullptr, d_flags);
      HIP_TRY(hipGetLastError());
      k_window_count<<<ceil_div(g_np, 256), 256, 0, st>>>(g_scal, P<uint8_t>(ctx->skip), g_np, d_msms, m, g_bits,
                                                           GROUP_LDS_BUCKETS, P<uint32_t>(ctx->counts), d_flags);
      HIP_TRY(hipGetLastError());
    }
    ECC_TRY(scan_u32(ctx, P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), g.B + 1,
                     P<uint32_t>(ctx->scan_tmp), scan_tmp_words(g.B + 1), st));
    if (g.n) {
      k_window_group_lds<true><<<m, GROUP_LDS_WG, 0, st>>>(g_scal, P<uint8_t>(ctx->skip), d_msms, g_bits, nullptr,
                                                            P<uint32_t>(ctx->offsets), P<uint32_t>(ctx->sorted),
                                                            d_flags);
      HIP_TRY(hipGetLastError());
      k_window_scatter<<<ceil_div(g_np, 256), 256, 0, st>>>(g_scal, P<uint8_t>(ctx->skip), g_np, d_msms, m, g_bits,
                                                             GROUP_LDS_BUCKETS, P<uint32_t>(ctx->offsets),
                                                             P<uint32_t>(ctx->cursor), P<uint32_t>(ctx->sorted));
      HIP_TRY(hipGetLastError());
    }
  }
  if (g.B) {
    k_plan<PLAN_WG><<<ceil_div(g.B, PLAN_WG), PLAN_WG, 0, st>>>(
        P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), uint32_t(g.B), P<uint2>(ctx->desc),
        GP<size_t>(ctx, g.off_desc_base), P<uint2>(ctx->tails), GP<size_t>(ctx, g.off_tail_base), d_flags + 1,
        d_flags + 1 + MAX_ROUNDS, d_maxn);
    HIP_TRY(hipGetLastError());
  }
  const uint32_t lmax = finish_enabled(ctx, m) ? ctx->fin_lmax : 0u;
  k_round_params<<<1, 64, 0, st>>>(d_flags + 1, lanes_max, ROUND_WG, g.kmin, P<uint4>(ctx->rparams), d_maxn, lmax);
  HIP_TRY(hipGetLastError());
  if (prof) ECC_TRY(record(ctx, 1, st));

  uint32_t counts[MAX_ROUNDS], tails[MAX_ROUNDS];
  // rounds launched (eager: those with work, up to the hand-over to the
  // finishing pass; graph: the bound, each reading its own parameters)
  int nr = g.B ? std::max(1, g.rounds) : 0;
  bool finish = g.B != 0 && !exact_rounds && lmax != 0;
  uint64_t adds = 0;
  if (exact_rounds) {
    HIP_TRY(hipMemcpyAsync(ctx->host_small, d_flags, (2 + 2 * MAX_ROUNDS) * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    memcpy(counts, ctx->host_small + 1, sizeof(counts));
    memcpy(tails, ctx->host_small + 1 + MAX_ROUNDS, sizeof(tails));
    int with_work = 0;
    while (with_work < MAX_ROUNDS && (counts[with_work] || tails[with_work])) with_work++;
    nr = int(finish_round(counts, ctx->host_small[1 + 2 * MAX_ROUNDS], uint32_t(with_work), lmax, 2 * lanes_max));
    finish = nr < with_work;
    for (int r = 0; r < nr; r++) adds += counts[r];  // the batch-affine additions of the rounds run
  }
  const Planes<C> A = planes<C>(ctx->slots, g.slot_cap), Bp = planes<C>(ctx->slots2, g.slot_cap);
  for (int r = 0; r < nr; r++) {
    const Planes<C>& out = (r & 1) ? Bp : A;
    const Planes<C>& in = (r & 1) ? A : Bp;  // the previous round's output (unused in round 0)
    if (prof) ECC_TRY(record(ctx, 2 + 2 * r, st));
    uint32_t blocks = lanes_max / ROUND_WG;
    if (exact_rounds) blocks = round_lane_count(counts[r], lanes_max, ROUND_WG, g.kmin) / ROUND_WG;
    if (ctx->round_variant & RV_KERNEL_MASK) {
      const size_t chain_words = (g.E / 2 + 1 + lanes_max + ROUND_WG) * C::F::NL;
      HIP_TRY(launch_round_variant_bls(ctx->round_variant & RV_KERNEL_MASK, blocks, st, P<uint32_t>(ctx->bases),
                                       P<uint32_t>(ctx->sorted), in.x, in.y, out.x, out.y,
                                       P<uint2>(ctx->desc) + g.desc_base[r], P<uint4>(ctx->rparams) + r,
                                       r == 0 ? 1 : 0, P<uint32_t>(ctx->mscr), P<uint2>(ctx->tails) + g.tail_base[r],
                                       d_flags + 1 + MAX_ROUNDS + r, P<uint32_t>(ctx->mscr) + chain_words));
    } else {
      launch_round<C>(g.occ, blocks, st, P<uint32_t>(ctx->bases), P<uint32_t>(ctx->sorted), in.x, in.y, out.x,
                      out.y, P<uint2>(ctx->desc) + g.desc_base[r], P<uint4>(ctx->rparams) + r, r == 0 ? 1 : 0,
                      P<uint32_t>(ctx->mscr), P<uint2>(ctx->tails) + g.tail_base[r], d_flags + 1 + MAX_ROUNDS + r);
      HIP_TRY(hipGetLastError());
    }
    if (prof) ECC_TRY(record(ctx, 3 + 2 * r, st));
  }
  if (finish) {
    // the rounds left out: each bucket's remaining partial sums on its own lane
    if (prof) ECC_TRY(record(ctx, 2 + 2 * nr, st));
    k_bucket_finish<C, FINISH_WG><<<ceil_div(g.B, FINISH_WG), FINISH_WG, 0, st>>>(
        P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), uint32_t(g.B), A.x, A.y, Bp.x, Bp.y,
        P<uint32_t>(ctx->fzz), P<uint4>(ctx->rparams) + MAX_ROUNDS);
    HIP_TRY(hipGetLastError());
    if (prof) ECC_TRY(record(ctx, 3 + 2 * nr, st));
  }
  if (g.waves.size()) {
    // bucket sums in XYZZ form where the finishing pass ran (or, in a graph,
    // may run: then the reduction reads from the device whether it did)
    const unsigned blocks = unsigned(ceil_div(g.waves.size() * 64, REDUCE_WG));
    if (finish) {
      k_reduce_a<C, REDUCE_WG, true><<<blocks, REDUCE_WG, 0, st>>>(
          P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), A.x, A.y, Bp.x, Bp.y, GP<RedJob>(ctx, g.off_jobs),
          GP<RedWave>(ctx, g.off_waves), uint32_t(g.waves.size()), P<uint32_t>(ctx->segS), P<uint32_t>(ctx->segT),
          P<uint32_t>(ctx->winsum), P<uint32_t>(ctx->fzz), P<uint4>(ctx->rparams) + MAX_ROUNDS);
    } else {
      k_reduce_a<C, REDUCE_WG><<<blocks, REDUCE_WG, 0, st>>>(
          P<uint32_t>(ctx->counts), P<uint32_t>(ctx->offsets), A.x, A.y, Bp.x, Bp.y, GP<RedJob>(ctx, g.off_jobs),
          GP<RedWave>(ctx, g.off_waves), uint32_t(g.waves.size()), P<uint32_t>(ctx->segS), P<uint32_t>(ctx->segT),
          P<uint32_t>(ctx->winsum));
    }
    HIP_TRY(hipGetLastError());
  }
  if (g.big.size()) {
    k_reduce_b<C><<<uint32_t(g.big.size()) * REDB_PARTS, 64 * REDB_WAVES, 0, st>>>(
        P<uint32_t>(ctx->segS), P<uint32_t>(ctx->segT), GP<RedJob>(ctx, g.off_jobs), GP<uint32_t>(ctx, g.off_big));
    HIP_TRY(hipGetLastError());
    k_reduce_c<C><<<uint32_t(g.big.size()), 64 * REDC_WAVES, 0, st>>>(P<uint32_t>(ctx->segT), GP<RedJob>(ctx, g.off_jobs),
                                                          GP<uint32_t>(ctx, g.off_big), P<uint32_t>(ctx->winsum));
    HIP_TRY(hipGetLastError());
  }
  const size_t ev_red = 2 + 2 * MAX_ROUNDS, ev_comb = ev_red + 1;
  if (prof) ECC_TRY(record(ctx, ev_red, st));
  if (m <= COMBINE_WAVE_MAX) {
    k_combine<C><<<m, 64, 0, st>>>(P<uint32_t>(ctx->winsum), d_msms, d_flags, d_out, d_inf);
  } else {
    k_combine_lanes<C><<<ceil_div(m, 64), 64, 0, st>>>(P<uint32_t>(ctx->winsum), d_msms, m, d_flags, d_out, d_inf);
  }
  HIP_TRY(hipGetLastError());
  if (prof) ECC_TRY(record(ctx, ev_comb, st));
  if (rounds_run) *rounds_run = nr;
  if (adds_run) *adds_run = adds;
  if (finished) *finished = finish;
  return ECC_OK;
}

// status of the input-error bits of an MSM call
ecc_status msm_error_status(ecc_ctx* ctx, uint32_t errbits) {
  if (errbits & ERRF_SCALAR_RANGE) return fail(ctx, ECC_ERR_RANGE, "a scalar is >= 2^bitlen(r)");
  if (errbits & ERRF_RANGE) return fail(ctx, ECC_ERR_RANGE, "a base coordinate is >= p");
  if (errbits & ERRF_NOT_ON_CURVE) return fail(ctx, ECC_ERR_NOT_ON_CURVE, "a base is not on the curve");
  if (errbits & ERRF_SPLIT) return fail(ctx, ECC_ERR_DEVICE, "internal: endomorphism split out of range");
  return ECC_OK;
}

// error bits left by the last enqueue_msm (after the stream has drained)
ecc_status msm_errors(ecc_ctx* ctx, hipStream_t st, int bits) {
  HIP_TRY(hipMemcpyAsync(ctx->host_small, ctx->flags.p, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const uint32_t errbits = ctx->host_small[0];
  if (errbits & ERRF_SCALAR_RANGE) return fail(ctx, ECC_ERR_RANGE, "a scalar is >= 2^%d", bits);
  return msm_error_status(ctx, errbits);
}

// end of an asynchronous MSM call: its error bits are OR-ed into the sticky
// word on the stream (read by ecc_ctx_sync), and the stream is remembered
ecc_status note_async(ecc_ctx* ctx, hipStream_t st) {
  if (!ctx->sticky.p) {
    ECC_TRY(ensure(ctx, ctx->sticky, 256));
    ECC_TRY(fill_u32(ctx, P<uint32_t>(ctx->sticky), 1, 0u, st));
  }
  k_or_u32<<<1, 64, 0, st>>>(P<uint32_t>(ctx->flags), P<uint32_t>(ctx->sticky));
  HIP_TRY(hipGetLastError());
  if (std::find(ctx->pending.begin(), ctx->pending.end(), st) == ctx->pending.end()) ctx->pending.push_back(st);
  return ECC_OK;
}

// nr rounds, then (finished) the per-lane finishing pass, whose events follow
// the rounds' at 2 + 2 nr and 3 + 2 nr
void account(ecc_ctx* ctx, size_t n, int nr, uint64_t adds, size_t m, bool finished) {
  ecc_stats& S = ctx->stats;
  const size_t ev_red = 2 + 2 * MAX_ROUNDS, ev_comb = ev_red + 1;
  const int launches = nr + (finished ? 1 : 0);
  S.msm_calls += m;
  S.points += n;
  S.round_launches += nr;
  S.round_adds += adds;
  S.prepare_ms += elapsed(ctx, 0, 1);
  for (int r = 0; r < nr; r++) S.round_ms += elapsed(ctx, 2 + 2 * r, 3 + 2 * r);
  if (finished) S.finish_ms += elapsed(ctx, 2 + 2 * nr, 3 + 2 * nr);
  S.reduce_ms += elapsed(ctx, launches ? 3 + 2 * (launches - 1) : 1, ev_red);
  S.combine_ms += elapsed(ctx, ev_red, ev_comb);
  S.total_ms += elapsed(ctx, 0, ev_comb);
}

// Replay (or capture, on first use) the whole launch sequence of a geometry
// as one hipGraph.  The key holds everything the captured launches depend
// on: the geometry, the flags, the caller's pointers and the context's
// buffer generation (any reallocation invalidates earlier captures).
template <class C>
ecc_status run_graph(ecc_ctx* ctx, const Geometry& g, const uint32_t* d_bases_in, const uint32_t* d_scalars,
                     uint32_t flags, uint32_t* d_out, uint8_t* d_inf, hipStream_t st) {
  std::vector<uint64_t> key;
  key.reserve(16 + g.msms.size());
  key.push_back(uint64_t(C::ID));
  key.push_back(ctx->generation);
  key.push_back(flags);
  key.push_back(uint64_t(ctx->round_variant));
  key.push_back(reinterpret_cast<uint64_t>(d_bases_in));
  key.push_back(reinterpret_cast<uint64_t>(d_scalars));
  key.push_back(reinterpret_cast<uint64_t>(d_out));
  key.push_back(reinterpret_cast<uint64_t>(d_inf));
  key.push_back(reinterpret_cast<uint64_t>(st));
  for (const MsmDesc& d : g.msms) key.push_back((uint64_t(d.n) << 32) | (uint64_t(d.c) << 8) | d.W);
  for (size_t i = 0; i < ctx->graphs.size(); i++) {
    if (ctx->graphs[i].key == key) {
      HIP_TRY(hipGraphLaunch(ctx->graphs[i].exec, st));
      return ECC_OK;
    }
  }
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  ecc_status s = enqueue_msm<C>(ctx, g, d_bases_in, d_scalars, flags, d_out, d_inf, st, false, nullptr, nullptr);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (s != ECC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(ctx, ECC_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ctx, ECC_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  if (ctx->graphs.size() >= GRAPH_CACHE) {
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back(GraphEntry{std::move(key), exec});
  HIP_TRY(hipGraphLaunch(exec, st));
  return ECC_OK;
}

// ecc_msm and ecc_msm_batch: sizes[i] points per MSM (host array)
template <class C>
ecc_status msm_batch_impl(ecc_ctx* ctx, const uint64_t* bases_in, const uint64_t* scalars_in,
                          const uint64_t* sizes, size_t m, uint64_t* out_xy, uint8_t* out_inf,
                          const ecc_opts* opts) {
  constexpr int IOW = 2 * C::F::N32;  // words of a boundary point
  const uint32_t flags = opts ? opts->flags : 0u;
  const bool host = flags & ECC_HOST_PTRS;
  const bool use_graph = (flags & ECC_USE_GRAPH) && !host;
  const bool async = flags & ECC_ASYNC;
  hipStream_t st = pick_stream(ctx, opts);
  int c = opts ? opts->window_c : 0;
  if (c != 0 && (c < 2 || c > 20)) return fail(ctx, ECC_ERR_ARG, "window_c %d outside [2, 20]", c);
  if (async && host) return fail(ctx, ECC_ERR_ARG, "ECC_ASYNC needs device pointers");
  if ((flags & ECC_BASES_PER_MSM) && host) return fail(ctx, ECC_ERR_ARG, "ECC_BASES_PER_MSM needs device pointers");
  if (m == 0) return ECC_OK;
  Geometry g;
  const bool per_msm = flags & ECC_BASES_PER_MSM;
  const int glv_bits = (Glv<C>::HAS && !(flags & ECC_NO_ENDOMORPHISM)) ? glv_bits_of<C>() : 0;
  ECC_TRY(build_geometry(ctx, C::ID, C::SCALAR_BITS, sizes, m, c, g, glv_bits, per_msm));
  if (per_msm) {
    const uint64_t* const* tab = reinterpret_cast<const uint64_t* const*>(bases_in);
    g.ptrs.resize(m);
    for (size_t j = 0; j < m; j++) {
      if (sizes[j] && !tab[j]) return fail(ctx, ECC_ERR_ARG, "null base pointer of MSM %zu", j);
      g.ptrs[j] = reinterpret_cast<uint64_t>(tab[j]);
    }
    bases_in = nullptr;
  }
  uint32_t lanes_max = 0;
  ECC_TRY(round_lanes<C>(ctx, g.occ, &lanes_max));
  // every buffer of the call is sized before anything is enqueued
  ctx->reserving = true;
  ecc_status rs = reserve_msm<C>(ctx, g, lanes_max);
  if (rs == ECC_OK) rs = ensure(ctx, ctx->geo, g.bytes);
  if (rs == ECC_OK && host) {
    rs = ensure(ctx, ctx->stage_a, g.n * IOW * 4);
    if (rs == ECC_OK) rs = ensure(ctx, ctx->stage_b, g.n * 32);
    if (rs == ECC_OK) rs = ensure(ctx, ctx->stage_c, m * (IOW * 4 + 1) + 64);
  }
  ctx->reserving = false;
  ECC_TRY(rs);

  const uint32_t* d_bases_in = reinterpret_cast<const uint32_t*>(bases_in);
  const uint32_t* d_scalars = reinterpret_cast<const uint32_t*>(scalars_in);
  uint32_t* d_out = reinterpret_cast<uint32_t*>(out_xy);
  uint8_t* d_inf = out_inf;
  if (host) {
    if (g.n) {
      HIP_TRY(hipMemcpyAsync(ctx->stage_a.p, bases_in, g.n * IOW * 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(ctx->stage_b.p, scalars_in, g.n * 32, hipMemcpyHostToDevice, st));
    }
    d_bases_in = P<uint32_t>(ctx->stage_a);
    d_scalars = P<uint32_t>(ctx->stage_b);
    d_out = P<uint32_t>(ctx->stage_c);
    d_inf = reinterpret_cast<uint8_t*>(d_out + m * IOW);
  }
  ECC_TRY(upload_geometry(ctx, g, st));

  int nr = 0;
  uint64_t adds = 0;
  bool finished = false;
  if (use_graph) {
    ECC_TRY(run_graph<C>(ctx, g, d_bases_in, d_scalars, flags, d_out, d_inf, st));
  } else {
    // an asynchronous call cannot wait for the round counts: every round of
    // the bound reads its own launch parameters on the device
    ECC_TRY(enqueue_msm<C>(ctx, g, d_bases_in, d_scalars, flags, d_out, d_inf, st, !async, &nr, &adds, &finished));
  }
  if (async) return note_async(ctx, st);
  ECC_TRY(msm_errors(ctx, st, C::SCALAR_BITS));
  if (host) {
    HIP_TRY(hipMemcpyAsync(out_xy, d_out, m * IOW * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(out_inf, d_inf, m, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->profiling && !use_graph) account(ctx, g.n, nr, adds, m, finished);
  return ECC_OK;
}


// Device scratch an ecc_msm_batch call of these sizes would hold: the same
// geometry and the same requests as the call, added up instead of allocated.
template <class C>
ecc_status msm_plan_impl(ecc_ctx* ctx, const uint64_t* sizes, size_t m, const ecc_opts* opts, size_t* bytes) {
  constexpr int IOW = 2 * C::F::N32;
  const uint32_t flags = opts ? opts->flags : 0u;
  int c = opts ? opts->window_c : 0;
  if (c != 0 && (c < 2 || c > 20)) return fail(ctx, ECC_ERR_ARG, "window_c %d outside [2, 20]", c);
  *bytes = 0;
  if (m == 0) return ECC_OK;
  Geometry g;
  const int glv_bits = (Glv<C>::HAS && !(flags & ECC_NO_ENDOMORPHISM)) ? glv_bits_of<C>() : 0;
  ECC_TRY(build_geometry(ctx, C::ID, C::SCALAR_BITS, sizes, m, c, g, glv_bits, (flags & ECC_BASES_PER_MSM) != 0));
  uint32_t lanes_max = 0;
  ECC_TRY(round_lanes<C>(ctx, g.occ, &lanes_max));
  ctx->planning = true;
  ctx->plan_bytes = 0;
  ecc_status s = reserve_msm<C>(ctx, g, lanes_max);
  if (s == ECC_OK) s = ensure(ctx, ctx->geo, g.bytes);
  if (s == ECC_OK && (flags & ECC_HOST_PTRS)) {
    s = ensure(ctx, ctx->stage_a, g.n * IOW * 4);
    if (s == ECC_OK) s = ensure(ctx, ctx->stage_b, g.n * 32);
    if (s == ECC_OK) s = ensure(ctx, ctx->stage_c, m * (IOW * 4 + 1) + 64);
  }
  ctx->planning = false;
  *bytes = ctx->plan_bytes;
  return s;
}

template <class C>
ecc_status test_bucket_sort_impl(ecc_ctx* ctx, const uint64_t* scalars, size_t n, int c, int method,
                                 uint32_t* counts, uint32_t* offsets, uint32_t* sorted) {
  if (c < 2 || c > 20) return fail(ctx, ECC_ERR_ARG, "window_c %d outside [2, 20]", c);
  if (method < 0 || method > 2) return fail(ctx, ECC_ERR_ARG, "method %d outside [0, 2]", method);
  hipStream_t st = ctx->stream;
  Geometry g;
  uint64_t sz = n;
  ECC_TRY(build_geometry(ctx, C::ID, C::SCALAR_BITS, &sz, 1, c, g));
  if (n == 0) {
    // an empty MSM has no windows; the bucket layout of window width c is still reported
    g.msms[0].W = uint32_t((C::SCALAR_BITS + 1 + c - 1) / c);
    g.B = size_t(g.msms[0].W) << (c - 1);
  }
  SortGeom sg;
  const bool lds = method != 1 && sort_geometry(g, sg);
  if (method == 2 && !lds)
    return fail(ctx, ECC_ERR_ARG, "the two-level sort needs one non-empty MSM and window_c <= %d", RADIX_SORT_MAX_C);
  ECC_TRY(ensure(ctx, ctx->cursor, g.B * 4));
  ECC_TRY(ensure(ctx, ctx->flags, (1 + MAX_ROUNDS) * 4));
  ECC_TRY(ensure(ctx, ctx->scan_tmp, scan_tmp_words(g.B + 1) * 4));
  if (lds) ECC_TRY(reserve_radix_sort(ctx, sg));
  ECC_TRY(upload_geometry(ctx, g, st));
  uint32_t* d_flags = P<uint32_t>(ctx->flags);
  const uint32_t* d_s = reinterpret_cast<const uint32_t*>(scalars);
  ECC_TRY(fill_u32(ctx, d_flags, 1, 0u, st));
  if (lds) {
    ECC_TRY(enqueue_radix_sort(ctx, sg, d_s, nullptr, C::SCALAR_BITS, counts, offsets, sorted, d_flags, st));
  } else {
    ECC_TRY(fill_u32(ctx, counts, g.B + 1, 0u, st));
    ECC_TRY(fill_u32(ctx, P<uint32_t>(ctx->cursor), g.B, 0u, st));
    const MsmDesc* d_msms = GP<MsmDesc>(ctx, g.off_msms);
    if (n) {
      k_window_count<<<ceil_div(n, 256), 256, 0, st>>>(d_s, nullptr, n, d_msms, 1u, C::SCALAR_BITS, 0u, counts,
                                                       d_flags);
      HIP_TRY(hipGetLastError());
    }
    ECC_TRY(scan_u32(ctx, counts, offsets, g.B + 1, P<uint32_t>(ctx->scan_tmp), scan_tmp_words(g.B + 1), st));
    if (n) {
      k_window_scatter<<<ceil_div(n, 256), 256, 0, st>>>(d_s, nullptr, n, d_msms, 1u, C::SCALAR_BITS, 0u, offsets,
                                                         P<uint32_t>(ctx->cursor), sorted);
      HIP_TRY(hipGetLastError());
    }
  }
  HIP_TRY(hipMemcpyAsync(ctx->host_small, d_flags, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->host_small[0] & ERRF_SCALAR_RANGE) return fail(ctx, ECC_ERR_RANGE, "a scalar is >= 2^%d", C::SCALAR_BITS);
  return ECC_OK;
}


// ---- window tuner -----------------------------------------------------------


// median wall time of `reps` synchronous MSMs (after one warm-up call)
template <class C>
ecc_status time_msm(ecc_ctx* ctx, const uint64_t* bases, const uint64_t* scalars, size_t n, uint64_t* out,
                    uint8_t* inf, int c, int reps, double* ms) {
  ecc_opts o{0u, c, nullptr};
  const uint64_t sz = n;
  ECC_TRY(msm_batch_impl<C>(ctx, bases, scalars, &sz, 1, out, inf, &o));
  std::vector<double> t;
  for (int r = 0; r < reps; r++) {
    double t0 = now_ms();
    ECC_TRY(msm_batch_impl<C>(ctx, bases, scalars, &sz, 1, out, inf, &o));
    t.push_back(now_ms() - t0);
  }
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return ECC_OK;
}

// For each size 2^lg: seeded bases k_i G and scalars of the curve's bit
// length made on the device, then the fastest window width among the cost
// model's choice and its neighbours, then the fastest additions-per-lane
// target at that width.  Results go to the context's table.
template <class C>
ecc_status tune_impl(ecc_ctx* ctx, int lg_lo, int lg_hi, int reps) {
  constexpr int IOW = 2 * C::F::N32;
  hipStream_t st = ctx->stream;
  for (int lg = lg_lo; lg <= lg_hi; lg++) {
    const size_t n = size_t(1) << lg;
    DevBuf kb, bb, sb, ob;
    auto release = [&]() {
      for (DevBuf* b : {&kb, &bb, &sb, &ob})
        if (b->p) {
          (void)hipFree(b->p);
          ctx->held -= b->cap;
        }
    };
    ecc_status s = ensure(ctx, kb, n * 32);
    if (s == ECC_OK) s = ensure(ctx, bb, n * IOW * 4);
    if (s == ECC_OK) s = ensure(ctx, sb, n * 32);
    if (s == ECC_OK) s = ensure(ctx, ob, IOW * 4 + 64);
    if (s != ECC_OK) {
      release();
      return s;
    }
    const uint64_t seed = 0x7475E5ull * uint64_t(lg + 1) + uint64_t(C::ID);
    k_random_scalars<<<ceil_div(n, 256), 256, 0, st>>>(P<uint32_t>(kb), n, seed, C::SCALAR_BITS - 2);
    k_random_scalars<<<ceil_div(n, 256), 256, 0, st>>>(P<uint32_t>(sb), n, seed ^ 0x5CA1A85ull, C::SCALAR_BITS);
    k_fixed_base<C, 256><<<ceil_div(n, 256), 256, 0, st>>>(P<uint32_t>(kb), n, P<uint32_t>(bb), 0);
    if (hipStreamSynchronize(st) != hipSuccess) {
      release();
      return fail(ctx, ECC_ERR_DEVICE, "tuning input generation failed");
    }
    const uint64_t* bases = static_cast<const uint64_t*>(bb.p);
    const uint64_t* scal = static_cast<const uint64_t*>(sb.p);
    uint64_t* out = static_cast<uint64_t*>(ob.p);
    uint8_t* inf = reinterpret_cast<uint8_t*>(out + IOW / 2);
    const int c0 = glv_bits_of<C>() ? model_window(glv_bits_of<C>(), 2 * n, 5.0) : model_window(C::SCALAR_BITS, n, 5.0);
    int best_c = c0;
    double best = 1e300;
    ctx->kmin_override = KMIN;
    // the model's neighbourhood, and the widest window the two-level sort
    // takes (often the fastest: fewer windows, and the sort stays in LDS)
    std::vector<int> cands;
    for (int c = std::max(2, c0 - 3); c <= std::min(20, c0 + 2); c++) cands.push_back(c);
    if (std::find(cands.begin(), cands.end(), int(RADIX_SORT_MAX_C)) == cands.end())
      cands.push_back(int(RADIX_SORT_MAX_C));
    for (int c : cands) {
      if (s != ECC_OK) break;
      double ms = 0;
      s = time_msm<C>(ctx, bases, scal, n, out, inf, c, reps, &ms);
      if (s == ECC_OK && ms < best) {
        best = ms;
        best_c = c;
      }
    }
    int best_k = KMIN;
    for (int k : {2, 4, 16}) {
      if (s != ECC_OK) break;
      ctx->kmin_override = k;
      double ms = 0;
      s = time_msm<C>(ctx, bases, scal, n, out, inf, best_c, reps, &ms);
      if (s == ECC_OK && ms < best) {
        best = ms;
        best_k = k;
      }
    }
    int best_o = ROUND_OCC;
    ctx->kmin_override = best_k;
    for (int o : {2}) {
      if (s != ECC_OK) break;
      ctx->occ_override = o;
      double ms = 0;
      s = time_msm<C>(ctx, bases, scal, n, out, inf, best_c, reps, &ms);
      if (s == ECC_OK && ms < best) {
        best = ms;
        best_o = o;
      }
    }
    ctx->kmin_override = 0;
    ctx->occ_override = 0;
    release();
    if (s != ECC_OK) return s;
    ctx->tuned[C::ID][lg] = best_c;
    ctx->tuned_kmin[C::ID][lg] = best_k;
    ctx->tuned_occ[C::ID][lg] = best_o;
  }
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
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0) {
    ctx->cu_count = prop.multiProcessorCount;
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    ctx->device_key = arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
  }
  // a blocking stream: ordered with work on the legacy default stream, where
  // callers that name no stream usually put the work that writes the inputs
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamDefault) != hipSuccess ||
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
  for (hipStream_t s : ctx->pending) (void)hipStreamSynchronize(s);
  for (DevBuf* b : scratch_bufs(ctx))
    if (b->p) (void)hipFree(b->p);
  for (DevBuf* b : {&ctx->gtab[3], &ctx->gtab[4], &ctx->gcomb[1], &ctx->gcomb[2], &ctx->gcomb[3], &ctx->gcomb[4]})
    if (b->p) (void)hipFree(b->p);
  if (ctx->sticky.p) (void)hipFree(ctx->sticky.p);
  if (ctx->geo_copied) (void)hipEventDestroy(ctx->geo_copied);
  if (ctx->host_geo) (void)hipHostFree(ctx->host_geo);
  for (GraphEntry& e : ctx->graphs) (void)hipGraphExecDestroy(e.exec);
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

ecc_status ecc_ctx_set_round_variant(ecc_ctx* ctx, int variant) {
  if (!ctx) return ECC_ERR_ARG;
  const int kv = variant & ~(RV_FINISH | RV_ROUNDS_ONLY);
  bool known = kv == 0 && !((variant & RV_FINISH) && (variant & RV_ROUNDS_ONLY));
  for (int v : ROUND_VARIANTS) known = known || (v == kv && !((variant & RV_FINISH) && (variant & RV_ROUNDS_ONLY)));
  if (!known) return fail(ctx, ECC_ERR_ARG, "round variant %d is not built", variant);
  ctx->round_variant = variant;
  return ECC_OK;
}

ecc_status ecc_ctx_get_stats(const ecc_ctx* ctx, ecc_stats* out) {
  if (!ctx || !out) return ECC_ERR_ARG;
  *out = ctx->stats;
  return ECC_OK;
}

ecc_status ecc_ctx_sync(ecc_ctx* ctx) {
  ECC_TRY(enter(ctx));
  for (hipStream_t s : ctx->pending) HIP_TRY(hipStreamSynchronize(s));
  ctx->pending.clear();
  if (!ctx->sticky.p) return ECC_OK;
  HIP_TRY(hipMemcpy(ctx->host_small, ctx->sticky.p, 4, hipMemcpyDeviceToHost));
  const uint32_t errbits = ctx->host_small[0];
  if (errbits == 0) return ECC_OK;
  ECC_TRY(fill_u32(ctx, P<uint32_t>(ctx->sticky), 1, 0u, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return msm_error_status(ctx, errbits);
}

ecc_status ecc_msm(ecc_ctx* ctx, ecc_curve curve, const uint64_t* bases, const uint64_t* scalars, size_t n,
                   uint64_t* out_xy, uint8_t* out_inf, const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (!out_xy || !out_inf) return fail(ctx, ECC_ERR_ARG, "null output pointer");
  if (n && (!bases || !scalars)) return fail(ctx, ECC_ERR_ARG, "null input pointer with n > 0");
  if (n > (size_t(1) << 28)) return fail(ctx, ECC_ERR_ARG, "n = %zu exceeds 2^28", n);
  if (opts && (opts->flags & ~uint32_t(ECC_IN_MONTGOMERY | ECC_CHECK_ON_CURVE | ECC_HOST_PTRS | ECC_USE_GRAPH |
                                        ECC_NO_ENDOMORPHISM | ECC_ASYNC)))
    return fail(ctx, ECC_ERR_ARG, "unknown flag bits 0x%x", opts->flags);
  const uint64_t sz = n;
  switch (curve) {
    case ECC_BN254_G1:
      if (ctx->round_variant & RV_KERNEL_MASK)
        return fail(ctx, ECC_ERR_UNSUPPORTED, "round kernel variants are built for BLS12-381 only");
      return msm_batch_impl<BN254>(ctx, bases, scalars, &sz, 1, out_xy, out_inf, opts);
    case ECC_BLS12_381_G1: return msm_batch_impl<BLS12_381>(ctx, bases, scalars, &sz, 1, out_xy, out_inf, opts);
    case ECC_SECP256R1:
    case ECC_SM2: return fail(ctx, ECC_ERR_UNSUPPORTED, "MSM is provided for BN254 and BLS12-381 G1");
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_msm_batch(ecc_ctx* ctx, ecc_curve curve, const uint64_t* bases, const uint64_t* scalars,
                         const uint64_t* offsets, size_t m, uint64_t* out_xy, uint8_t* out_inf, const ecc_opts* opts) {
  ECC_TRY(enter(ctx));
  if (m == 0) return ECC_OK;
  if (!offsets) return fail(ctx, ECC_ERR_ARG, "null offsets");
  if (!out_xy || !out_inf) return fail(ctx, ECC_ERR_ARG, "null output pointer");
  if (m > (size_t(1) << 24)) return fail(ctx, ECC_ERR_ARG, "m = %zu exceeds 2^24", m);
  if (offsets[0] != 0) return fail(ctx, ECC_ERR_ARG, "offsets[0] = %llu, expected 0", (unsigned long long)offsets[0]);
  std::vector<uint64_t> sizes(m);
  for (size_t i = 0; i < m; i++) {
    if (offsets[i + 1] < offsets[i]) return fail(ctx, ECC_ERR_ARG, "offsets decrease at %zu", i);
    sizes[i] = offsets[i + 1] - offsets[i];
  }
  const uint64_t total = offsets[m];
  if (total && (!bases || !scalars)) return fail(ctx, ECC_ERR_ARG, "null input pointer with points");
  if (total > (uint64_t(1) << 30)) return fail(ctx, ECC_ERR_ARG, "%llu points exceed 2^30", (unsigned long long)total);
  if (opts && (opts->flags & ~uint32_t(ECC_IN_MONTGOMERY | ECC_CHECK_ON_CURVE | ECC_HOST_PTRS | ECC_USE_GRAPH |
                                        ECC_NO_ENDOMORPHISM | ECC_ASYNC | ECC_BASES_PER_MSM)))
    return fail(ctx, ECC_ERR_ARG, "unknown flag bits 0x%x", opts->flags);
  switch (curve) {
    case ECC_BN254_G1:
      if (ctx->round_variant & RV_KERNEL_MASK)
        return fail(ctx, ECC_ERR_UNSUPPORTED, "round kernel variants are built for BLS12-381 only");
      return msm_batch_impl<BN254>(ctx, bases, scalars, sizes.data(), m, out_xy, out_inf, opts);
    case ECC_BLS12_381_G1:
      return msm_batch_impl<BLS12_381>(ctx, bases, scalars, sizes.data(), m, out_xy, out_inf, opts);
    case ECC_SECP256R1:
    case ECC_SM2: return fail(ctx, ECC_ERR_UNSUPPORTED, "MSM is provided for BN254 and BLS12-381 G1");
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}


ecc_status ecc_msm_batch_scratch_bytes(ecc_ctx* ctx, ecc_curve curve, const uint64_t* offsets, size_t m,
                                       const ecc_opts* opts, size_t* bytes) {
  ECC_TRY(enter(ctx));
  if (!bytes) return fail(ctx, ECC_ERR_ARG, "null output pointer");
  *bytes = 0;
  if (m == 0) return ECC_OK;
  if (!offsets) return fail(ctx, ECC_ERR_ARG, "null offsets");
  if (m > (size_t(1) << 24)) return fail(ctx, ECC_ERR_ARG, "m = %zu exceeds 2^24", m);
  std::vector<uint64_t> sizes(m);
  for (size_t i = 0; i < m; i++) {
    if (offsets[i + 1] < offsets[i]) return fail(ctx, ECC_ERR_ARG, "offsets decrease at %zu", i);
    sizes[i] = offsets[i + 1] - offsets[i];
  }
  switch (curve) {
    case ECC_BN254_G1: return msm_plan_impl<BN254>(ctx, sizes.data(), m, opts, bytes);
    case ECC_BLS12_381_G1: return msm_plan_impl<BLS12_381>(ctx, sizes.data(), m, opts, bytes);
    case ECC_SECP256R1:
    case ECC_SM2: return fail(ctx, ECC_ERR_UNSUPPORTED, "MSM is provided for BN254 and BLS12-381 G1");
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_tune(ecc_ctx* ctx, ecc_curve curve, int log2n_min, int log2n_max, int reps) {
  ECC_TRY(enter(ctx));
  if (log2n_min < 1 || log2n_max > 26 || log2n_min > log2n_max)
    return fail(ctx, ECC_ERR_ARG, "log2 sizes [%d, %d] outside [1, 26]", log2n_min, log2n_max);
  if (reps < 1 || reps > 101) return fail(ctx, ECC_ERR_ARG, "reps %d outside [1, 101]", reps);
  switch (curve) {
    case ECC_BN254_G1: return tune_impl<BN254>(ctx, log2n_min, log2n_max, reps);
    case ECC_BLS12_381_G1: return tune_impl<BLS12_381>(ctx, log2n_min, log2n_max, reps);
    case ECC_SECP256R1:
    case ECC_SM2: return fail(ctx, ECC_ERR_UNSUPPORTED, "MSM is provided for BN254 and BLS12-381 G1");
    default: return fail(ctx, ECC_ERR_ARG, "unknown curve %d", int(curve));
  }
}

ecc_status ecc_tuned_params(ecc_ctx* ctx, ecc_curve curve, size_t n, int* window_c, int* adds_per_lane) {
  ECC_TRY(enter(ctx));
  if (!window_c || !adds_per_lane) return fail(ctx, ECC_ERR_ARG, "null output pointer");
  if (curve != ECC_BN254_G1 && curve != ECC_BLS12_381_G1) return fail(ctx, ECC_ERR_ARG, "not an MSM curve");
  const int bits = curve == ECC_BN254_G1 ? BN254::SCALAR_BITS : BLS12_381::SCALAR_BITS;
  const int gb = curve == ECC_BN254_G1 ? glv_bits_of<BN254>() : glv_bits_of<BLS12_381>();
  *window_c = default_window(ctx, curve, gb, n, 2 * n);
  if (n == 0 || n > GLV_MAX_POINTS || *window_c > RADIX_SORT_MAX_C) *window_c = default_window(ctx, curve, bits, n, n);
  int lg = bit_length(n ? n : 1) - 1;
  *adds_per_lane = (lg < 32 && ctx->tuned_kmin[curve][lg] > 0) ? ctx->tuned_kmin[curve][lg] : KMIN;
  return ECC_OK;
}

ecc_status ecc_tune_save(ecc_ctx* ctx, const char* path) {
  ECC_TRY(enter(ctx));
  if (!path) return fail(ctx, ECC_ERR_ARG, "null path");
  FILE* f = fopen(path, "w");
  if (!f) return fail(ctx, ECC_ERR_ARG, "cannot write %s", path);
  fprintf(f, "# eccmi tuning table: device curve log2n window_c adds_per_lane round_occupancy\n");
  for (int cv = 1; cv <= 2; cv++)
    for (int lg = 0; lg < 32; lg++)
      if (ctx->tuned[cv][lg] > 0)
        fprintf(f, "%s %d %d %d %d %d\n", ctx->device_key.c_str(), cv, lg, ctx->tuned[cv][lg],
                ctx->tuned_kmin[cv][lg] > 0 ? ctx->tuned_kmin[cv][lg] : KMIN,
                ctx->tuned_occ[cv][lg] > 0 ? ctx->tuned_occ[cv][lg] : ROUND_OCC);
  bool ok = fclose(f) == 0;
  return ok ? ECC_OK : fail(ctx, ECC_ERR_ARG, "cannot write %s", path);
}

ecc_status ecc_tune_load(ecc_ctx* ctx, const char* path, int* loaded) {
  ECC_TRY(enter(ctx));
  if (!path) return fail(ctx, ECC_ERR_ARG, "null path");
  FILE* f = fopen(path, "r");
  if (!f) return fail(ctx, ECC_ERR_ARG, "cannot read %s", path);
  char line[256], dev[128];
  int count = 0;
  while (fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    int cv, lg, c, k, o;
    if (sscanf(line, "%127s %d %d %d %d %d", dev, &cv, &lg, &c, &k, &o) != 6) continue;
    if (ctx->device_key != dev || cv < 1 || cv > 2 || lg < 0 || lg > 31 || c < 2 || c > 20 || k < 1 || k > 64 ||
        (o != 2 && o != 3))
      continue;
    ctx->tuned[cv][lg] = c;
    ctx->tuned_kmin[cv][lg] = k;
    ctx->tuned_occ[cv][lg] = o;
    count++;
  }
  fclose(f);
  if (loaded) *loaded = count;
  return ECC_OK;
}


ecc_status ecc_test_bucket_sort(ecc_ctx* ctx, ecc_curve curve, const uint64_t* scalars, size_t n, int window_c,
                                int method, uint32_t* counts, uint32_t* offsets, uint32_t* sorted) {
  ECC_TRY(enter(ctx));
  if (!counts || !offsets || (n && (!scalars || !sorted))) return fail(ctx, ECC_ERR_ARG, "null pointer");
  switch (curve) {
    case ECC_BN254_G1:
      return test_bucket_sort_impl<BN254>(ctx, scalars, n, window_c, method, counts, offsets, sorted);
    case ECC_BLS12_381_G1:
      return test_bucket_sort_impl<BLS12_381>(ctx, scalars, n, window_c, method, counts, offsets, sorted);
    default: return fail(ctx, ECC_ERR_UNSUPPORTED, "bucket sort is provided for the MSM curves");
  }
}

}  // extern "C"
