// Device kernels of the MSM / verification path.
//
// Data layout in HBM (one device, AoS for points so that one gathered point is
// one or two cache lines; SoA where a lane walks its own sequence):
//   bases    : n points, 2 CW words each (x limbs then y limbs, Montgomery
//              form, canonical); the point at infinity is the all-ones x
//              sentinel
//   scalars  : n x 8 words (256-bit little-endian), as given by the caller
//   counts   : one u32 per bucket (window w, |digit| d) = w * D + d - 1
//   offsets  : exclusive prefix sums of counts (B + 1 entries)
//   sorted   : E entries, point index | sign << 31, grouped by bucket
//   slots A/B: two buffers of E + B + 2 entries, each an x plane and a y
//              plane of CW words per entry; round r writes A (r even) or B
//              (r odd); bucket b's entries start at bucket_slot(offsets[b], b)
//   desc     : per round, (first input entry, output entry) of every pair
//   tails    : per round, (input entry, output entry) of every odd last entry
//   mscr     : prefix products of the batch inversion, SoA by global lane
#pragma once
#include "lanefield.h"
#include "point.h"

namespace eccmi {

constexpr uint32_t SIGN_BIT = 0x80000000u;
constexpr int MAX_ROUNDS = 32;

enum : uint32_t { ERRF_RANGE = 1u, ERRF_NOT_ON_CURVE = 2u, ERRF_SCALAR_RANGE = 4u, ERRF_SPLIT = 8u };

// ---------------------------------------------------------------------------
// wave / workgroup helpers

template <class F>
__device__ __forceinline__ Fp<F> shfl_up_fp(const Fp<F>& a, int d) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = __shfl_up(a.w[i], d, 64);
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> shfl_down_fp(const Fp<F>& a, int d) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = __shfl_down(a.w[i], d, 64);
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> select_fp(bool c, const Fp<F>& a, const Fp<F>& b) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = c ? a.w[i] : b.w[i];
  return r;
}

// Gather-Apply-Scatter batch inversion over one workgroup (Section 3.2): every
// lane holds the product K of its own chain; the lanes' K are combined by
// prefix/suffix products inside each wave, the wave totals through LDS, one
// wave-uniform inversion is done for the whole workgroup, and the inverse is
// scattered back so that each lane receives K^-1.  All K must be nonzero.
template <class F, int WG, int V = 0>
__device__ Fp<F> wg_batch_inverse(const Fp<F>& K, Fp<F>* s_tot, Fp<F>* s_inv) {
  constexpr int NW = WG / 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Fp<F> one = fp_one<F>();
  // six steps, each advancing both scans by one product: the inclusive prefix
  // products P_l = K_0 ... K_l and the exclusive suffix products
  // X_l = K_{l+1} ... K_63 (X starts as K shifted down by one lane); the two
  // products of a step are independent, so their latencies overlap
  Fp<F> P = K;
  Fp<F> X = select_fp<F>(lane < 63, shfl_down_fp<F>(K, 1), one);
#pragma unroll 1
  for (int step = 0; step < 6; step++) {
    const int sh = 1 << step;
    const Fp<F> op = shfl_up_fp<F>(P, sh);
    const Fp<F> ox = shfl_down_fp<F>(X, sh);
    P = fp_mul<F>(P, select_fp<F>(lane >= sh, op, one));
    X = fp_mul<F>(X, select_fp<F>(lane + sh < 64, ox, one));
  }
  if (lane == 63) s_tot[wave] = P;
  __syncthreads();
  if (wave == 0) {
    // the same two scans over the NW wave totals, in lanes 0..NW-1
    Fp<F> Wv = lane < NW ? s_tot[lane < NW ? lane : 0] : one;
    Fp<F> Q = Wv;
    Fp<F> SQ = select_fp<F>(lane < NW - 1, shfl_down_fp<F>(Wv, 1), one);
    constexpr int LOGW = NW <= 1 ? 0 : NW <= 2 ? 1 : NW <= 4 ? 2 : NW <= 8 ? 3 : 4;
    for (int step = 0; step < 2 * LOGW; step++) {
      bool up = step < LOGW;
      int s = 1 << (up ? step : step - LOGW);
      Fp<F> cur = up ? Q : SQ;
      Fp<F> o = up ? shfl_up_fp<F>(cur, s) : shfl_down_fp<F>(cur, s);
      bool use = up ? (lane >= s) : (lane + s < NW);
      Fp<F> r = fp_mul<F>(cur, select_fp<F>(use, o, one));
      if (up) Q = r;
      else SQ = r;
    }
    Fp<F> G;
#pragma unroll
    for (int i = 0; i < F::NL; i++) G.w[i] = __builtin_amdgcn_readlane(Q.w[i], NW - 1);
    Fp<F> iG = fp_inv_uniform<F, V>(G);
    Fp<F> Qprev = select_fp<F>(lane >= 1, shfl_up_fp<F>(Q, 1), one);
    // 1/W_j = (1/G) (W_{j+1} ... W_{NW-1}) (W_0 ... W_{j-1})
    Fp<F> iW = iG;
    for (int t = 0; t < 2; t++) iW = fp_mul<F>(iW, t == 0 ? SQ : Qprev);
    if (lane < NW) s_inv[lane] = iW;
  }
  __syncthreads();
  // 1/K_l = (1/W) X_l P_{l-1}
  Fp<F> Pprev = select_fp<F>(lane >= 1, shfl_up_fp<F>(P, 1), one);
  Fp<F> r = s_inv[wave];
  for (int t = 0; t < 2; t++) r = fp_mul<F>(r, t == 0 ? X : Pprev);
  __syncthreads();
  return r;
}

// block-wide exclusive scan of one u32 per thread
template <int WG>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp, uint32_t& total) {
  constexpr int NW = WG / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    uint32_t o = __shfl_up(x, s, 64);
    if (lane >= s) x += o;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) {
    uint32_t t = s_tmp[i];
    before += (i < wave) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return before + x - v;
}

// ---------------------------------------------------------------------------
// ingest: boundary points (u64 limbs, canonical or in the boundary's
// Montgomery form) -> canonical working-form points (limbs, Montgomery R)

// One MSM of a batch: its points [first, first + n) of the concatenated
// input, its window width c, its W windows of 2^(c-1) buckets starting at
// bucket_base, and its W reduction jobs (one per window) starting at job_base.
struct MsmDesc {
  uint32_t first, n, c, W, bucket_base, job_base;
};

// index of the MSM holding point i (the MSMs tile [0, total) in order)
__device__ __forceinline__ uint32_t find_msm(const MsmDesc* __restrict__ msms, uint32_t m, uint32_t i) {
  uint32_t lo = 0, hi = m;  // invariant: msms[lo].first <= i < msms[hi].first (hi = m: end)
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (msms[mid].first <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Point i of the input is in[i] or, with a table of per-MSM base pointers
// (bases read in place, e.g. ranges of a resident set), ptrs[j][i - first_j]
// for the MSM j that holds it.
template <class C>
__global__ void k_ingest_points(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                uint8_t* __restrict__ skip, size_t n, int in_mont, int check_curve,
                                uint32_t* __restrict__ err, const uint64_t* __restrict__ ptrs = nullptr,
                                const MsmDesc* __restrict__ msms = nullptr, uint32_t m = 0) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t* src = in + i * 2 * N32;
  if (ptrs) {
    const uint32_t j = find_msm(msms, m, uint32_t(i));
    src = reinterpret_cast<const uint32_t*>(ptrs[j]) + size_t(uint32_t(i) - msms[j].first) * 2 * N32;
  }
  uint32_t xw[N32], yw[N32];
  words_load<F>(src, xw);
  words_load<F>(src + N32, yw);
  uint32_t any = 0;
#pragma unroll
  for (int k = 0; k < N32; k++) any |= xw[k] | yw[k];
  bool inf = any == 0;
  uint32_t e = 0;
  Affine<C> P;
  if (!inf) {
    if (!words_lt_p<F>(xw) || !words_lt_p<F>(yw)) e |= ERRF_RANGE;
    P.x = fp_from_words<F>(xw);
    P.y = fp_from_words<F>(yw);
    constexpr Words<F::NL> rin = F::RIN, r2 = F::R2;
    const Fp<F> k = fp_from<F>(in_mont ? rin : r2);
    P.x = fp_canonical<F>(fp_mul<F>(P.x, k));
    P.y = fp_canonical<F>(fp_mul<F>(P.y, k));
    if (check_curve && !e && !affine_on_curve<C>(P)) e |= ERRF_NOT_ON_CURVE;
  } else {
    P.x = fp_inf_marker<F>();
    P.y = fp_zero<F>();
  }
  if (e) atomicOr(err, e);
  affine_store<C>(out + i * affine_words<C>(), P);
  // a rejected point is left out of the buckets; the call then reports the error
  if (skip) skip[i] = (inf || e) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// scalar windows with signed digits: digit_w = bits[c w, c w + c) + carry,
// mapped to [-2^(c-1), 2^(c-1)] with a carry into the next window.

// word k of a scalar (0 past the top) by selects, so that a position known
// only at run time does not send the scalar to scratch memory
__device__ __forceinline__ uint32_t scalar_word(const uint32_t s[8], int k) {
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) v = k == i ? s[i] : v;
  return v;
}

__device__ __forceinline__ uint32_t window_bits(const uint32_t s[8], int pos, int c) {
  int word = pos >> 5, sh = pos & 31;
  uint32_t v = scalar_word(s, word) >> sh;
  if (sh + c > 32) v |= scalar_word(s, word + 1) << (32 - sh);
  return v & ((1u << c) - 1u);
}

__device__ __forceinline__ void load_scalar(const uint32_t* __restrict__ p, uint32_t s[8]) {
  const uint4* v = reinterpret_cast<const uint4*>(p);
  uint4 a = v[0], b = v[1];
  s[0] = a.x; s[1] = a.y; s[2] = a.z; s[3] = a.w;
  s[4] = b.x; s[5] = b.y; s[6] = b.z; s[7] = b.w;
}

__device__ __forceinline__ bool scalar_fits(const uint32_t s[8], int bits) {
  for (int w = 0; w < 8; w++) {
    int lo = 32 * w;
    if (lo >= bits) {
      if (s[w]) return false;
    } else if (bits - lo < 32) {
      if (s[w] >> (bits - lo)) return false;
    }
  }
  return true;
}

// buckets of an MSM whose grouping one workgroup does in LDS (batches), and
// the most points such an MSM may have (a larger one, e.g. with a forced
// narrow window, would serialise on one CU: the per-point kernels take it)
constexpr uint32_t GROUP_LDS_BUCKETS = 16384;
constexpr uint32_t GROUP_LDS_MAX_POINTS = 1u << 16;
constexpr int GROUP_LDS_WG = 1024;

// true if the per-point kernels leave this MSM to the LDS kernels (lds_cap:
// GROUP_LDS_BUCKETS when those run, 0 otherwise)
__device__ __forceinline__ bool grouped_in_lds(const MsmDesc& md, uint32_t lds_cap) {
  return (md.W << (md.c - 1)) <= lds_cap && md.n <= GROUP_LDS_MAX_POINTS;
}

// count the entries of every bucket
static __global__ void k_window_count(const uint32_t* __restrict__ scalars, const uint8_t* __restrict__ skip, size_t n,
                               const MsmDesc* __restrict__ msms, uint32_t m, int bits, uint32_t lds_cap,
                               uint32_t* __restrict__ counts, uint32_t* __restrict__ err) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t s[8];
  load_scalar(scalars + 8 * i, s);
  if (!scalar_fits(s, bits)) {
    atomicOr(err, ERRF_SCALAR_RANGE);
    return;
  }
  if (skip && skip[i]) return;
  const MsmDesc md = msms[find_msm(msms, m, uint32_t(i))];
  if (grouped_in_lds(md, lds_cap)) return;
  const int c = int(md.c);
  const uint32_t D = 1u << (c - 1);
  uint32_t carry = 0;
  for (int w = 0; w < int(md.W); w++) {
    int32_t d = int32_t(window_bits(s, c * w, c) + carry);
    carry = 0;
    if (d > int32_t(D)) {
      d -= int32_t(1u << c);
      carry = 1;
    }
    if (d != 0) {
      uint32_t mag = d < 0 ? uint32_t(-d) : uint32_t(d);
      atomicAdd(&counts[md.bucket_base + w * D + mag - 1], 1u);
    }
  }
}

// place every entry into its bucket's range
static __global__ void k_window_scatter(const uint32_t* __restrict__ scalars, const uint8_t* __restrict__ skip, size_t n,
                                 const MsmDesc* __restrict__ msms, uint32_t m, int bits, uint32_t lds_cap,
                                 const uint32_t* __restrict__ offsets, uint32_t* __restrict__ cursor,
                                 uint32_t* __restrict__ sorted) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t s[8];
  load_scalar(scalars + 8 * i, s);
  if (!scalar_fits(s, bits)) return;
  if (skip && skip[i]) return;
  const MsmDesc md = msms[find_msm(msms, m, uint32_t(i))];
  if (grouped_in_lds(md, lds_cap)) return;
  const int c = int(md.c);
  const uint32_t D = 1u << (c - 1);
  uint32_t carry = 0;
  for (int w = 0; w < int(md.W); w++) {
    int32_t d = int32_t(window_bits(s, c * w, c) + carry);
    carry = 0;
    if (d > int32_t(D)) {
      d -= int32_t(1u << c);
      carry = 1;
    }
    if (d != 0) {
      uint32_t mag = d < 0 ? uint32_t(-d) : uint32_t(d);
      uint32_t b = md.bucket_base + w * D + mag - 1;
      uint32_t pos = atomicAdd(&cursor[b], 1u);
      sorted[offsets[b] + pos] = uint32_t(i) | (d < 0 ? SIGN_BIT : 0u);
    }
  }
}

// The same grouping for the MSMs of a batch whose W 2^(c-1) buckets fit in
// LDS: one workgroup per MSM (blockIdx.x) walks its points with the
// counters (count pass) or the bucket cursors (scatter pass) in LDS, so that
// no entry takes a device-wide atomic.  MSMs with more buckets return at
// once and are left to the per-point kernels.
template <bool SCATTER>
__global__ void __launch_bounds__(GROUP_LDS_WG) k_window_group_lds(const uint32_t* __restrict__ scalars,
                                                                   const uint8_t* __restrict__ skip,
                                                                   const MsmDesc* __restrict__ msms, int bits,
                                                                   uint32_t* __restrict__ counts,
                                                                   const uint32_t* __restrict__ offsets,
                                                                   uint32_t* __restrict__ sorted,
                                                                   uint32_t* __restrict__ err) {
  __shared__ uint32_t s_b[GROUP_LDS_BUCKETS];
  const MsmDesc md = msms[blockIdx.x];
  if (md.W == 0 || !grouped_in_lds(md, GROUP_LDS_BUCKETS)) return;  // uniform per workgroup
  const int c = int(md.c);
  const uint32_t D = 1u << (c - 1);
  const uint32_t B = md.W << (c - 1);
  for (uint32_t b = threadIdx.x; b < B; b += GROUP_LDS_WG)
    s_b[b] = SCATTER ? offsets[md.bucket_base + b] : 0u;
  __syncthreads();
  for (uint32_t i = md.first + threadIdx.x; i < md.first + md.n; i += GROUP_LDS_WG) {
    uint32_t s[8];
    load_scalar(scalars + 8 * size_t(i), s);
    if (!scalar_fits(s, bits)) {
      if (!SCATTER) atomicOr(err, ERRF_SCALAR_RANGE);
      continue;
    }
    if (skip && skip[i]) continue;
    uint32_t carry = 0;
    for (int w = 0; w < int(md.W); w++) {
      int32_t d = int32_t(window_bits(s, c * w, c) + carry);
      carry = 0;
      if (d > int32_t(D)) {
        d -= int32_t(1u << c);
        carry = 1;
      }
      if (d != 0) {
        const uint32_t mag = d < 0 ? uint32_t(-d) : uint32_t(d);
        const uint32_t pos = atomicAdd(&s_b[w * D + mag - 1], 1u);
        if (SCATTER) sorted[pos] = i | (d < 0 ? SIGN_BIT : 0u);
      }
    }
  }
  if (!SCATTER) {
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < B; b += GROUP_LDS_WG) counts[md.bucket_base + b] = s_b[b];
  }
}

// ---- bucket grouping of one MSM: signed digits, then a two-level counting
// sort.  k_sort_digits writes the signed digit of every (window, point) as a
// 16-bit code d + D - 1 (so that digit 0 is D - 1).  The bucket index
// |d| - 1 of a non-zero digit splits into a coarse bin (its high bits) and a
// fine bucket (its low fb bits).  Per (window, chunk of points) k_sort_count
// counts the coarse bins in LDS; one exclusive scan over
// H[window][coarse][chunk] gives every (window, coarse, chunk) its first
// position, so that k_sort_coarse writes the entries of a chunk and coarse
// bin as one contiguous run.  Per (window, coarse bin) k_sort_fine counts the
// fine buckets, writes the bucket counts and offsets and orders the bin's
// entries by fine bucket in LDS before writing them out contiguously (a bin
// too large for LDS takes a second pass over global memory instead).

struct SortGeom {
  uint32_t n, np;  // points, row stride of the digit table (n rounded up to 8)
  uint32_t c, W;   // window width and number of windows
  uint32_t fb;     // fine bits: a coarse bin holds 2^fb buckets
  uint32_t ncw;    // coarse bins per window, 2^(c - 1 - fb)
  uint32_t chunk;  // points per chunk of the coarse passes (a multiple of 8)
  uint32_t nch;    // chunks per window
  uint32_t vb;     // bits of the point index in a packed entry (vb + 1 + fb <= 32)
};

constexpr int SORTC_WG = 256;               // coarse passes
constexpr int SORTF_WG = 256;               // fine pass
constexpr uint32_t SORT_COARSE_MAX = 8192;  // coarse bins of a window (LDS counters)
constexpr uint32_t SORT_FINE_MAXB = 2048;   // buckets of a coarse bin (LDS counters)
constexpr uint32_t SORT_FINE_CAP = 8192;    // entries of a coarse bin ordered in LDS

static __global__ void __launch_bounds__(256) k_sort_digits(const uint32_t* __restrict__ scalars,
                                                     const uint8_t* __restrict__ skip, SortGeom g, int bits,
                                                     uint16_t* __restrict__ dig, uint32_t* __restrict__ err) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= g.np) return;
  const int c = int(g.c);
  const uint32_t D = 1u << (c - 1);
  bool live = i < g.n;
  uint32_t s[8];
  if (live) {
    load_scalar(scalars + 8 * size_t(i), s);
    if (!scalar_fits(s, bits)) {
      atomicOr(err, ERRF_SCALAR_RANGE);
      live = false;
    } else if (skip && skip[i]) {
      live = false;
    }
  }
  uint32_t carry = 0;
  for (uint32_t w = 0; w < g.W; w++) {
    uint32_t code = D - 1;
    if (live) {
      int32_t d = int32_t(window_bits(s, c * int(w), c) + carry);
      carry = 0;
      if (d > int32_t(D)) {
        d -= int32_t(1u << c);
        carry = 1;
      }
      code = uint32_t(d + int32_t(D) - 1);
    }
    dig[size_t(w) * g.np + i] = uint16_t(code);
  }
}

// bucket index |d| - 1 and sign of a non-zero digit code
__device__ __forceinline__ uint32_t code_bucket(uint32_t code, uint32_t D) {
  return code >= D ? code - D : D - 2 - code;
}

// the eight codes of one 16-byte load, with the point index of the first
struct Codes8 {
  uint32_t w[4];
  __device__ __forceinline__ uint32_t at(int k) const { return (w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu; }
};

template <bool SCATTER>
__device__ __forceinline__ void sort_coarse_chunk(const uint16_t* __restrict__ dig, const SortGeom& g,
                                                  uint32_t* s_cnt, uint32_t* __restrict__ part) {
  const uint32_t w = blockIdx.x / g.nch, ch = blockIdx.x % g.nch;
  const uint32_t D = 1u << (g.c - 1);
  const uint32_t lo = ch * (g.chunk / 8), hi = min(g.np, (ch + 1) * g.chunk) / 8;
  const uint4* src = reinterpret_cast<const uint4*>(dig + size_t(w) * g.np);
  const uint32_t fmask = (1u << g.fb) - 1u;
  constexpr int U = 4;  // 16-byte loads in flight per thread
  for (uint32_t v0 = lo + threadIdx.x; v0 < hi; v0 += U * SORTC_WG) {
    Codes8 q[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t v = v0 + u * SORTC_WG;
      const uint32_t z = (D - 1) * 0x10001u;  // eight zero digits
      const uint4 t = v < hi ? src[v] : make_uint4(z, z, z, z);
      q[u].w[0] = t.x;
      q[u].w[1] = t.y;
      q[u].w[2] = t.z;
      q[u].w[3] = t.w;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const uint32_t code = q[u].at(k);
        if (code == D - 1) continue;
        const uint32_t b = code_bucket(code, D);
        if (SCATTER) {
          const uint32_t pos = atomicAdd(&s_cnt[b >> g.fb], 1u);
          const uint32_t i = (v0 + u * SORTC_WG) * 8 + k;
          part[pos] = i | ((code < D - 1 ? 1u : 0u) << g.vb) | ((b & fmask) << (g.vb + 1));
        } else {
          atomicAdd(&s_cnt[b >> g.fb], 1u);
        }
      }
    }
  }
}

// H[(w ncw + coarse) nch + chunk] <- entries of the chunk in the coarse bin
static __global__ void __launch_bounds__(SORTC_WG) k_sort_count(const uint16_t* __restrict__ dig, SortGeom g,
                                                         uint32_t* __restrict__ H) {
  __shared__ uint32_t s_cnt[SORT_COARSE_MAX];
  for (uint32_t b = threadIdx.x; b < g.ncw; b += SORTC_WG) s_cnt[b] = 0;
  __syncthreads();
  sort_coarse_chunk<false>(dig, g, s_cnt, nullptr);
  __syncthreads();
  const uint32_t w = blockIdx.x / g.nch, ch = blockIdx.x % g.nch;
  for (uint32_t b = threadIdx.x; b < g.ncw; b += SORTC_WG) H[(size_t(w) * g.ncw + b) * g.nch + ch] = s_cnt[b];
}

// packed entries (point | sign << vb | fine << (vb + 1)) grouped by (window,
// coarse bin).  The chunk is taken in tiles of SORTC_TILE codes: a tile's
// entries are first grouped by coarse bin in LDS, then written out with
// consecutive lanes on consecutive words of each bin's run, so that a run
// leaves in whole segments rather than as one scattered word per entry.
// Dynamic LDS: sort_coarse_lds_bytes(ncw).
constexpr uint32_t SORTC_TILE = 8 * 4 * SORTC_WG;  // four 16-byte loads of codes per thread

__host__ __device__ constexpr size_t sort_coarse_lds_bytes(uint32_t ncw) {
  return size_t(3) * ncw * 4 + size_t(SORTC_TILE) * 6 + (SORTC_WG / 64) * 4;
}

static __global__ void __launch_bounds__(SORTC_WG) k_sort_coarse(const uint16_t* __restrict__ dig, SortGeom g,
                                                          const uint32_t* __restrict__ Hs,
                                                          uint32_t* __restrict__ part) {
  extern __shared__ uint32_t smem[];
  uint32_t* s_cur = smem;               // ncw: global position of each bin's next entry
  uint32_t* s_cnt = s_cur + g.ncw;      // ncw: entries of the tile per bin
  uint32_t* s_off = s_cnt + g.ncw;      // ncw: first place of each bin in the tile
  uint32_t* s_ent = s_off + g.ncw;      // SORTC_TILE entries, grouped by bin
  uint16_t* s_bin = reinterpret_cast<uint16_t*>(s_ent + SORTC_TILE);  // their bins
  uint32_t* s_tmp = reinterpret_cast<uint32_t*>(s_bin + SORTC_TILE);  // scan partials
  const uint32_t w = blockIdx.x / g.nch, ch = blockIdx.x % g.nch;
  const uint32_t D = 1u << (g.c - 1);
  const uint32_t fmask = (1u << g.fb) - 1u;
  for (uint32_t b = threadIdx.x; b < g.ncw; b += SORTC_WG) {
    s_cur[b] = Hs[(size_t(w) * g.ncw + b) * g.nch + ch];
    s_cnt[b] = 0;
  }
  __syncthreads();
  const uint32_t lo = ch * (g.chunk / 8), hi = min(g.np, (ch + 1) * g.chunk) / 8;
  const uint4* src = reinterpret_cast<const uint4*>(dig + size_t(w) * g.np);
  const uint32_t per = (g.ncw + SORTC_WG - 1) / SORTC_WG;  // bins per thread in the scan
  constexpr int U = 4;
  for (uint32_t t0 = lo; t0 < hi; t0 += SORTC_TILE / 8) {
    // the tile's codes: entry and (bin, rank in the bin) of each, or none
    uint32_t ent[U * 8], br[U * 8];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint32_t v = t0 + u * SORTC_WG + threadIdx.x;
      const uint32_t z = (D - 1) * 0x10001u;  // eight zero digits
      const uint4 t = v < hi ? src[v] : make_uint4(z, z, z, z);
      Codes8 q;
      q.w[0] = t.x;
      q.w[1] = t.y;
      q.w[2] = t.z;
      q.w[3] = t.w;
#pragma unroll
      for (int k = 0; k < 8; k++) {
        const uint32_t code = q.at(k);
        br[u * 8 + k] = ~0u;
        ent[u * 8 + k] = 0;
        if (code != D - 1) {
          const uint32_t b = code_bucket(code, D);
          const uint32_t bin = b >> g.fb;
          const uint32_t rank = atomicAdd(&s_cnt[bin], 1u);
          ent[u * 8 + k] = (v * 8 + k) | ((code < D - 1 ? 1u : 0u) << g.vb) | ((b & fmask) << (g.vb + 1));
          br[u * 8 + k] = (bin << 16) | rank;
        }
      }
    }
    __syncthreads();
    // first place of each bin in the tile: each thread scans `per` consecutive bins
    uint32_t sum = 0;
    for (uint32_t i = 0; i < per; i++) {
      const uint32_t b = threadIdx.x * per + i;
      sum += b < g.ncw ? s_cnt[b] : 0u;
    }
    uint32_t total = 0;
    uint32_t run = block_exclusive_scan<SORTC_WG>(sum, s_tmp, total);
    for (uint32_t i = 0; i < per; i++) {
      const uint32_t b = threadIdx.x * per + i;
      if (b < g.ncw) {
        s_off[b] = run;
        run += s_cnt[b];
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < U * 8; e++) {
      if (br[e] != ~0u) {
        const uint32_t bin = br[e] >> 16, at = s_off[bin] + (br[e] & 0xFFFFu);
        s_ent[at] = ent[e];
        s_bin[at] = uint16_t(bin);
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < total; i += SORTC_WG) {
      const uint32_t bin = s_bin[i];
      part[s_cur[bin] + (i - s_off[bin])] = s_ent[i];
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < g.ncw; b += SORTC_WG) {
      s_cur[b] += s_cnt[b];
      s_cnt[b] = 0;
    }
    __syncthreads();
  }
}

// exclusive scan of s[0 .. n) in place (n <= SORT_FINE_MAXB), block of SORTF_WG
__device__ __forceinline__ void block_exclusive_scan(uint32_t* s, uint32_t n, uint32_t* s_wave) {
  constexpr uint32_t PER = SORT_FINE_MAXB / SORTF_WG;
  const uint32_t t = threadIdx.x, lane = t & 63u, wave = t >> 6;
  uint32_t v[PER];
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t j = t * PER + k;
    v[k] = j < n ? s[j] : 0u;
    sum += v[k];
  }
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d);
    if (lane >= uint32_t(d)) inc += o;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (uint32_t k = 0; k < wave; k++) base += s_wave[k];
  uint32_t run = base + inc - sum;
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t j = t * PER + k;
    if (j < n) s[j] = run;
    run += v[k];
  }
  __syncthreads();
}

// per (window, coarse bin): bucket counts and offsets, entries in bucket order
static __global__ void __launch_bounds__(SORTF_WG) k_sort_fine(const uint32_t* __restrict__ part, SortGeom g,
                                                        const uint32_t* __restrict__ Hs,
                                                        uint32_t* __restrict__ counts,
                                                        uint32_t* __restrict__ offsets,
                                                        uint32_t* __restrict__ sorted) {
  __shared__ uint32_t s_h[SORT_FINE_MAXB];
  __shared__ uint32_t s_in[SORT_FINE_CAP];
  __shared__ uint32_t s_out[SORT_FINE_CAP];
  __shared__ uint32_t s_wave[SORTF_WG / 64];
  const uint32_t t = threadIdx.x;
  const uint32_t w = blockIdx.x / g.ncw, cb = blockIdx.x % g.ncw;
  const size_t hb = (size_t(w) * g.ncw + cb) * g.nch;
  const uint32_t lo = Hs[hb], hi = Hs[hb + g.nch];
  const uint32_t cnt = hi - lo;
  const uint32_t nf = 1u << g.fb;
  const uint32_t sh = g.vb + 1;
  const uint32_t vmask = (1u << g.vb) - 1u;
  const bool in_lds = cnt <= SORT_FINE_CAP;
  for (uint32_t f = t; f < nf; f += SORTF_WG) s_h[f] = 0;
  __syncthreads();
  for (uint32_t j = t; j < cnt; j += SORTF_WG) {
    const uint32_t e = part[lo + j];
    if (in_lds) s_in[j] = e;
    atomicAdd(&s_h[e >> sh], 1u);
  }
  __syncthreads();
  const uint32_t D = 1u << (g.c - 1);
  const size_t b0 = size_t(w) * D + (size_t(cb) << g.fb);
  for (uint32_t f = t; f < nf; f += SORTF_WG) counts[b0 + f] = s_h[f];
  block_exclusive_scan(s_h, nf, s_wave);
  for (uint32_t f = t; f < nf; f += SORTF_WG) offsets[b0 + f] = lo + s_h[f];
  if (blockIdx.x == 0 && t == 0) {
    const size_t B = size_t(g.W) * D;
    counts[B] = 0;
    offsets[B] = Hs[size_t(g.W) * g.ncw * g.nch];
  }
  __syncthreads();
  if (in_lds) {
    for (uint32_t j = t; j < cnt; j += SORTF_WG) {
      const uint32_t e = s_in[j];
      const uint32_t pos = atomicAdd(&s_h[e >> sh], 1u);
      s_out[pos] = (e & vmask) | (((e >> g.vb) & 1u) << 31);
    }
    __syncthreads();
    for (uint32_t j = t; j < cnt; j += SORTF_WG) sorted[lo + j] = s_out[j];
  } else {
    for (uint32_t j = t; j < cnt; j += SORTF_WG) {
      const uint32_t e = part[lo + j];
      const uint32_t pos = atomicAdd(&s_h[e >> sh], 1u);
      sorted[lo + pos] = (e & vmask) | (((e >> g.vb) & 1u) << 31);
    }
  }
}

// ---- endomorphism split (single MSM on BN254 / BLS12-381) ------------------
// The MSM over n points becomes one over 2n: point i with scalar k1 and point
// n + i, (beta x_i, y_i) = [lambda] P_i, with scalar k2, where
// k_i = k1 + lambda k2 (mod r) and |k1|, |k2| < 2^BITS.  A negative half
// negates its point, so the digits are those of |k1| and |k2|.

// (k g + 2^319) >> 320 for 256-bit k and g (three words: the result is below 2^192)
__device__ __forceinline__ void glv_round320(const uint64_t k[4], const uint64_t (&g)[4], uint64_t c[3]) {
  uint64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 4; i++) {
    uint64_t cy = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const unsigned __int128 v = (unsigned __int128)k[i] * g[j] + t[i + j] + cy;
      t[i + j] = uint64_t(v);
      cy = uint64_t(v >> 64);
    }
    t[i + 4] = cy;
  }
  unsigned __int128 v = (unsigned __int128)t[4] + (1ull << 63);
  v = (unsigned __int128)t[5] + uint64_t(v >> 64);
  c[0] = uint64_t(v);
  v = (unsigned __int128)t[6] + uint64_t(v >> 64);
  c[1] = uint64_t(v);
  c[2] = t[7] + uint64_t(v >> 64);
}

// acc -= a b (mod 2^192)
__device__ __forceinline__ void glv_submul3(uint64_t acc[3], const uint64_t a[3], const uint64_t (&b)[3]) {
  uint64_t p[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 3; i++) {
    uint64_t cy = 0;
#pragma unroll
    for (int j = 0; i + j < 3; j++) {
      const unsigned __int128 v = (unsigned __int128)a[i] * b[j] + p[i + j] + cy;
      p[i + j] = uint64_t(v);
      cy = uint64_t(v >> 64);
    }
  }
  uint64_t br = 0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const uint64_t d = acc[k] - p[k];
    const uint64_t b1 = acc[k] < p[k];
    acc[k] = d - br;
    br = b1 | (d < br);
  }
}

// sign and magnitude of a 192-bit two's complement value; false if |v| >= 2^bits
__device__ __forceinline__ bool glv_magnitude(const uint64_t v[3], int bits, uint32_t m[8], bool& neg) {
  neg = (v[2] >> 63) != 0;
  uint64_t a[3] = {v[0], v[1], v[2]};
  if (neg) {
    uint64_t cy = 1;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const uint64_t t = ~a[k] + cy;
      cy = (cy && t == 0) ? 1 : 0;
      a[k] = t;
    }
  }
  const bool ok = a[2] == 0 && (bits >= 128 || (a[1] >> (bits - 64)) == 0);
#pragma unroll
  for (int k = 0; k < 2; k++) {
    m[2 * k] = uint32_t(a[k]);
    m[2 * k + 1] = uint32_t(a[k] >> 32);
  }
#pragma unroll
  for (int k = 4; k < 8; k++) m[k] = 0;
  return ok;
}

// k (eight 32-bit words, below 2^bitlen(r)) -> |k1|, |k2| and their signs
template <class C>
__device__ __forceinline__ bool glv_split(const uint32_t s[8], uint32_t m1[8], bool& n1, uint32_t m2[8], bool& n2) {
  using G = Glv<C>;
  constexpr Words<8> R32 = C::ORDER;
  uint64_t k[4], r[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    k[i] = uint64_t(s[2 * i]) | (uint64_t(s[2 * i + 1]) << 32);
    r[i] = uint64_t(R32.w[2 * i]) | (uint64_t(R32.w[2 * i + 1]) << 32);
  }
  // k mod r: k < 2^bitlen(r) < 2 r
  bool ge = true;
#pragma unroll
  for (int i = 3; i >= 0; i--) {
    if (k[i] != r[i]) {
      ge = k[i] > r[i];
      break;
    }
  }
  if (ge) {
    uint64_t br = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const uint64_t d = k[i] - r[i];
      const uint64_t b1 = k[i] < r[i];
      k[i] = d - br;
      br = b1 | (d < br);
    }
  }
  uint64_t c1[3], c2[3];
  glv_round320(k, G::G1, c1);
  glv_round320(k, G::G2, c2);
  uint64_t k1[3] = {k[0], k[1], k[2]};
  glv_submul3(k1, c1, G::A1);
  glv_submul3(k1, c2, G::A2);
  uint64_t k2[3] = {0, 0, 0};
  glv_submul3(k2, c1, G::B1);
  glv_submul3(k2, c2, G::B2);
  const bool ok1 = glv_magnitude(k1, G::BITS, m1, n1);
  const bool ok2 = glv_magnitude(k2, G::BITS, m2, n2);
  return ok1 && ok2;
}

// signed-digit codes of all windows of s into column col of the digit table
__device__ __forceinline__ void put_digits(const uint32_t s[8], bool live, const SortGeom& g,
                                           uint16_t* __restrict__ dig, uint32_t col) {
  const int c = int(g.c);
  const uint32_t D = 1u << (c - 1);
  uint32_t carry = 0;
  for (uint32_t w = 0; w < g.W; w++) {
    uint32_t code = D - 1;
    if (live) {
      int32_t d = int32_t(window_bits(s, c * int(w), c) + carry);
      carry = 0;
      if (d > int32_t(D)) {
        d -= int32_t(1u << c);
        carry = 1;
      }
      code = uint32_t(d + int32_t(D) - 1);
    }
    dig[size_t(w) * g.np + col] = uint16_t(code);
  }
}

// Ingest of a single MSM with the endomorphism split: thread i converts base
// i, writes the points i and n + i (negated where their half-scalar is
// negative) and the digit codes of |k1| and |k2| into columns i and n + i.
// Threads past n fill the padding columns [2n, np) with zero digits.  A
// point at infinity, a rejected base or a rejected scalar contributes no
// digits; rejections set error bits.
template <class C>
__global__ void __launch_bounds__(256) k_ingest_glv(const uint32_t* __restrict__ in,
                                                    const uint32_t* __restrict__ scalars, uint32_t n, int in_mont,
                                                    int check_curve, SortGeom g, int bits,
                                                    uint32_t* __restrict__ out, uint16_t* __restrict__ dig,
                                                    uint32_t* __restrict__ err) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  constexpr int PW = affine_words<C>();
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) {
    const uint32_t col = n + i;
    if (col < g.np) {
      uint32_t z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      put_digits(z, false, g, dig, col);
    }
    return;
  }
  uint32_t xw[N32], yw[N32];
  words_load<F>(in + size_t(i) * 2 * N32, xw);
  words_load<F>(in + size_t(i) * 2 * N32 + N32, yw);
  uint32_t any = 0;
#pragma unroll
  for (int k = 0; k < N32; k++) any |= xw[k] | yw[k];
  const bool inf = any == 0;
  uint32_t e = 0;
  Affine<C> P1, P2;
  if (!inf) {
    if (!words_lt_p<F>(xw) || !words_lt_p<F>(yw)) e |= ERRF_RANGE;
    Affine<C> P;
    P.x = fp_from_words<F>(xw);
    P.y = fp_from_words<F>(yw);
    constexpr Words<F::NL> rin = F::RIN, r2 = F::R2;
    const Fp<F> kin = fp_from<F>(in_mont ? rin : r2);
    P.x = fp_canonical<F>(fp_mul<F>(P.x, kin));
    P.y = fp_canonical<F>(fp_mul<F>(P.y, kin));
    if (check_curve && !e && !affine_on_curve<C>(P)) e |= ERRF_NOT_ON_CURVE;
    constexpr Words<F::NL> beta = Glv<C>::BETA;
    P1 = P;
    P2.x = fp_canonical<F>(fp_mul<F>(P.x, fp_from<F>(beta)));
    P2.y = P.y;
  } else {
    P1.x = P2.x = fp_inf_marker<F>();
    P1.y = P2.y = fp_zero<F>();
  }
  uint32_t s[8];
  load_scalar(scalars + 8 * size_t(i), s);
  bool live = !inf && !e;
  if (!scalar_fits(s, bits)) {
    e |= ERRF_SCALAR_RANGE;
    live = false;
  }
  uint32_t m1[8], m2[8];
  bool n1 = false, n2 = false;
  if (live && !glv_split<C>(s, m1, n1, m2, n2)) {
    e |= ERRF_SPLIT;
    live = false;
  }
  if (e) atomicOr(err, e);
  if (live && n1) P1.y = fp_neg_canonical<F>(P1.y);
  if (live && n2) P2.y = fp_neg_canonical<F>(P2.y);
  affine_store<C>(out + size_t(i) * PW, P1);
  affine_store<C>(out + size_t(n + i) * PW, P2);
  put_digits(m1, live, g, dig, i);
  put_digits(m2, live, g, dig, n + i);
}

// Ingest of a batch with the endomorphism split: input point i (of MSM j,
// read in place through ptrs[j] when given) becomes points 2i and 2i + 1,
// P_i and phi(P_i) = (beta x, y), each negated where its half-scalar is
// negative, and their half-scalars |k1|, |k2| (below 2^bits_half, as 8-word
// scalars) go to hs[2i] and hs[2i + 1].  MSM j then covers [2 first_j,
// 2 first_j + 2 n_j) of the doubled index space (msms[] holds the doubled
// ranges), so the batch grouping runs on it unchanged.  A point at infinity
// or a rejected base or scalar is skipped (both halves); rejections set
// error bits.
template <class C>
__global__ void __launch_bounds__(256) k_ingest_glv_batch(const uint32_t* __restrict__ in,
                                                          const uint32_t* __restrict__ scalars, uint32_t n,
                                                          int in_mont, int check_curve, int bits,
                                                          uint32_t* __restrict__ out, uint32_t* __restrict__ hs,
                                                          uint8_t* __restrict__ skip, uint32_t* __restrict__ err,
                                                          const uint64_t* __restrict__ ptrs,
                                                          const MsmDesc* __restrict__ msms, uint32_t m) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  constexpr int PW = affine_words<C>();
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint32_t* src = in + size_t(i) * 2 * N32;
  if (ptrs) {
    const uint32_t j = find_msm(msms, m, 2 * i);
    src = reinterpret_cast<const uint32_t*>(ptrs[j]) + size_t(i - msms[j].first / 2) * 2 * N32;
  }
  uint32_t xw[N32], yw[N32];
  words_load<F>(src, xw);
  words_load<F>(src + N32, yw);
  uint32_t any = 0;
#pragma unroll
  for (int k = 0; k < N32; k++) any |= xw[k] | yw[k];
  const bool inf = any == 0;
  uint32_t e = 0;
  Affine<C> P1, P2;
  if (!inf) {
    if (!words_lt_p<F>(xw) || !words_lt_p<F>(yw)) e |= ERRF_RANGE;
    Affine<C> P;
    P.x = fp_from_words<F>(xw);
    P.y = fp_from_words<F>(yw);
    constexpr Words<F::NL> rin = F::RIN, r2 = F::R2;
    const Fp<F> kin = fp_from<F>(in_mont ? rin : r2);
    P.x = fp_canonical<F>(fp_mul<F>(P.x, kin));
    P.y = fp_canonical<F>(fp_mul<F>(P.y, kin));
    if (check_curve && !e && !affine_on_curve<C>(P)) e |= ERRF_NOT_ON_CURVE;
    constexpr Words<F::NL> beta = Glv<C>::BETA;
    P1 = P;
    P2.x = fp_canonical<F>(fp_mul<F>(P.x, fp_from<F>(beta)));
    P2.y = P.y;
  } else {
    P1.x = P2.x = fp_inf_marker<F>();
    P1.y = P2.y = fp_zero<F>();
  }
  uint32_t s[8];
  load_scalar(scalars + 8 * size_t(i), s);
  bool live = !inf && !e;
  if (!scalar_fits(s, bits)) {
    e |= ERRF_SCALAR_RANGE;
    live = false;
  }
  uint32_t m1[8] = {0, 0, 0, 0, 0, 0, 0, 0}, m2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool n1 = false, n2 = false;
  if (live && !glv_split<C>(s, m1, n1, m2, n2)) {
    e |= ERRF_SPLIT;
    live = false;
  }
  if (e) atomicOr(err, e);
  if (live && n1) P1.y = fp_neg_canonical<F>(P1.y);
  if (live && n2) P2.y = fp_neg_canonical<F>(P2.y);
  affine_store<C>(out + size_t(2 * i) * PW, P1);
  affine_store<C>(out + size_t(2 * i + 1) * PW, P2);
  uint4* h = reinterpret_cast<uint4*>(hs + size_t(2 * i) * 8);
  h[0] = make_uint4(m1[0], m1[1], m1[2], m1[3]);
  h[1] = make_uint4(m1[4], m1[5], m1[6], m1[7]);
  h[2] = make_uint4(m2[0], m2[1], m2[2], m2[3]);
  h[3] = make_uint4(m2[4], m2[5], m2[6], m2[7]);
  skip[2 * i] = skip[2 * i + 1] = live ? 0 : 1;
}

// n uniform words of at most `bits` bits each group of 8 (a 256-bit value
// below 2^bits), from a counter-based mix of (seed, index); inputs for the
// window tuner only
static __global__ void k_random_scalars(uint32_t* __restrict__ out, size_t n, uint64_t seed, int bits) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 8; k++) {
    // SplitMix64 finaliser on (seed, i, k)
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t(i) * 8 + uint64_t(k) + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    uint32_t v = uint32_t(z);
    int lo = 32 * k;
    if (lo >= bits) v = 0;
    else if (bits - lo < 32) v &= (1u << (bits - lo)) - 1u;
    out[i * 8 + k] = v;
  }
}

// fill n words with v (used instead of memset so that a captured launch
// sequence holds kernel nodes only)
static __global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// *sticky |= *bits (one thread)
static __global__ void k_or_u32(const uint32_t* __restrict__ bits, uint32_t* __restrict__ sticky) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *sticky |= *bits;
}

static __global__ void k_fill_u8(uint8_t* __restrict__ p, size_t n, uint8_t v) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// exclusive scan (three phases: block scan, scan of block sums, add back)

constexpr int SCAN_WG = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_TILE = SCAN_WG * SCAN_PER_THREAD;

static __global__ void __launch_bounds__(SCAN_WG) k_scan_tiles(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        uint32_t* __restrict__ sums, size_t n) {
  __shared__ uint32_t s_tmp[SCAN_WG / 64];
  size_t base = size_t(blockIdx.x) * SCAN_TILE + size_t(threadIdx.x) * SCAN_PER_THREAD;
  uint32_t v[SCAN_PER_THREAD];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; k++) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    local += v[k];
  }
  uint32_t total;
  uint32_t before = block_exclusive_scan<SCAN_WG>(local, s_tmp, total);
#pragma unroll
  for (int k = 0; k < SCAN_PER_THREAD; k++) {
    if (base + k < n) out[base + k] = before;
    before += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

static __global__ void k_scan_add(uint32_t* __restrict__ out, const uint32_t* __restrict__ sums, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / SCAN_TILE];
}

// ---------------------------------------------------------------------------
// per-bucket addition schedule.
//
// Round r of bucket b takes its l_r live entries (l_0 = n_b, l_{r+1} =
// ceil(l_r / 2)) as the pairs (2i, 2i + 1), i < floor(l_r / 2), adds each
// pair into entry i of the round's output, and copies an odd last entry to
// entry floor(l_r / 2).  Round 0 reads the sorted entries of the bucket
// (points gathered from the bases, negated for negative digits); later rounds
// read the previous round's output.  Outputs alternate between two slot
// buffers (A for even rounds, B for odd), each with separate x and y planes,
// so that a pair's two x coordinates are adjacent.  A bucket's entries start
// at an even slot index (bucket_slot), which keeps a pair inside one
// 128-byte line of each plane.  A bucket takes part in rounds 0 .. R_b - 1,
// R_b = max(1, ceil(log2 n_b)), and its sum ends at bucket_slot in buffer
// A when R_b is odd, B when it is even.

__host__ __device__ inline uint32_t bucket_slot(uint32_t offset, uint32_t b) { return (offset + b + 1u) & ~1u; }

__host__ __device__ inline int bucket_rounds(uint32_t n) {
  int r = 0;
  while ((1u << r) < n) r++;
  return r < 1 ? 1 : r;
}

// descriptors: (first input entry, output entry) per pair, and per odd tail.
// A thread writes the pairs of its own bucket; a bucket of more than
// PLAN_BIG_PAIRS pairs in a round (a skewed window, e.g. a top window that
// holds only a few bits of every scalar, so that a handful of buckets take
// most of its points) is written by the whole workgroup instead, so that no
// single thread walks hundreds of thousands of entries.
constexpr uint32_t PLAN_BIG_PAIRS = 256;

template <int WG>
__global__ void __launch_bounds__(WG) k_plan(const uint32_t* __restrict__ counts, const uint32_t* __restrict__ offsets,
                                             uint32_t B, uint2* __restrict__ desc, const size_t* __restrict__ desc_base,
                                             uint2* __restrict__ tails, const size_t* __restrict__ tail_base,
                                             uint32_t* __restrict__ round_counts, uint32_t* __restrict__ tail_counts,
                                             uint32_t* __restrict__ max_count) {
  __shared__ uint32_t s_tmp[WG / 64];
  __shared__ uint32_t s_base[2];
  __shared__ uint32_t s_nbig;
  __shared__ uint32_t s_big_in[WG], s_big_so[WG], s_big_at[WG], s_big_pairs[WG];
  const uint32_t b = blockIdx.x * WG + threadIdx.x;
  const uint32_t n = b < B ? counts[b] : 0u;
  const uint32_t off = b < B ? offsets[b] : 0u;
  const uint32_t so = bucket_slot(off, b);
  {  // the largest bucket: a wave maximum, an LDS maximum, one device atomic per workgroup
    __shared__ uint32_t s_max;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    uint32_t mx = n;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, uint32_t(__shfl_xor(int(mx), d, 64)));
    if ((threadIdx.x & 63) == 0 && mx) atomicMax(&s_max, mx);
    __syncthreads();
    if (threadIdx.x == 0 && s_max) atomicMax(max_count, s_max);
  }
  for (int r = 0; r < MAX_ROUNDS; r++) {
    const uint32_t l = uint32_t((uint64_t(n) + (1ull << r) - 1) >> r);
    const bool active = r == 0 ? l >= 1 : l >= 2;
    const uint32_t pairs = active ? l >> 1 : 0u;
    const uint32_t tail = active ? (l & 1u) : 0u;
    uint32_t tot_p, tot_t;
    const uint32_t lp = block_exclusive_scan<WG>(pairs, s_tmp, tot_p);
    const uint32_t lt = block_exclusive_scan<WG>(tail, s_tmp, tot_t);
    if (tot_p == 0 && tot_t == 0) break;
    if (threadIdx.x == 0) {
      s_base[0] = tot_p ? atomicAdd(&round_counts[r], tot_p) : 0u;
      s_base[1] = tot_t ? atomicAdd(&tail_counts[r], tot_t) : 0u;
    }
    __syncthreads();
    const uint32_t bp = s_base[0], bt = s_base[1];
    if (threadIdx.x == 0) s_nbig = 0;
    __syncthreads();
    const uint32_t in = r == 0 ? off : so;  // round 0 reads the sorted entries
    if (pairs > PLAN_BIG_PAIRS) {
      const uint32_t k = atomicAdd(&s_nbig, 1u);  // k < WG: one slot per thread at most
      s_big_in[k] = in;
      s_big_so[k] = so;
      s_big_at[k] = bp + lp;
      s_big_pairs[k] = pairs;
    }
    {
      // the other buckets' pairs: each lane writes its own run when the runs
      // are short; when some run of the wave is long, the wave writes the
      // runs one after another, consecutive lanes on consecutive pairs
      const uint32_t mine = pairs > PLAN_BIG_PAIRS ? 0u : pairs;
      uint2* dr = desc + desc_base[r] + bp;
      uint32_t wmax = mine;
#pragma unroll
      for (int dd = 32; dd >= 1; dd >>= 1) wmax = max(wmax, uint32_t(__shfl_xor(int(wmax), dd, 64)));
      if (wmax < 8) {
        for (uint32_t j = 0; j < mine; j++) dr[lp + j] = make_uint2(in + 2 * j, so + j);
      } else {
        const uint32_t lane = threadIdx.x & 63u;
        for (int t = 0; t < 64; t++) {
          const uint32_t np = __builtin_amdgcn_readlane(mine, t);
          if (np == 0) continue;
          const uint32_t at = __builtin_amdgcn_readlane(lp, t);
          const uint32_t tin = __builtin_amdgcn_readlane(in, t);
          const uint32_t tso = __builtin_amdgcn_readlane(so, t);
          for (uint32_t j = lane; j < np; j += 64) dr[at + j] = make_uint2(tin + 2 * j, tso + j);
        }
      }
    }
    if (tail) tails[tail_base[r] + bt + lt] = make_uint2(in + l - 1, so + pairs);
    __syncthreads();
    const uint32_t nbig = s_nbig;
    for (uint32_t k = 0; k < nbig; k++) {
      const uint32_t bin = s_big_in[k], bso = s_big_so[k], np = s_big_pairs[k];
      uint2* d = desc + desc_base[r] + s_big_at[k];
      for (uint32_t j = threadIdx.x; j < np; j += WG) d[j] = make_uint2(bin + 2 * j, bso + j);
    }
    __syncthreads();  // the slots are refilled in the next round
  }
}

// ---------------------------------------------------------------------------
// one round of pairwise batch-affine additions (Section 3: Montgomery's trick
// over all additions of the round; x-only compress, DCWPA recomputing the
// denominators, GAS inversion per workgroup)

// the x and y coordinates of input entry e of a round: gathered from the
// bases through the sorted entry in round 0 (y negated for a negative digit),
// from the previous round's planes otherwise
template <class C>
__device__ __forceinline__ Fp<typename C::F> load_x(const uint32_t* __restrict__ bases,
                                                    const uint32_t* __restrict__ sorted,
                                                    const uint32_t* __restrict__ in_x, uint32_t e, int from_bases) {
  using F = typename C::F;
  constexpr int PW = affine_words<C>();
  if (from_bases) {
    uint32_t idx = sorted[e] & ~SIGN_BIT;
    return fp_load<F>(bases + size_t(idx) * PW);
  }
  return fp_load<F>(in_x + size_t(e) * F::CW);
}

template <class C>
__device__ __forceinline__ Fp<typename C::F> load_y(const uint32_t* __restrict__ bases,
                                                    const uint32_t* __restrict__ sorted,
                                                    const uint32_t* __restrict__ in_y, uint32_t e, int from_bases) {
  using F = typename C::F;
  constexpr int PW = affine_words<C>();
  if (from_bases) {
    uint32_t idx = sorted[e];
    Fp<F> y = fp_load<F>(bases + size_t(idx & ~SIGN_BIT) * PW + F::CW);
    return (idx & SIGN_BIT) ? fp_neg_canonical<F>(y) : y;
  }
  return fp_load<F>(in_y + size_t(e) * F::CW);
}

// the same split in two steps, so that a loop can resolve an entry one step
// before it loads the point: the source of entry e is its sorted word in
// round 0 (point index, sign of the digit) and e itself in later rounds
__device__ __forceinline__ uint32_t entry_src(const uint32_t* __restrict__ sorted, uint32_t e, int from_bases) {
  return from_bases ? sorted[e] : e;
}

template <class C>
__device__ __forceinline__ Fp<typename C::F> src_x(const uint32_t* __restrict__ bases,
                                                   const uint32_t* __restrict__ in_x, uint32_t s, int from_bases) {
  using F = typename C::F;
  if (from_bases) return fp_load<F>(bases + size_t(s & ~SIGN_BIT) * affine_words<C>());
  return fp_load<F>(in_x + size_t(s) * F::CW);
}

template <class C>
__device__ __forceinline__ Fp<typename C::F> src_y(const uint32_t* __restrict__ bases,
                                                   const uint32_t* __restrict__ in_y, uint32_t s, int from_bases) {
  using F = typename C::F;
  if (from_bases) {
    Fp<F> y = fp_load<F>(bases + size_t(s & ~SIGN_BIT) * affine_words<C>() + F::CW);
    return (s & SIGN_BIT) ? fp_neg_canonical<F>(y) : y;
  }
  return fp_load<F>(in_y + size_t(s) * F::CW);
}

enum : int { CLS_ADD = 0, CLS_DBL = 1, CLS_INF = 2, CLS_COPY1 = 3, CLS_COPY2 = 4 };

// lanes used for a round of n additions on a grid of at most `cap` lanes:
// enough lanes for about kmin additions each, a multiple of the workgroup
__host__ __device__ inline uint32_t round_lane_count(uint32_t n, uint32_t cap, uint32_t wg, uint32_t kmin) {
  uint32_t t = (n + kmin - 1) / kmin;
  t = (t + wg - 1) / wg * wg;
  if (t < wg) t = wg;
  return t < cap ? t : cap;
}

// The last rounds hold few additions each and so are bound by the latency
// of their inversion rather than by work.  Once a round would hold fewer
// than `few` additions (it can no longer give the grid's lanes two each) and
// every bucket is down to at most `lmax` partial sums, the remaining rounds
// are replaced by one pass that adds each bucket's partial sums on its own
// lane (k_bucket_finish).  Rounds run: the first such R >= 1 when it is
// fewer than the nr rounds with work (lmax = 0: never).  counts[r]: the
// additions of round r.
__host__ __device__ inline uint32_t finish_round(const uint32_t* counts, uint32_t max_count, uint32_t nr,
                                                 uint32_t lmax, uint32_t few) {
  if (lmax == 0) return nr;
  for (uint32_t R = 1; R < nr; R++)
    if (counts[R] < few && ((uint64_t(max_count) + (1ull << R) - 1) >> R) <= lmax) return R;
  return nr;
}

// launch parameters of every round from the per-round addition counts
// (counts[r]) and copy counts (counts[MAX_ROUNDS + r]), one thread:
// (additions, lanes, additions per lane, active); rounds past
// the last one get n = 0, rounds replaced by k_bucket_finish active = 0;
// params[MAX_ROUNDS] = (rounds run, rounds with work).
static __global__ void k_round_params(const uint32_t* __restrict__ counts, uint32_t cap, uint32_t wg, uint32_t kmin,
                                      uint4* __restrict__ params, const uint32_t* __restrict__ max_count,
                                      uint32_t lmax) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // rounds with work: additions, or (round 0 only) copies of one-entry buckets;
  // the copies of every round follow the additions at counts + MAX_ROUNDS
  uint32_t nr = 0;
  while (nr < MAX_ROUNDS && (counts[nr] || counts[MAX_ROUNDS + nr])) nr++;
  const uint32_t R = finish_round(counts, *max_count, nr, lmax, 2 * cap);
  for (int r = 0; r < MAX_ROUNDS; r++) {
    uint32_t n = counts[r];
    uint32_t T = round_lane_count(n, cap, wg, kmin);
    params[r] = make_uint4(n, T, n ? (n + T - 1) / T : 0u, uint32_t(r) < R ? 1u : 0u);
  }
  params[MAX_ROUNDS] = make_uint4(R, nr, 0u, 0u);
}

// Design variants of the round kernel, for ablations of the choices the paper
// makes for batch PADD (Section 3.3).  The default (0) is the library's form;
// each bit switches one choice off.  Every variant computes the same sums.
enum : int {
  RV_STORE_DENOM = 1,  // store each denominator in the compress step and load it
                       // back in the decompress step instead of recomputing it
                       // from the reloaded coordinates
  RV_AOS_CHAIN = 2,    // prefix products stored per lane, contiguous (each lane's
                       // chain in one run) instead of limb-major planes whose
                       // accesses coalesce across the lanes of a wave
  RV_SPLIT_APPLY = 4,  // decompress writes every inverse 1/d_i to memory and a
                       // second kernel (k_round_apply) does the additions,
                       // reloading the points, instead of one fused DCWPA step
  RV_LANE_INV = 8,     // every lane inverts its own chain product (Fermat) instead
                       // of one GAS inversion per workgroup (Section 3.2)
  RV_HALF_PREFIX = 64, // find-then-recompute (Section 3.4) in the rounds: the compress
                       // step stores the prefix products of even steps only, and the
                       // decompress step recomputes an odd step's M_i = M_{i-1} d_{i-1}
                       // (one more product per two additions, half the chain traffic)
  // host-side choices of where the rounds stop (the round kernel is unchanged):
  // by default a single MSM stops them early and adds each bucket's last
  // partial sums on its own lane (k_bucket_finish), a batch runs them to the end
  RV_FINISH = 16,      // the finishing pass for batches too
  RV_ROUNDS_ONLY = 32, // rounds to the end for every call (the paper's form)
  RV_KERNEL_MASK = 15 | 64  // the bits that select a round-kernel variant
};

// word offset of prefix product i of lane g (T lanes, at most kmax products
// per lane) and the stride between its limbs
template <int V, int NL>
__device__ __forceinline__ size_t chain_at(uint32_t i, uint32_t g, uint32_t T, uint32_t kmax) {
  if constexpr ((V & RV_AOS_CHAIN) != 0) return (size_t(g) * kmax + i) * NL;
  else return size_t(i) * NL * T + g;
}
template <int V>
__device__ __forceinline__ size_t chain_stride(uint32_t T) {
  if constexpr ((V & RV_AOS_CHAIN) != 0) return 1;
  else return T;
}

// a^-1 R (for a R in the working form) by Fermat, a^(p-2), on one lane:
// square-and-multiply over the bits of p - 2, most significant first
template <class F>
__device__ __noinline__ Fp<F> fp_inv_fermat(const Fp<F>& a) {
  constexpr Words<F::N32> p = F::P32;
  Fp<F> r = fp_one<F>();
#pragma unroll 1
  for (int wi = F::N32 - 1; wi >= 0; wi--) {
    const uint32_t e = p.w[wi] - (wi == 0 ? 2u : 0u);  // p is odd and its low word exceeds 2
#pragma unroll 1
    for (int b = 31; b >= 0; b--) {
      r = fp_sqr<F>(r);
      if ((e >> b) & 1u) r = fp_mul<F>(r, a);
    }
  }
  return r;
}

// Wave priority by progress through a round.  The workgroups that share a
// compute unit hold the same work, but the arbiter favours some of them: they
// finish early and leave the unit to the last one, which then runs alone at a
// fraction of the issue rate.  A wave lowers its priority as it passes each
// quarter of its work (a compress step weighs 1, a decompress step 2), so the
// waves that lag are issued first.  `done` and `total` are wave-uniform.
__device__ __forceinline__ void round_priority(uint32_t done, uint32_t total) {
  const uint32_t band = uint32_t(4 * done >= total) + uint32_t(4 * done >= 2 * total) + uint32_t(4 * done >= 3 * total);
  if (band == 0) __builtin_amdgcn_s_setprio(3);
  else if (band == 1) __builtin_amdgcn_s_setprio(2);
  else if (band == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// Round parameters (additions n, lanes T, additions per lane kmax) are read
// from device memory (written by k_round_params after planning), so the
// launch needs no host round trip; lanes beyond T leave at once.
// OCC: waves per SIMD the register allocation aims at (a tuning knob);
// V: design variant (RV_* bits, 0 in the library's own path).  dscr is the
// stored-denominator area of RV_STORE_DENOM (laid out like mscr).
template <class C, int WG, int OCC, int V = 0>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(OCC))) k_bucket_round(const uint32_t* __restrict__ bases,
                                                     const uint32_t* __restrict__ sorted,
                                                     const uint32_t* __restrict__ in_x, const uint32_t* __restrict__ in_y,
                                                     uint32_t* __restrict__ out_x, uint32_t* __restrict__ out_y,
                                                     const uint2* __restrict__ desc,
                                                     const uint4* __restrict__ prm, int from_bases,
                                                     uint32_t* __restrict__ mscr, const uint2* __restrict__ tails,
                                                     const uint32_t* __restrict__ n_tails,
                                                     uint32_t* __restrict__ dscr = nullptr) {
  using F = typename C::F;
  constexpr int NL = F::NL;
  constexpr int CW = F::CW;
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  const uint4 pr = *prm;
  const uint32_t n_adds = pr.x, T = pr.y, kmax = pr.z;
  if (blockIdx.x * WG >= T || pr.w == 0) return;  // uniform: lanes past T, or a round left to k_bucket_finish
  const uint32_t g = blockIdx.x * WG + threadIdx.x;
  // odd last entries of the round's buckets: plain copies to their outputs
  const uint32_t nt = *n_tails;
  for (uint32_t t = g; t < nt; t += T) {
    const uint2 d = tails[t];
    Fp<F> x = load_x<C>(bases, sorted, in_x, d.x, from_bases);
    Fp<F> y = load_y<C>(bases, sorted, in_y, d.x, from_bases);
    fp_store<F>(out_x + size_t(d.y) * CW, x);
    fp_store<F>(out_y + size_t(d.y) * CW, y);
  }
  if (n_adds == 0) return;  // uniform: a round of copies only
  uint32_t cnt = 0;
  if (g < n_adds) cnt = min(kmax, (n_adds - 1 - g) / T + 1);
  const Fp<F> one = fp_one<F>();
  const size_t cs = chain_stride<V>(T);

  // compress: M_i = d_0 ... d_{i-1}, acc = d_0 ... d_{cnt-1}; the stored
  // points are canonical, so coordinate equality is limb equality.  A pair is
  // input entries (e, e + 1); its sum goes to output entry o.  The loads run
  // ahead of the products in three stages, so that no step waits on a chain
  // of dependent loads: descriptors two steps ahead, the entries' sources
  // (sorted words in round 0) and then the x coordinates one step ahead.
  Fp<F> acc = one;
  uint32_t s1c = 0, s2c = 0, s1n = 0, s2n = 0, e_ahead = 0;
  Fp<F> x1n, x2n;
  if (cnt > 0) {
    const uint32_t e0 = desc[g].x;
    s1c = entry_src(sorted, e0, from_bases);
    s2c = entry_src(sorted, e0 + 1, from_bases);
    x1n = src_x<C>(bases, in_x, s1c, from_bases);
    x2n = src_x<C>(bases, in_x, s2c, from_bases);
    if (cnt > 1) {
      const uint32_t e1 = desc[g + T].x;
      s1n = entry_src(sorted, e1, from_bases);
      s2n = entry_src(sorted, e1 + 1, from_bases);
    }
    if (cnt > 2) e_ahead = desc[g + 2 * T].x;
  }
  const uint32_t work = 3 * kmax;  // progress units of the longest lane
  round_priority(0, work);
  for (uint32_t i = 0; i < cnt; i++) {
    round_priority(__builtin_amdgcn_readfirstlane(i), work);
    const uint32_t s1 = s1c, s2 = s2c;
    const Fp<F> x1 = x1n, x2 = x2n;
    if (i + 1 < cnt) {
      s1c = s1n;
      s2c = s2n;
      x1n = src_x<C>(bases, in_x, s1c, from_bases);
      x2n = src_x<C>(bases, in_x, s2c, from_bases);
      if (i + 2 < cnt) {
        s1n = entry_src(sorted, e_ahead, from_bases);
        s2n = entry_src(sorted, e_ahead + 1, from_bases);
        if (i + 3 < cnt) e_ahead = desc[g + (i + 3) * T].x;
      }
    }
    bool inf1 = !from_bases && fp_is_inf_marker<F>(x1);
    bool inf2 = !from_bases && fp_is_inf_marker<F>(x2);
    bool eqx = fp_eq_canonical<F>(x1, x2);
    Fp<F> d = fp_sub_lazy<F>(x2, x1);
    if (inf1 || inf2 || eqx) {
      d = one;
      if (!inf1 && !inf2) {
        Fp<F> y1 = src_y<C>(bases, in_y, s1, from_bases);
        Fp<F> y2 = src_y<C>(bases, in_y, s2, from_bases);
        if (fp_eq_canonical<F>(y1, y2)) d = fp_dbl<F>(y1);
      }
    }
    if constexpr ((V & RV_HALF_PREFIX) != 0) {
      if ((i & 1u) == 0) fp_store_soa<F>(mscr + chain_at<V, NL>(i >> 1, g, T, kmax), cs, acc);
    } else {
      const size_t at = chain_at<V, NL>(i, g, T, kmax);
      fp_store_soa<F>(mscr + at, cs, acc);
      if constexpr ((V & RV_STORE_DENOM) != 0) fp_store_soa<F>(dscr + at, cs, d);
    }
    acc = fp_mul<F>(acc, d);
  }

  Fp<F> inv;
  if constexpr ((V & RV_LANE_INV) != 0) {
    inv = fp_inv_fermat<F>(acc);
  } else {
    inv = wg_batch_inverse<F, WG, 10 + OCC>(acc, s_tot, s_inv);
  }

  if constexpr ((V & RV_HALF_PREFIX) != 0) {
    // decompress with find-then-recompute: an odd step rebuilds its M_i from
    // the stored M_{i-1} and the denominator d_{i-1} of the step below it (the
    // compress step's d, special lanes included); that step then reuses
    // M_{i-1} and its sources, and loads its x coordinates again (from cache)
    Fp<F> m_e;
    uint32_t s1_e = 0, s2_e = 0;
    uint2 dsc_e = make_uint2(0u, 0u);
    bool carried = false;
    for (int i = int(cnt) - 1; i >= 0; i--) {
      round_priority(__builtin_amdgcn_readfirstlane(kmax + 2 * (kmax - 1 - uint32_t(i))), work);
      uint2 dsc;
      uint32_t s1, s2;
      Fp<F> x1, x2, m;
      if (carried) {
        dsc = dsc_e;
        s1 = s1_e;
        s2 = s2_e;
        x1 = src_x<C>(bases, in_x, s1, from_bases);
        x2 = src_x<C>(bases, in_x, s2, from_bases);
        m = m_e;
        carried = false;
      } else {
        dsc = desc[g + uint32_t(i) * T];
        s1 = entry_src(sorted, dsc.x, from_bases);
        s2 = entry_src(sorted, dsc.x + 1, from_bases);
        x1 = src_x<C>(bases, in_x, s1, from_bases);
        x2 = src_x<C>(bases, in_x, s2, from_bases);
        if ((i & 1) == 0) {
          m = fp_load_soa<F>(mscr + chain_at<V, NL>(uint32_t(i) >> 1, g, T, kmax), cs);
        } else {
          dsc_e = desc[g + uint32_t(i - 1) * T];
          s1_e = entry_src(sorted, dsc_e.x, from_bases);
          s2_e = entry_src(sorted, dsc_e.x + 1, from_bases);
          const Fp<F> x1_e = src_x<C>(bases, in_x, s1_e, from_bases);
          const Fp<F> x2_e = src_x<C>(bases, in_x, s2_e, from_bases);
          m_e = fp_load_soa<F>(mscr + chain_at<V, NL>(uint32_t(i - 1) >> 1, g, T, kmax), cs);
          // d_{i-1} exactly as the compress step formed it
          Fp<F> de = fp_sub_lazy<F>(x2_e, x1_e);
          const bool ei1 = !from_bases && fp_is_inf_marker<F>(x1_e);
          const bool ei2 = !from_bases && fp_is_inf_marker<F>(x2_e);
          if (ei1 || ei2 || fp_eq_canonical<F>(x1_e, x2_e)) {
            de = one;
            if (!ei1 && !ei2) {
              Fp<F> ya = src_y<C>(bases, in_y, s1_e, from_bases);
              Fp<F> yb = src_y<C>(bases, in_y, s2_e, from_bases);
              if (fp_eq_canonical<F>(ya, yb)) de = fp_dbl<F>(ya);
            }
          }
          m = fp_mul<F>(m_e, de);
          carried = true;
        }
      }
      Fp<F> y1 = src_y<C>(bases, in_y, s1, from_bases);
      Fp<F> y2 = src_y<C>(bases, in_y, s2, from_bases);
      bool inf1 = !from_bases && fp_is_inf_marker<F>(x1);
      bool inf2 = !from_bases && fp_is_inf_marker<F>(x2);
      bool eqx = fp_eq_canonical<F>(x1, x2);
      int cls = CLS_ADD;
      Fp<F> d = fp_sub_lazy<F>(x2, x1);
      if (inf1 || inf2 || eqx) {
        d = one;
        if (inf1) cls = CLS_COPY2;
        else if (inf2) cls = CLS_COPY1;
        else if (fp_eq_canonical<F>(y1, y2)) {
          cls = CLS_DBL;
          d = fp_dbl<F>(y1);
        } else {
          cls = CLS_INF;
        }
      }
      Fp<F> invd = fp_mul<F>(inv, m);  // 1 / d_i
      inv = fp_mul<F>(inv, d);         // 1 / (d_0 ... d_{i-1})
      Fp<F> num = fp_sub_lazy<F>(y2, y1);
      if (cls == CLS_DBL) num = tangent_numerator<C>(x1, one);
      Fp<F> lam = fp_mul<F>(num, invd);
      Fp<F> x3 = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lam), x1), x2));
      Fp<F> y3 = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lam, fp_sub_lazy<F>(x1, x3)), y1));
      if (cls != CLS_ADD) {
        if (cls == CLS_COPY1) { x3 = x1; y3 = y1; }
        if (cls == CLS_COPY2) { x3 = x2; y3 = src_y<C>(bases, in_y, s2, from_bases); }
        if (cls == CLS_INF) x3 = fp_inf_marker<F>();
      }
      fp_store<F>(out_x + size_t(dsc.y) * CW, x3);
      fp_store<F>(out_y + size_t(dsc.y) * CW, y3);
    }
    return;
  }
  // decompress combined with the point additions (RV_SPLIT_APPLY: the
  // inverses only, stored over the prefix products for k_round_apply); the
  // descriptors run two steps ahead and the entries' sources one step ahead,
  // so that a step's point loads wait on no other load
  uint2 dsc_n = make_uint2(0u, 0u), dsc_ahead = make_uint2(0u, 0u);
  uint32_t r1n = 0, r2n = 0;
  if (cnt > 0) {
    dsc_n = desc[g + (cnt - 1) * T];
    r1n = entry_src(sorted, dsc_n.x, from_bases);
    r2n = entry_src(sorted, dsc_n.x + 1, from_bases);
    if (cnt > 1) dsc_ahead = desc[g + (cnt - 2) * T];
  }
  for (int i = int(cnt) - 1; i >= 0; i--) {
    round_priority(__builtin_amdgcn_readfirstlane(kmax + 2 * (kmax - 1 - uint32_t(i))), work);
    const uint2 dsc = dsc_n;
    const uint32_t s1 = r1n, s2 = r2n;
    if (i > 0) {
      dsc_n = dsc_ahead;
      r1n = entry_src(sorted, dsc_n.x, from_bases);
      r2n = entry_src(sorted, dsc_n.x + 1, from_bases);
      if (i > 1) dsc_ahead = desc[g + uint32_t(i - 2) * T];
    }
    const size_t at = chain_at<V, NL>(uint32_t(i), g, T, kmax);
    Fp<F> x1 = src_x<C>(bases, in_x, s1, from_bases);
    Fp<F> x2 = src_x<C>(bases, in_x, s2, from_bases);
    Fp<F> y1, y2;
    if constexpr ((V & RV_SPLIT_APPLY) == 0) {
      y1 = src_y<C>(bases, in_y, s1, from_bases);
      y2 = src_y<C>(bases, in_y, s2, from_bases);
    }
    bool inf1 = !from_bases && fp_is_inf_marker<F>(x1);
    bool inf2 = !from_bases && fp_is_inf_marker<F>(x2);
    bool eqx = fp_eq_canonical<F>(x1, x2);
    int cls = CLS_ADD;
    Fp<F> d = fp_sub_lazy<F>(x2, x1);
    if (inf1 || inf2 || eqx) {
      d = one;
      if constexpr ((V & RV_SPLIT_APPLY) != 0) {
        if (!inf1 && !inf2) {
          y1 = src_y<C>(bases, in_y, s1, from_bases);
          y2 = src_y<C>(bases, in_y, s2, from_bases);
        }
      }
      if (inf1) cls = CLS_COPY2;
      else if (inf2) cls = CLS_COPY1;
      else if (fp_eq_canonical<F>(y1, y2)) {
        cls = CLS_DBL;
        d = fp_dbl<F>(y1);
      } else {
        cls = CLS_INF;
      }
    }
    if constexpr ((V & RV_STORE_DENOM) != 0) d = fp_load_soa<F>(dscr + at, cs);
    Fp<F> m = fp_load_soa<F>(mscr + at, cs);
    Fp<F> invd = fp_mul<F>(inv, m);  // 1 / d_i
    inv = fp_mul<F>(inv, d);         // 1 / (d_0 ... d_{i-1})
    if constexpr ((V & RV_SPLIT_APPLY) != 0) {
      fp_store_soa<F>(mscr + at, cs, invd);
      continue;
    }
    Fp<F> num = fp_sub_lazy<F>(y2, y1);
    if (cls == CLS_DBL) num = tangent_numerator<C>(x1, one);
    Fp<F> lam = fp_mul<F>(num, invd);
    Fp<F> x3 = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lam), x1), x2));
    Fp<F> y3 = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lam, fp_sub_lazy<F>(x1, x3)), y1));
    if (cls != CLS_ADD) {
      if (cls == CLS_COPY1) { x3 = x1; y3 = y1; }
      // y2 is read again here rather than kept live across the products
      if (cls == CLS_COPY2) { x3 = x2; y3 = src_y<C>(bases, in_y, s2, from_bases); }
      if (cls == CLS_INF) x3 = fp_inf_marker<F>();
    }
    fp_store<F>(out_x + size_t(dsc.y) * CW, x3);
    fp_store<F>(out_y + size_t(dsc.y) * CW, y3);
  }
}

// The additions of a round whose inverses k_bucket_round<..., RV_SPLIT_APPLY>
// left in mscr (same round parameters, lanes and chain layout): the unfused
// form of the DCWPA step, which loads every pair's points a second time.
template <class C, int WG, int V>
__global__ void __launch_bounds__(WG) k_round_apply(const uint32_t* __restrict__ bases,
                                                    const uint32_t* __restrict__ sorted,
                                                    const uint32_t* __restrict__ in_x, const uint32_t* __restrict__ in_y,
                                                    uint32_t* __restrict__ out_x, uint32_t* __restrict__ out_y,
                                                    const uint2* __restrict__ desc, const uint4* __restrict__ prm,
                                                    int from_bases, const uint32_t* __restrict__ mscr) {
  using F = typename C::F;
  constexpr int NL = F::NL;
  constexpr int CW = F::CW;
  const uint4 pr = *prm;
  const uint32_t n_adds = pr.x, T = pr.y, kmax = pr.z;
  if (blockIdx.x * WG >= T || n_adds == 0 || pr.w == 0) return;
  const uint32_t g = blockIdx.x * WG + threadIdx.x;
  uint32_t cnt = 0;
  if (g < n_adds) cnt = min(kmax, (n_adds - 1 - g) / T + 1);
  const Fp<F> one = fp_one<F>();
  const size_t cs = chain_stride<V>(T);
  for (uint32_t i = 0; i < cnt; i++) {
    const uint2 dsc = desc[g + i * T];
    const uint32_t e1 = dsc.x;
    Fp<F> x1 = load_x<C>(bases, sorted, in_x, e1, from_bases);
    Fp<F> x2 = load_x<C>(bases, sorted, in_x, e1 + 1, from_bases);
    Fp<F> y1 = load_y<C>(bases, sorted, in_y, e1, from_bases);
    Fp<F> y2 = load_y<C>(bases, sorted, in_y, e1 + 1, from_bases);
    bool inf1 = !from_bases && fp_is_inf_marker<F>(x1);
    bool inf2 = !from_bases && fp_is_inf_marker<F>(x2);
    bool eqx = fp_eq_canonical<F>(x1, x2);
    int cls = CLS_ADD;
    if (inf1 || inf2 || eqx) {
      if (inf1) cls = CLS_COPY2;
      else if (inf2) cls = CLS_COPY1;
      else if (fp_eq_canonical<F>(y1, y2)) cls = CLS_DBL;
      else cls = CLS_INF;
    }
    const Fp<F> invd = fp_load_soa<F>(mscr + chain_at<V, NL>(i, g, T, kmax), cs);
    Fp<F> num = fp_sub_lazy<F>(y2, y1);
    if (cls == CLS_DBL) num = tangent_numerator<C>(x1, one);
    Fp<F> lam = fp_mul<F>(num, invd);
    Fp<F> x3 = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lam), x1), x2));
    Fp<F> y3 = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lam, fp_sub_lazy<F>(x1, x3)), y1));
    if (cls != CLS_ADD) {
      if (cls == CLS_COPY1) { x3 = x1; y3 = y1; }
      if (cls == CLS_COPY2) { x3 = x2; y3 = y2; }
      if (cls == CLS_INF) x3 = fp_inf_marker<F>();
    }
    fp_store<F>(out_x + size_t(dsc.y) * CW, x3);
    fp_store<F>(out_y + size_t(dsc.y) * CW, y3);
  }
}

// The rounds left out by finish_round: each bucket that still holds more than
// one partial sum (its l = ceil(n / 2^R) entries after R rounds, in the
// buffer round R - 1 wrote) adds them on its own lane in XYZZ coordinates and
// leaves the sum in that form for the reduction: X and Y where the reduction
// reads a bucket's sum (bucket_slot, in buffer A when its full round count R_b
// is odd; the infinity marker in X for a sum at infinity), ZZ and ZZZ at
// fzz[b].  A lane reads all its entries before it writes, and the entries of
// different buckets are disjoint, so the write may land on its own first
// entry.  prm_fin = (R, rounds with work).
template <class C, int WG>
__global__ void __launch_bounds__(WG) k_bucket_finish(const uint32_t* __restrict__ counts,
                                                      const uint32_t* __restrict__ offsets, uint32_t B,
                                                      uint32_t* __restrict__ ax, uint32_t* __restrict__ ay,
                                                      uint32_t* __restrict__ bx, uint32_t* __restrict__ by,
                                                      uint32_t* __restrict__ fzz, const uint4* __restrict__ prm_fin) {
  using F = typename C::F;
  constexpr int CW = F::CW;
  const uint4 pf = *prm_fin;
  const uint32_t R = pf.x;
  if (R >= pf.y) return;  // uniform: every round ran
  const uint32_t b = blockIdx.x * WG + threadIdx.x;
  const uint32_t n = b < B ? counts[b] : 0u;
  const int Rb = bucket_rounds(n);
  if (n == 0 || uint32_t(Rb) <= R) return;  // empty, or finished by the rounds
  const uint32_t l = uint32_t((uint64_t(n) + (1ull << R) - 1) >> R);
  const size_t so = size_t(bucket_slot(offsets[b], b));
  const uint32_t* sx = (R & 1) ? ax : bx;
  const uint32_t* sy = (R & 1) ? ay : by;
  XYZZ<C> S = xyzz_inf<C>();
  for (uint32_t k = 0; k < l; k++) {
    Affine<C> P;
    P.x = fp_load<F>(sx + (so + k) * CW);
    P.y = fp_load<F>(sy + (so + k) * CW);
    S = xyzz_add_affine_in<C>(S, P);
  }
  const bool inf = xyzz_is_inf<C>(S);
  uint32_t* dx = (Rb & 1) ? ax : bx;
  uint32_t* dy = (Rb & 1) ? ay : by;
  fp_store<F>(dx + so * CW, inf ? fp_inf_marker<F>() : S.X);
  fp_store<F>(dy + so * CW, S.Y);
  fp_store<F>(fzz + size_t(b) * 2 * CW, S.ZZ);
  fp_store<F>(fzz + size_t(b) * 2 * CW + CW, S.ZZZ);
}

// ---------------------------------------------------------------------------
// bucket reduction: window sum S = sum over d = 1..D of d * B_d, for every
// reduction job (one window of one MSM, D = 2^(c-1) buckets).
//
// A job is spread over Lambda lanes (a power of two, about D / 4, at most
// 8192), lane t covering the L = D / Lambda buckets d = t L + 1 .. t L + L.
// Each lane forms by running sums (from its top bucket down)
//   S_t = sum_k B_{tL+k},  T_t = sum_k k B_{tL+k}   (k = 1..L),
// so that its buckets contribute T_t + t L S_t.  A segment of sigma lanes
// (sigma = min(Lambda, 64), aligned inside one wave) then forms
//   U = sum_t S_t,  Y = sum_t T_t + L sum_t t S_t        (seg_weighted_sum).
// A job of at most 64 lanes is then done (S = Y).  A larger job has
// G = Lambda / 64 whole waves, wave g contributing Y_g + 64 L g U_g, and a
// second pass (one wave per such job) applies the same combination to the
// (U_g, Y_g) with multiplier 64 L.  Several small jobs of one segment size
// share a wave.

template <class C>
__device__ __forceinline__ XYZZ<C> shfl_down_xyzz(const XYZZ<C>& P, int d) {
  using F = typename C::F;
  XYZZ<C> r;
  r.X = shfl_down_fp<F>(P.X, d);
  r.Y = shfl_down_fp<F>(P.Y, d);
  r.ZZ = shfl_down_fp<F>(P.ZZ, d);
  r.ZZZ = shfl_down_fp<F>(P.ZZZ, d);
  return r;
}

template <class C>
__device__ __forceinline__ XYZZ<C> shfl_xor_xyzz(const XYZZ<C>& P, int m) {
  using F = typename C::F;
  XYZZ<C> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    r.X.w[i] = __shfl_xor(P.X.w[i], m, 64);
    r.Y.w[i] = __shfl_xor(P.Y.w[i], m, 64);
    r.ZZ.w[i] = __shfl_xor(P.ZZ.w[i], m, 64);
    r.ZZZ.w[i] = __shfl_xor(P.ZZZ.w[i], m, 64);
  }
  return r;
}

template <class C>
__device__ __forceinline__ XYZZ<C> shfl_xyzz(const XYZZ<C>& P, int src) {
  using F = typename C::F;
  XYZZ<C> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    r.X.w[i] = __shfl(P.X.w[i], src, 64);
    r.Y.w[i] = __shfl(P.Y.w[i], src, 64);
    r.ZZ.w[i] = __shfl(P.ZZ.w[i], src, 64);
    r.ZZZ.w[i] = __shfl(P.ZZZ.w[i], src, 64);
  }
  return r;
}

template <class C>
__device__ __forceinline__ XYZZ<C> select_xyzz(bool c, const XYZZ<C>& a, const XYZZ<C>& b) {
  using F = typename C::F;
  XYZZ<C> r;
  r.X = select_fp<F>(c, a.X, b.X);
  r.Y = select_fp<F>(c, a.Y, b.Y);
  r.ZZ = select_fp<F>(c, a.ZZ, b.ZZ);
  r.ZZZ = select_fp<F>(c, a.ZZZ, b.ZZZ);
  return r;
}

// Segments of 2^lgS lanes (aligned) inside one wave; lane t of a segment
// holds S_t, and get_T() returns its T_t.  Every lane of a segment returns
//   Y = sum_t T_t + 2^lgM sum_t t S_t,
// and put_U(U) runs in the segment's first lane with U = sum_t S_t.
// sum_t t S_t is the sum over t >= 1 of the suffix sums sum_{u >= t} S_u: an
// inclusive suffix scan, 2^lgM times each suffix sum but the first, plus
// T_t, then a butterfly sum inside the segment.  T_t is fetched only when it
// is added and U leaves as soon as it is known, so that neither occupies
// registers across the scan and the doublings.
template <class C, class GetT, class PutU>
__device__ __forceinline__ XYZZ<C> seg_weighted_sum(const XYZZ<C>& S, int lgS, int lgM, GetT get_T, PutU put_U) {
  const int lane = threadIdx.x & 63;
  const int seg = 1 << lgS;
  const int t = lane & (seg - 1);
  // one loop over all steps, so that the (inlined) addition and doubling
  // each appear once: lgS suffix-scan additions, lgM doublings, the
  // addition of T, lgS butterfly additions
  const int nsteps = lgS + lgM + 1 + lgS;
  XYZZ<C> a = S;
  for (int st = 0; st < nsteps; st++) {
    if (st == lgS && t == 0) put_U(a);  // the segment total, after the scan
    if (st >= lgS && st < lgS + lgM) {
      a = xyzz_dbl_in<C>(a);
      continue;
    }
    XYZZ<C> b;
    if (st < lgS) {
      const int off = 1 << st;
      b = select_xyzz<C>(t + off < seg, shfl_down_xyzz<C>(a, off), xyzz_inf<C>());
    } else if (st == lgS + lgM) {
      a = select_xyzz<C>(t >= 1, a, xyzz_inf<C>());
      b = get_T();
    } else {
      b = shfl_xor_xyzz<C>(a, seg >> (st - lgS - lgM));
    }
    a = xyzz_add_in<C>(a, b);
  }
  return a;
}

// XYZZ point to and from LDS, one word per (limb, thread): word k of the
// thread's point at s[k * WG + thread]
template <class C, int WG>
__device__ __forceinline__ void xyzz_to_lds(uint32_t* s, const XYZZ<C>& P) {
  constexpr int NL = C::F::NL;
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NL; i++) {
    s[(0 * NL + i) * WG + t] = P.X.w[i];
    s[(1 * NL + i) * WG + t] = P.Y.w[i];
    s[(2 * NL + i) * WG + t] = P.ZZ.w[i];
    s[(3 * NL + i) * WG + t] = P.ZZZ.w[i];
  }
}

template <class C, int WG>
__device__ __forceinline__ XYZZ<C> xyzz_from_lds(const uint32_t* s) {
  constexpr int NL = C::F::NL;
  const uint32_t t = threadIdx.x;
  XYZZ<C> P;
#pragma unroll
  for (int i = 0; i < NL; i++) {
    P.X.w[i] = s[(0 * NL + i) * WG + t];
    P.Y.w[i] = s[(1 * NL + i) * WG + t];
    P.ZZ.w[i] = s[(2 * NL + i) * WG + t];
    P.ZZZ.w[i] = s[(3 * NL + i) * WG + t];
  }
  return P;
}

template <class C>
__device__ __forceinline__ Affine<C> bucket_sum(const uint32_t* __restrict__ counts,
                                                const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ ax,
                                                const uint32_t* __restrict__ ay, const uint32_t* __restrict__ bx,
                                                const uint32_t* __restrict__ by, uint32_t b) {
  using F = typename C::F;
  const uint32_t n = counts[b];
  Affine<C> a;
  if (n == 0) {
    a.x = fp_inf_marker<F>();
    a.y = fp_zero<F>();
    return a;
  }
  const size_t e = size_t(bucket_slot(offsets[b], b)) * F::CW;
  const bool in_a = (bucket_rounds(n) & 1) != 0;
  a.x = fp_load<F>((in_a ? ax : bx) + e);
  a.y = fp_load<F>((in_a ? ay : by) + e);
  return a;
}

// The same as a point in XYZZ coordinates, for a reduction after the
// finishing pass: a bucket the pass finished (fin, and more than 2^R entries)
// takes ZZ and ZZZ from fzz[b], any other one is affine (ZZ = ZZZ = 1).
template <class C>
__device__ __forceinline__ XYZZ<C> bucket_sum_xyzz(const uint32_t* __restrict__ counts,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ ax, const uint32_t* __restrict__ ay,
                                                   const uint32_t* __restrict__ bx, const uint32_t* __restrict__ by,
                                                   const uint32_t* __restrict__ fzz, bool fin, uint32_t R,
                                                   uint32_t b) {
  using F = typename C::F;
  const uint32_t n = counts[b];
  XYZZ<C> r = xyzz_inf<C>();
  if (n == 0) return r;
  const int Rb = bucket_rounds(n);
  const size_t e = size_t(bucket_slot(offsets[b], b)) * F::CW;
  const bool in_a = (Rb & 1) != 0;
  const Fp<F> x = fp_load<F>((in_a ? ax : bx) + e);
  if (fp_is_inf_marker<F>(x)) return r;
  r.X = x;
  r.Y = fp_load<F>((in_a ? ay : by) + e);
  if (fin && uint32_t(Rb) > R) {
    r.ZZ = fp_load<F>(fzz + size_t(b) * 2 * F::CW);
    r.ZZZ = fp_load<F>(fzz + size_t(b) * 2 * F::CW + F::CW);
  } else {
    r.ZZ = r.ZZZ = fp_one<F>();
  }
  return r;
}

// lanes of a reduction job with 2^lgD buckets: log2 Lambda.  Two buckets
// per lane, at most 2^13 lanes (the level-B kernels' REDB_PARTS workgroups of
// REDB_WAVES waves), which leaves the 2^15-bucket windows of a c = 16 MSM
// four buckets per lane: for them one wave per SIMD with longer chains beat
// twice the segments
__host__ __device__ inline int reduce_lg_lanes(int lgD) {
  int l = lgD - 1;
  if (l < 0) l = 0;
  if (l > 13) l = 13;
  return l;
}

// per reduction job: first bucket, log2 D, (for jobs of more than one wave)
// the index of its first wave result, and log2 of its lanes (the host's
// choice: reduce_lg_lanes, or fewer lanes with longer chains when a batch has
// so many buckets that the reduction is bound by its total work rather than
// by one chain's latency)
struct RedJob {
  uint32_t bucket, lgD, seg_base, lgLam;
};

// per level-A wave: first job, log2 of the segment size, number of jobs in
// the wave, and the wave's index g inside its job (jobs of several waves)
struct RedWave {
  uint32_t job, lgS, njobs, g;
};

// FIN: the bucket sums may come from the finishing pass (bucket_sum_xyzz, with
// prm_fin = (R, rounds with work)); otherwise every bucket sum is affine.
template <class C, int WG, bool FIN = false>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(2, 2))) k_reduce_a(const uint32_t* __restrict__ counts,
                                                 const uint32_t* __restrict__ offsets,
                                                 const uint32_t* __restrict__ ax, const uint32_t* __restrict__ ay,
                                                 const uint32_t* __restrict__ bx, const uint32_t* __restrict__ by,
                                                 const RedJob* __restrict__ jobs, const RedWave* __restrict__ waves,
                                                 uint32_t nwaves, uint32_t* __restrict__ segU,
                                                 uint32_t* __restrict__ segY, uint32_t* __restrict__ winsum,
                                                 const uint32_t* __restrict__ fzz = nullptr,
                                                 const uint4* __restrict__ prm_fin = nullptr) {
  constexpr int XW = xyzz_words<C>();
  const uint32_t gw = (blockIdx.x * WG + threadIdx.x) >> 6;  // uniform per wave
  if (gw >= nwaves) return;
  const uint32_t lane = threadIdx.x & 63;
  const RedWave wv = waves[gw];
  const int lgS = int(wv.lgS);
  const uint32_t slot = lane >> lgS;           // job slot inside the wave
  const uint32_t t = lane & ((1u << lgS) - 1u);  // lane inside the segment
  const bool active = slot < wv.njobs;
  const RedJob jb = jobs[wv.job + (active ? slot : 0u)];
  const int lgD = int(jb.lgD);
  const int lgLam = int(jb.lgLam);
  const int lgL = lgD - lgLam;
  const uint32_t L = 1u << lgL;
  const uint32_t base = ((wv.g << 6) + t) * L;  // buckets base + 1 .. base + L of the job
  __shared__ uint32_t s_T[4 * C::F::NL * WG];
  XYZZ<C> S = xyzz_inf<C>(), T = xyzz_inf<C>();
  if (active) {
    if constexpr (FIN) {
      const uint4 pf = *prm_fin;
      const bool fin = pf.x < pf.y;
      for (int k = int(L); k >= 1; k--) {
        const XYZZ<C> Bz =
            bucket_sum_xyzz<C>(counts, offsets, ax, ay, bx, by, fzz, fin, pf.x, jb.bucket + base + uint32_t(k) - 1);
        S = xyzz_add_in<C>(S, Bz);
        T = xyzz_add_in<C>(T, S);
      }
    } else {
      for (int k = int(L); k >= 1; k--) {
        Affine<C> B = bucket_sum<C>(counts, offsets, ax, ay, bx, by, jb.bucket + base + uint32_t(k) - 1);
        S = xyzz_add_affine_in<C>(S, B);
        T = xyzz_add_in<C>(T, S);
      }
    }
  }
  // T waits in LDS (read back by the same thread) while the scan and the doublings run
  xyzz_to_lds<C, WG>(s_T, T);
  const bool big = lgLam > 6;
  const XYZZ<C> Y = seg_weighted_sum<C>(
      S, lgS, lgL, [&]() { return xyzz_from_lds<C, WG>(s_T); },
      [&](const XYZZ<C>& U) {
        if (active && big) xyzz_store<C>(segU + size_t(jb.seg_base + wv.g) * XW, U);
      });
  if (active && t == 0) {
    if (!big) xyzz_store<C>(winsum + size_t(wv.job + slot) * XW, Y);
    else xyzz_store<C>(segY + size_t(jb.seg_base + wv.g) * XW, Y);
  }
}

// Level B, for jobs of G = Lambda / 64 > 1 level-A waves (big_jobs lists
// them), with the lane-parallel field: the job's result is
//   sum_g Y_g + 2^lgM sum_g g U_g,  lgM = 6 + lgL  (g < G),
// from the level-A sums (U_g, Y_g).  Workgroup q of the job takes the
// segments g = q nw + w, one per wave w (nw = min(G, REDB_WAVES) waves, the
// point replicated over the wave's four rows), and exchanges points between
// waves through LDS:
//   suffix scan over the waves: a_w = sum_{u >= w} U_{q nw + u};
//   wave w >= 1: 2^lgM a_w + Y_g; wave 0: 2^(lgM + lg nw) q a_0 + Y_g (the
//   offset q nw of the workgroup's segments, applied to their total);
//   butterfly sum over the waves.
// Each workgroup leaves its part in segY at its first segment; k_reduce_c
// adds the G / nw (at most REDB_PARTS) parts of a job.  The chains are bound
// by latency: four waves per workgroup put the 2^13 lanes of the largest
// jobs' level-A waves on every compute unit at one wave per SIMD, where
// sixteen would leave three quarters of the units idle and four waves on
// each SIMD of the others.
constexpr int REDB_LG_WAVES = 2;
constexpr int REDB_WAVES = 1 << REDB_LG_WAVES;
constexpr int REDB_LG_PARTS = 5;
constexpr int REDB_PARTS = 1 << REDB_LG_PARTS;
// k_reduce_c: one workgroup per job, each wave adding parts w, w + REDC_WAVES, ...
constexpr int REDC_LG_WAVES = REDB_LG_PARTS < 4 ? REDB_LG_PARTS : 4;
constexpr int REDC_WAVES = 1 << REDC_LG_WAVES;
static_assert(6 + REDB_LG_WAVES + REDB_LG_PARTS == 13, "level B covers the 2^13 lanes of the largest job");

template <class C>
__global__ void __launch_bounds__(64 * REDB_WAVES) k_reduce_b(const uint32_t* __restrict__ segU,
                                                             uint32_t* __restrict__ segY,
                                                             const RedJob* __restrict__ jobs,
                                                             const uint32_t* __restrict__ big_jobs) {
  using F = typename C::F;
  constexpr int XW = xyzz_words<C>();
  __shared__ uint32_t s_pt[REDB_WAVES][4][16];
  __shared__ uint32_t s_inf[REDB_WAVES];
  const uint32_t j = big_jobs[blockIdx.x / REDB_PARTS];
  const uint32_t q = blockIdx.x % REDB_PARTS;
  const RedJob jb = jobs[j];
  const int lgLam = int(jb.lgLam);
  const int lgG = lgLam - 6;
  const int lgL = int(jb.lgD) - lgLam;
  const int lgM = 6 + lgL;
  const int lgnw = lgG < REDB_LG_WAVES ? lgG : REDB_LG_WAVES;
  const uint32_t nw = 1u << lgnw;
  const uint32_t Q = 1u << (lgG - lgnw);
  if (q >= Q) return;  // uniform per workgroup
  const uint32_t w = threadIdx.x >> 6;
  const bool live = w < nw;
  const LpK<F> k = lp_consts<F>();
  const size_t g = size_t(jb.seg_base) + q * nw + w;
  LpPoint<C> a, T;
  a.X = a.Y = a.ZZ = a.ZZZ = 0;
  a.inf = true;
  T = a;
  if (live) {
    a = lp_point_load<C>(segU + g * XW, k);
    T = lp_point_load<C>(segY + g * XW, k);
  }
  // every wave (live or not) takes part in each exchange
  auto exchange = [&](const LpPoint<C>& mine, uint32_t partner, bool valid) {
    if ((threadIdx.x & 63u) < 16u) {
      const uint32_t l = threadIdx.x & 15u;
      s_pt[w][0][l] = mine.X;
      s_pt[w][1][l] = mine.Y;
      s_pt[w][2][l] = mine.ZZ;
      s_pt[w][3][l] = mine.ZZZ;
      if (l == 0) s_inf[w] = mine.inf ? 1u : 0u;
    }
    __syncthreads();
    LpPoint<C> o;
    o.X = o.Y = o.ZZ = o.ZZZ = 0;
    o.inf = true;
    if (valid) {
      const uint32_t l = lane16();
      o.X = s_pt[partner][0][l];
      o.Y = s_pt[partner][1][l];
      o.ZZ = s_pt[partner][2][l];
      o.ZZZ = s_pt[partner][3][l];
      o.inf = s_inf[partner] != 0;
    }
    __syncthreads();
    return o;
  };
  for (int st = 0; st < lgnw; st++) {
    const uint32_t o = 1u << st;
    const LpPoint<C> b = exchange(a, w + o, live && w + o < nw);
    if (live) a = lp_add_pts<C>(a, b, k);
  }
  if (live) {
    if (w > 0) {
      for (int i = 0; i < lgM; i++) a = lp_dbl<C>(a, k);
    } else {
      for (int i = 0; i < lgM + lgnw; i++) a = lp_dbl<C>(a, k);
      // a <- q a (q < REDB_PARTS), double-and-add from the top bit
      const LpPoint<C> base = a;
      a.inf = true;
      for (int bit = REDB_LG_PARTS - 1; bit >= 0; bit--) {
        a = lp_dbl<C>(a, k);
        if ((q >> bit) & 1u) a = lp_add_pts<C>(a, base, k);
      }
    }
    a = lp_add_pts<C>(a, T, k);
  }
  for (int st = lgnw - 1; st >= 0; st--) {
    const uint32_t partner = w ^ (1u << st);
    const LpPoint<C> b = exchange(a, partner, live);
    if (live) a = lp_add_pts<C>(a, b, k);
  }
  if (w == 0) lp_point_store<C>(segY + (size_t(jb.seg_base) + q * nw) * XW, a, k);
}

// the parts of each big job: winsum_j = sum over workgroups q of
// segY[seg_base + q nw]; wave w adds the parts w, w + V, ... (V = min(Q,
// REDC_WAVES) waves), then a tree through LDS sums the waves into wave 0:
// at level st the waves w = 0 mod 2^(st+1) add wave w + 2^st, so that the
// waves that still add share their SIMDs with fewer and fewer others
template <class C>
__global__ void __launch_bounds__(64 * REDC_WAVES) k_reduce_c(const uint32_t* __restrict__ segY,
                                                              const RedJob* __restrict__ jobs,
                                                              const uint32_t* __restrict__ big_jobs,
                                                              uint32_t* __restrict__ winsum) {
  using F = typename C::F;
  constexpr int XW = xyzz_words<C>();
  __shared__ uint32_t s_pt[REDC_WAVES][4][16];
  __shared__ uint32_t s_inf[REDC_WAVES];
  const uint32_t j = big_jobs[blockIdx.x];
  const RedJob jb = jobs[j];
  const int lgG = int(jb.lgLam) - 6;
  const int lgnw = lgG < REDB_LG_WAVES ? lgG : REDB_LG_WAVES;
  const uint32_t nw = 1u << lgnw;
  const int lgQ = lgG - lgnw;
  const uint32_t Q = 1u << lgQ;
  const int lgV = lgQ < REDC_LG_WAVES ? lgQ : REDC_LG_WAVES;
  const uint32_t V = 1u << lgV;
  const uint32_t w = threadIdx.x >> 6;
  const bool live = w < V;
  const LpK<F> k = lp_consts<F>();
  LpPoint<C> a;
  a.X = a.Y = a.ZZ = a.ZZZ = 0;
  a.inf = true;
  if (live) {
    for (uint32_t part = w; part < Q; part += V)
      a = lp_add_pts<C>(a, lp_point_load<C>(segY + (size_t(jb.seg_base) + part * nw) * XW, k), k);
  }
  for (int st = 0; st < lgV; st++) {
    const uint32_t o = 1u << st;
    const bool sender = (w & (2u * o - 1u)) == o;
    const bool receiver = live && (w & (2u * o - 1u)) == 0u;
    if (sender && (threadIdx.x & 63u) < 16u) {
      const uint32_t l = threadIdx.x & 15u;
      s_pt[w][0][l] = a.X;
      s_pt[w][1][l] = a.Y;
      s_pt[w][2][l] = a.ZZ;
      s_pt[w][3][l] = a.ZZZ;
      if (l == 0) s_inf[w] = a.inf ? 1u : 0u;
    }
    __syncthreads();
    LpPoint<C> b;
    b.X = b.Y = b.ZZ = b.ZZZ = 0;
    b.inf = true;
    if (receiver) {
      const uint32_t l = lane16();
      b.X = s_pt[w + o][0][l];
      b.Y = s_pt[w + o][1][l];
      b.ZZ = s_pt[w + o][2][l];
      b.ZZZ = s_pt[w + o][3][l];
      b.inf = s_inf[w + o] != 0;
    }
    __syncthreads();
    if (receiver) a = lp_add_pts<C>(a, b, k);
  }
  if (w == 0) lp_point_store<C>(winsum + size_t(j) * XW, a, k);
}

// Output of one MSM: canonical affine words, or the infinity flag.  Nothing
// is written when an input error was flagged (the call then fails).
template <class C>
__device__ __forceinline__ void write_result(const XYZZ<C>& R, uint32_t* __restrict__ out_xy,
                                             uint8_t* __restrict__ out_inf, bool leader) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  bool inf = xyzz_is_inf<C>(R);
  Affine<C> a = xyzz_to_affine_uniform<C>(R);
  uint32_t xw[N32], yw[N32];
  fp_to_words<F>(fp_from_mont<F>(a.x), xw);
  fp_to_words<F>(fp_from_mont<F>(a.y), yw);
  if (inf) {
#pragma unroll
    for (int k = 0; k < N32; k++) xw[k] = yw[k] = 0;
  }
  if (leader) {
    words_store<F>(out_xy, xw);
    words_store<F>(out_xy + N32, yw);
    out_inf[0] = inf ? 1 : 0;
  }
}

// window combination (Horner over windows, c doublings between windows) of
// MSM blockIdx.x on one wave, the products of each formula spread over lanes
template <class C>
__global__ void __launch_bounds__(64) k_combine(const uint32_t* __restrict__ winsum, const MsmDesc* __restrict__ msms,
                                                const uint32_t* __restrict__ err, uint32_t* __restrict__ out_xy,
                                                uint8_t* __restrict__ out_inf) {
  using F = typename C::F;
  constexpr int XW = xyzz_words<C>();
  if (*err) return;
  const MsmDesc md = msms[blockIdx.x];
  const LpK<F> k = lp_consts<F>();
  LpPoint<C> R;
  R.X = R.Y = R.ZZ = R.ZZZ = 0;
  R.inf = true;
  if (md.n) {
    R = lp_point_load<C>(winsum + size_t(md.job_base + md.W - 1) * XW, k);
    // the next window's sum is loaded one window ahead, while the doublings run
    constexpr int CW = F::CW;
    uint32_t nx = 0, ny = 0, nzz = 0, nzzz = 0;
    auto fetch = [&](int w) {
      const uint32_t* p = winsum + size_t(md.job_base + uint32_t(w)) * XW;
      nx = lp_load<F>(p);
      ny = lp_load<F>(p + CW);
      nzz = lp_load<F>(p + 2 * CW);
      nzzz = lp_load<F>(p + 3 * CW);
    };
    if (md.W >= 2) fetch(int(md.W) - 2);
    for (int w = int(md.W) - 2; w >= 0; w--) {
      LpPoint<C> S;
      S.X = nx;
      S.Y = ny;
      S.ZZ = nzz;
      S.ZZZ = nzzz;
      if (w > 0) fetch(w - 1);
      for (int i = 0; i < int(md.c); i++) R = lp_dbl<C>(R, k);
      S.inf = lp_is_zero<F>(S.ZZ, k);
      R = lp_add_pts<C>(R, S, k);
    }
  }
  write_result<C>(lp_point_to_xyzz<C>(R, k), out_xy + size_t(blockIdx.x) * 2 * F::N32, out_inf + blockIdx.x,
                  threadIdx.x == 0);
}

// the same with one lane per MSM, for batches of many MSMs
template <class C>
__global__ void __launch_bounds__(64) k_combine_lanes(const uint32_t* __restrict__ winsum,
                                                      const MsmDesc* __restrict__ msms, uint32_t m,
                                                      const uint32_t* __restrict__ err,
                                                      uint32_t* __restrict__ out_xy, uint8_t* __restrict__ out_inf) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  constexpr int XW = xyzz_words<C>();
  if (*err) return;
  const uint32_t i = blockIdx.x * 64 + threadIdx.x;
  if (i >= m) return;
  const MsmDesc md = msms[i];
  XYZZ<C> R = xyzz_inf<C>();
  if (md.n) {
    R = xyzz_load<C>(winsum + size_t(md.job_base + md.W - 1) * XW);
    for (int w = int(md.W) - 2; w >= 0; w--) {
      for (int k = 0; k < int(md.c); k++) R = xyzz_dbl<C>(R);
      R = xyzz_add<C>(R, xyzz_load<C>(winsum + size_t(md.job_base + w) * XW));
    }
  }
  bool inf = xyzz_is_inf<C>(R);
  Affine<C> a;
  if (inf) {
    a.x = fp_zero<F>();
    a.y = fp_zero<F>();
  } else {
    // per-lane normalisation: ZZ ZZZ inverted by the lane itself
    uint32_t w[N32], iw[N32];
    fp_to_words<F>(fp_canonical<F>(fp_mul<F>(R.ZZ, R.ZZZ)), w);
    inverse_words<F, 2>(w, iw);
    constexpr Words<F::NL> r3 = F::R3;
    Fp<F> t = fp_mul<F>(fp_from_words<F>(iw), fp_from<F>(r3));
    a.x = fp_from_mont<F>(fp_mul<F>(R.X, fp_mul<F>(t, R.ZZZ)));
    a.y = fp_from_mont<F>(fp_mul<F>(R.Y, fp_mul<F>(t, R.ZZ)));
  }
  uint32_t xw[N32], yw[N32];
  fp_to_words<F>(a.x, xw);
  fp_to_words<F>(a.y, yw);
  words_store<F>(out_xy + size_t(i) * 2 * N32, xw);
  words_store<F>(out_xy + size_t(i) * 2 * N32 + N32, yw);
  out_inf[i] = inf ? 1 : 0;
}

template <class C>
__global__ void k_write_inf(uint32_t* __restrict__ out_xy, uint8_t* __restrict__ out_inf, uint32_t m) {
  using F = typename C::F;
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  for (int k = 0; k < 2 * F::N32; k++) out_xy[size_t(i) * 2 * F::N32 + k] = 0;
  out_inf[i] = 1;
}

// ---------------------------------------------------------------------------
// fixed-base scalar multiplication k_i G (Algorithm 1 per lane in XYZZ, the
// doublings of G computed along), normalised by one GAS batch inversion

// The affine form of Q written at out as x then y (N32 words each), plain or
// (out_mont) times R' = 2^(32 N32); O (inf) as zeros.  One GAS inversion of
// ZZ ZZZ for the workgroup, so every lane must call it; only active lanes
// write.
template <class C, int WG>
__device__ __forceinline__ void store_xyzz_affine(const XYZZ<C>& Q, bool inf, bool active, uint32_t* __restrict__ out,
                                                  int out_mont, Fp<typename C::F>* s_tot, Fp<typename C::F>* s_inv) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  Fp<F> z = inf ? fp_one<F>() : fp_mul<F>(Q.ZZ, Q.ZZZ);
  Fp<F> t = wg_batch_inverse<F, WG>(z, s_tot, s_inv);
  Fp<F> x = fp_mul<F>(Q.X, fp_mul<F>(t, Q.ZZZ));
  Fp<F> y = fp_mul<F>(Q.Y, fp_mul<F>(t, Q.ZZ));
  constexpr Words<F::NL> rout = F::ROUT;
  Fp<F> k1 = fp_zero<F>();
  k1.w[0] = 1;
  // Montgomery product with 1 leaves x; with R' = 2^(32 N32) leaves x R'
  Fp<F> k = out_mont ? fp_from<F>(rout) : k1;
  x = fp_canonical<F>(fp_mul<F>(x, k));
  y = fp_canonical<F>(fp_mul<F>(y, k));
  uint32_t xw[N32], yw[N32];
  fp_to_words<F>(x, xw);
  fp_to_words<F>(y, yw);
  if (inf) {
#pragma unroll
    for (int j = 0; j < N32; j++) xw[j] = yw[j] = 0;
  }
  if (active) {
    words_store<F>(out, xw);
    words_store<F>(out + N32, yw);
  }
}

template <class C, int WG>
__global__ void __launch_bounds__(WG) k_fixed_base(const uint32_t* __restrict__ ks, size_t n,
                                                   uint32_t* __restrict__ out, int out_mont) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  bool active = i < n;
  uint32_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (active) load_scalar(ks + 8 * i, s);
  constexpr Words<F::NL> gx = C::GX, gy = C::GY;
  XYZZ<C> P;
  P.X = fp_from<F>(gx);
  P.Y = fp_from<F>(gy);
  P.ZZ = fp_one<F>();
  P.ZZZ = fp_one<F>();
  XYZZ<C> Q = xyzz_inf<C>();
  for (int b = 0; b < 256; b++) {
    if ((s[b >> 5] >> (b & 31)) & 1u) Q = xyzz_add<C>(Q, P);
    P = xyzz_dbl<C>(P);
  }
  store_xyzz_affine<C, WG>(Q, xyzz_is_inf<C>(Q), active, out + i * 2 * N32, out_mont, s_tot, s_inv);
}

// ---------------------------------------------------------------------------
// elementwise test kernels (exported only for parity tests); their I/O is
// canonical u64 limbs

template <class C>
__device__ __forceinline__ Fp<typename C::F> load_io_mont(const uint32_t* __restrict__ p) {
  using F = typename C::F;
  uint32_t w[F::N32];
  words_load<F>(p, w);
  return fp_to_mont<F>(fp_from_words<F>(w));
}

template <class C>
__device__ __forceinline__ void store_io_plain(uint32_t* __restrict__ p, const Fp<typename C::F>& a) {
  using F = typename C::F;
  uint32_t w[F::N32];
  fp_to_words<F>(fp_from_mont<F>(a), w);
  words_store<F>(p, w);
}

template <class C>
__global__ void k_test_fp_mul(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                              uint32_t* __restrict__ r, size_t n) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Fp<F> x = load_io_mont<C>(a + i * N32);
  if (a == b) {  // the same operand array: the squaring routine
    store_io_plain<C>(r + i * N32, fp_sqr<F>(x));
    return;
  }
  Fp<F> y = load_io_mont<C>(b + i * N32);
  store_io_plain<C>(r + i * N32, fp_mul<F>(x, y));
}

// the lane-parallel field (four elements per wave, one per 16-lane row):
// op 0: a b, op 1: a - b, op 2: (3a)(a + b) - 2b, and the differences of the
// point formulas on product outputs (the widest operands lp_sub takes):
// op 3: 3(ab) - a^2, op 4: (3 b^2 + ab) - a^2, op 5: a^2 - (ab + 2 b^2);
// a Y coordinate left unreduced (lp_sub_y): op 6: (2(ab - a^2))^2 (the
// doubling's first product), op 7: ab - a^2 reduced as a point store does
template <class C>
__global__ void __launch_bounds__(64) k_test_lane_field(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                                                        uint32_t* __restrict__ r, size_t n, int op) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  const LpK<F> k = lp_consts<F>();
  const size_t e = size_t(blockIdx.x) * 4 + row4();
  const bool live = e < n;
  Fp<F> x = fp_zero<F>(), y = fp_zero<F>();
  if (live) {
    x = load_io_mont<C>(a + e * N32);
    y = load_io_mont<C>(b + e * N32);
  }
  const uint32_t j = lane16();
  uint32_t xa = 0, yb = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    xa = j == uint32_t(i) ? x.w[i] : xa;
    yb = j == uint32_t(i) ? y.w[i] : yb;
  }
  uint32_t z;
  if (op == 0) {
    z = lp_mul<F>(xa, yb, k);
  } else if (op == 1) {
    z = lp_sub<F>(xa, yb, k);
  } else if (op == 2) {
    const uint32_t m = lp_carry32<F>(xa + xa + xa);
    z = lp_sub<F>(lp_mul<F>(m, xa + yb, k), yb + yb, k);
  } else {
    const uint32_t ab = lp_mul<F>(xa, yb, k), aa = lp_mul<F>(xa, xa, k), bb = lp_mul<F>(yb, yb, k);
    const uint32_t y = lp_sub_y<F>(ab, aa, k);
    if (op == 3) z = lp_sub<F>(ab + ab + ab, aa, k);
    else if (op == 4) z = lp_sub<F>(lp_carry32<F>(bb + bb + bb + ab), aa, k);
    else if (op == 5) z = lp_sub<F>(aa, lp_carry32<F>(ab + bb + bb), k);
    else if (op == 6) z = lp_mul<F>(y + y, y + y, k);
    else z = lp_reduce<F>(y, k);
  }
  z = lp_canonical<F>(z, k);
  Fp<F> o;
#pragma unroll
  for (int i = 0; i < F::NL; i++) o.w[i] = uint32_t(__shfl(int(z), int(threadIdx.x & 48u) + i, 64));
  if (live && j == 0) store_io_plain<C>(r + e * N32, o);
}

template <class C, int WG>
__global__ void __launch_bounds__(WG) k_test_fp_inv(const uint32_t* __restrict__ a, uint32_t* __restrict__ r,
                                                    size_t n) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  bool active = i < n;
  Fp<F> x = active ? load_io_mont<C>(a + i * N32) : fp_one<F>();
  bool zero = fp_is_zero<F>(x);
  if (zero) x = fp_one<F>();
  Fp<F> y = wg_batch_inverse<F, WG>(x, s_tot, s_inv);
  if (active) store_io_plain<C>(r + i * N32, zero ? fp_zero<F>() : y);
}

// canonical u64-limb points p_i, q_i -> input entries (2i, 2i+1) of the x
// and y planes, working form; pair i adds into output entry i
template <class C>
__global__ void k_test_pairs_in(const uint32_t* __restrict__ p, const uint32_t* __restrict__ q,
                                uint32_t* __restrict__ xs, uint32_t* __restrict__ ys, uint2* __restrict__ desc,
                                size_t n) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 2; k++) {
    const uint32_t* src = (k ? q : p) + i * 2 * N32;
    uint32_t xw[N32], yw[N32];
    words_load<F>(src, xw);
    words_load<F>(src + N32, yw);
    uint32_t any = 0;
    for (int j = 0; j < N32; j++) any |= xw[j] | yw[j];
    Affine<C> P;
    if (any == 0) {
      P.x = fp_inf_marker<F>();
      P.y = fp_zero<F>();
    } else {
      P.x = fp_canonical<F>(fp_to_mont<F>(fp_from_words<F>(xw)));
      P.y = fp_canonical<F>(fp_to_mont<F>(fp_from_words<F>(yw)));
    }
    fp_store<F>(xs + (2 * i + k) * F::CW, P.x);
    fp_store<F>(ys + (2 * i + k) * F::CW, P.y);
  }
  desc[i] = make_uint2(uint32_t(2 * i), uint32_t(i));
}

template <class C>
__global__ void k_test_pairs_out(const uint32_t* __restrict__ xs, const uint32_t* __restrict__ ys,
                                 uint32_t* __restrict__ r, size_t n) {
  using F = typename C::F;
  constexpr int N32 = F::N32;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Affine<C> P;
  P.x = fp_load<F>(xs + i * F::CW);
  P.y = fp_load<F>(ys + i * F::CW);
  uint32_t xw[N32], yw[N32];
  if (fp_is_inf_marker<F>(P.x)) {
    for (int j = 0; j < N32; j++) xw[j] = yw[j] = 0;
  } else {
    fp_to_words<F>(fp_from_mont<F>(P.x), xw);
    fp_to_words<F>(fp_from_mont<F>(P.y), yw);
  }
  words_store<F>(r + i * 2 * N32, xw);
  words_store<F>(r + i * 2 * N32 + N32, yw);
}

}  // namespace eccmi
