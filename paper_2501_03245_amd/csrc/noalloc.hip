// Allocation-free ECDSA verification (ecc_verify_batch_noalloc).
//
// The per-lane verification of ecc_verify_batch needs device memory beyond
// its inputs and outputs: the comb table of the generator (d 2^(8 j) G for
// j < 32, d < 256, per signing curve) and one table of d Q (d = 1..15) per
// request.  Here both live in one file-scope device array, `scratch`, so
// that the call makes no hipMalloc, hipFree or other allocating call: for
// callers that must not allocate (code under stream capture, tight serving
// loops).  Each GPU holds its own copy of the array for the life of the
// process, and every call on that GPU shares it, so calls that overlap on
// one GPU race.
//
// Layout of `scratch` (32-bit words):
//   [comb of secp256r1 | comb of SM2 | staging of the comb build | tables of d Q]
// The combs are built once per device, at that device's first call, by the
// same double-and-add and ingest kernels the context path uses; the staging
// area holds the comb scalars, the boundary-form points and an error word.
#include "host.h"

#include <mutex>

namespace {

constexpr size_t NOALLOC_MAX_REQUESTS = 8192;
constexpr size_t COMB_N = size_t(VCOMB_WINDOWS) * VCOMB_ENTRIES;

template <class C>
constexpr size_t comb_words() {
  return COMB_N * size_t(affine_words<C>());
}

template <class C>
constexpr size_t table_words() {
  return NOALLOC_MAX_REQUESTS * size_t(VT_N) * size_t(vt_slot<typename C::F>());
}

constexpr size_t round_up64(size_t w) { return (w + 63) / 64 * 64; }

constexpr size_t OFF_COMB_P256 = 0;
constexpr size_t OFF_COMB_SM2 = round_up64(OFF_COMB_P256 + comb_words<P256>());
constexpr size_t OFF_BUILD = round_up64(OFF_COMB_SM2 + comb_words<SM2>());
// scalars (8 words each), boundary points (2 N32 words each, 8 + 8 for both
// 256-bit curves), one error word
constexpr size_t BUILD_WORDS = COMB_N * 8 + COMB_N * 16 + 64;
constexpr size_t OFF_TABLES = round_up64(OFF_BUILD + BUILD_WORDS);
constexpr size_t TABLE_WORDS = table_words<P256>() > table_words<SM2>() ? table_words<P256>() : table_words<SM2>();
constexpr size_t SCRATCH_WORDS = OFF_TABLES + TABLE_WORDS;

static_assert(2 * P256::F::N32 == 16 && 2 * SM2::F::N32 == 16, "staging sized for 256-bit boundary points");

}  // namespace

// The array itself.  In host code its name is only a stand-in for the
// symbol: the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) uint32_t scratch[SCRATCH_WORDS];

namespace {

// comb scalar of entry e = 256 j + d: (d ? d : 1) 2^(8 j), as 8 words
static __global__ void k_comb_scalars(uint32_t* __restrict__ ks) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= COMB_N) return;
  const uint32_t j = uint32_t(e / VCOMB_ENTRIES), d = uint32_t(e % VCOMB_ENTRIES);
  const uint32_t v = d ? d : 1u;
  const uint32_t bit = 8 * j;
#pragma unroll
  for (int w = 0; w < 8; w++) ks[e * 8 + w] = (uint32_t(w) == bit / 32) ? (v << (bit % 32)) : 0u;
}

struct DeviceScratch {
  uint32_t* base = nullptr;  // device address of `scratch` on this device
  bool ready = false;        // both combs built
};

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
DeviceScratch g_dev[MAX_DEVICES];

template <class C>
hipError_t build_comb(uint32_t* base, size_t comb_off, hipStream_t st) {
  uint32_t* ks = base + OFF_BUILD;
  uint32_t* pts = ks + COMB_N * 8;
  uint32_t* err = pts + COMB_N * 16;
  const unsigned blocks = unsigned(ceil_div(COMB_N, 256));
  k_comb_scalars<<<blocks, 256, 0, st>>>(ks);
  k_fill_u32<<<1, 64, 0, st>>>(err, 1, 0u);
  k_fixed_base<C, 256><<<blocks, 256, 0, st>>>(ks, COMB_N, pts, 0);
  k_ingest_points<C><<<blocks, 256, 0, st>>>(pts, base + comb_off, nullptr, COMB_N, 0, 0, err);
  return hipGetLastError();
}

// set-up on the current device: the array's address, then both combs
ecc_status device_scratch(hipStream_t st, uint32_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return ECC_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceScratch& s = g_dev[dev];
  if (!s.base) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ECC_ERR_DEVICE;
    s.base = static_cast<uint32_t*>(p);
  }
  if (!s.ready) {
    if (build_comb<P256>(s.base, OFF_COMB_P256, st) != hipSuccess) return ECC_ERR_DEVICE;
    if (build_comb<SM2>(s.base, OFF_COMB_SM2, st) != hipSuccess) return ECC_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return ECC_ERR_DEVICE;
    s.ready = true;
  }
  *out = s.base;
  return ECC_OK;
}

template <class C>
ecc_status verify_noalloc(uint32_t* base, size_t comb_off, const uint8_t* hashes, const uint64_t* pubkeys,
                          const uint64_t* sigs, size_t m, uint8_t* valid, hipStream_t st) {
  static_assert(table_words<C>() <= TABLE_WORDS, "tables exceed the scratch array");
  k_verify_xyzz<C, VERIFY_LANE_WG><<<unsigned(ceil_div(m, VERIFY_LANE_WG)), VERIFY_LANE_WG, 0, st>>>(
      hashes, reinterpret_cast<const uint32_t*>(pubkeys), reinterpret_cast<const uint32_t*>(sigs), m,
      base + comb_off, base + OFF_TABLES, valid);
  if (hipGetLastError() != hipSuccess) return ECC_ERR_DEVICE;
  return hipStreamSynchronize(st) == hipSuccess ? ECC_OK : ECC_ERR_DEVICE;
}

}  // namespace

extern "C" {

size_t ecc_verify_batch_noalloc_max(void) { return NOALLOC_MAX_REQUESTS; }

ecc_status ecc_verify_batch_noalloc(ecc_curve curve, const uint8_t* hashes, const uint64_t* pubkeys,
                                    const uint64_t* sigs, size_t m, uint8_t* valid, void* stream) {
  if (m == 0) return ECC_OK;
  if (!hashes || !pubkeys || !sigs || !valid) return ECC_ERR_ARG;
  if (m > NOALLOC_MAX_REQUESTS) return ECC_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (curve) {
    case ECC_SECP256R1:
    case ECC_SM2: {
      uint32_t* base = nullptr;
      ECC_TRY(device_scratch(st, &base));
      if (curve == ECC_SECP256R1)
        return verify_noalloc<P256>(base, OFF_COMB_P256, hashes, pubkeys, sigs, m, valid, st);
      return verify_noalloc<SM2>(base, OFF_COMB_SM2, hashes, pubkeys, sigs, m, valid, st);
    }
    case ECC_BN254_G1:
    case ECC_BLS12_381_G1:
      // no ECDSA keys live on these curves: every request is invalid
      k_fill_u8<<<unsigned(ceil_div(m, 256)), 256, 0, st>>>(valid, m, 0);
      if (hipGetLastError() != hipSuccess) return ECC_ERR_DEVICE;
      return hipStreamSynchronize(st) == hipSuccess ? ECC_OK : ECC_ERR_DEVICE;
    default: return ECC_ERR_ARG;
  }
}

}  // extern "C"
