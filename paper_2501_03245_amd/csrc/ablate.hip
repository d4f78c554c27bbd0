// Design variants of the bucket-round kernel on BLS12-381 (RV_* in
// kernels.h), launched in place of the library's own round when a context
// asks for one (ecc_ctx_set_round_variant): the ablations of the choices of
// Sections 3.2 and 3.3.  Kept in a translation unit of its own so that the
// extra instantiations build in parallel with the rest.
#include "host.h"

namespace {

template <int V>
hipError_t launch_v(uint32_t blocks, hipStream_t st, const uint32_t* bases, const uint32_t* sorted,
                    const uint32_t* in_x, const uint32_t* in_y, uint32_t* out_x, uint32_t* out_y, const uint2* desc,
                    const uint4* prm, int from_bases, uint32_t* mscr, const uint2* tails, const uint32_t* n_tails,
                    uint32_t* dscr) {
  k_bucket_round<BLS12_381, ROUND_WG, ROUND_OCC, V><<<blocks, ROUND_WG, 0, st>>>(
      bases, sorted, in_x, in_y, out_x, out_y, desc, prm, from_bases, mscr, tails, n_tails, dscr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr ((V & RV_SPLIT_APPLY) != 0) {
    k_round_apply<BLS12_381, ROUND_WG, V><<<blocks, ROUND_WG, 0, st>>>(bases, sorted, in_x, in_y, out_x, out_y,
                                                                       desc, prm, from_bases, mscr);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

hipError_t launch_round_variant_bls(int variant, uint32_t blocks, hipStream_t st, const uint32_t* bases,
                                    const uint32_t* sorted, const uint32_t* in_x, const uint32_t* in_y,
                                    uint32_t* out_x, uint32_t* out_y, const uint2* desc, const uint4* prm,
                                    int from_bases, uint32_t* mscr, const uint2* tails, const uint32_t* n_tails,
                                    uint32_t* dscr) {
#define ECC_RV(V)                                                                                                 \
  case V:                                                                                                       \
    return launch_v<V>(blocks, st, bases, sorted, in_x, in_y, out_x, out_y, desc, prm, from_bases, mscr, tails, \
                       n_tails, dscr);
  switch (variant) {
    ECC_RV(RV_STORE_DENOM)
    ECC_RV(RV_AOS_CHAIN)
    ECC_RV(RV_STORE_DENOM | RV_AOS_CHAIN)
    ECC_RV(RV_SPLIT_APPLY)
    ECC_RV(RV_STORE_DENOM | RV_AOS_CHAIN | RV_SPLIT_APPLY)
    ECC_RV(RV_LANE_INV)
    ECC_RV(RV_HALF_PREFIX)
    default: return hipErrorInvalidValue;
  }
#undef ECC_RV
}
