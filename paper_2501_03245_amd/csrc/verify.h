// Batched ECDSA verification and signing on secp256r1 and SM2, and batched
// unknown-point multiplication on every curve.
//
// Per request: valid iff 1 <= r, s < n, Q is a curve point other than O, and
// with w = s^-1, u1 = e w, u2 = r w (mod n), R = u1 G + u2 Q is not O and
// R.x mod n = r.  The paper counts a verification as one fixed-point and one
// unknown-point multiplication (Section 5.2).  Two kernels compute it: the
// per-lane XYZZ form at the end of this file, and first the paper's batched
// affine form, where both multiplications run in one loop over the scalar
// bits from the least significant end, as in its batch PMUL (Section 3.4,
// Algorithm 3):
//
//   step j:  A1 <- A1 + 2^j G   if bit j of u1     (fixed point, table)
//            A2 <- A2 + P       if bit j of u2     (unknown point)
//            P  <- 2 P                              (P = 2^j Q)
//
// All three are affine operations whose denominators go into one
// Montgomery-trick chain per lane, inverted once per step for the whole
// workgroup (Gather-Apply-Scatter, Section 3.2).  The inverse of s mod n is
// batched the same way in F_n.  Finally R = A1 + A2 is one more batched step.
// One request per lane; lanes past the end run dummy requests so that every
// lane reaches every workgroup barrier.
#pragma once
#include "kernels.h"

namespace eccmi {

enum : int { OP_NOP = 5 };  // alongside CLS_ADD .. CLS_COPY2

template <class C>
struct AffOp {
  int cls;
  Fp<typename C::F> d;  // denominator put into the chain (1 when none is needed)
};

// affine A + B with A, B canonical (infinity flags ia, ib)
template <class C>
__device__ __forceinline__ AffOp<C> plan_add(const Affine<C>& A, bool ia, const Affine<C>& B, bool ib) {
  using F = typename C::F;
  AffOp<C> op;
  op.d = fp_one<F>();
  if (ia && ib) {
    op.cls = CLS_INF;
  } else if (ia) {
    op.cls = CLS_COPY2;
  } else if (ib) {
    op.cls = CLS_COPY1;
  } else if (fp_eq_canonical<F>(A.x, B.x)) {
    if (fp_eq_canonical<F>(A.y, B.y)) {
      op.cls = CLS_DBL;  // y != 0: these curves have no point of order 2
      op.d = fp_dbl<F>(A.y);
    } else {
      op.cls = CLS_INF;
    }
  } else {
    op.cls = CLS_ADD;
    op.d = fp_sub<F>(B.x, A.x);  // normalised: two denominators are multiplied together
  }
  return op;
}

// result of a planned addition given inv = 1 / op.d; canonical output
template <class C>
__device__ __forceinline__ void apply_add(const AffOp<C>& op, const Affine<C>& A, bool ia, const Affine<C>& B, bool ib,
                                          const Fp<typename C::F>& inv, Affine<C>& R, bool& rinf) {
  using F = typename C::F;
  if (op.cls == OP_NOP) {
    R = A;
    rinf = ia;
    return;
  }
  if (op.cls == CLS_INF) {
    rinf = true;
    R = A;
    return;
  }
  if (op.cls == CLS_COPY1) {
    R = A;
    rinf = false;
    return;
  }
  if (op.cls == CLS_COPY2) {
    R = B;
    rinf = false;
    return;
  }
  Fp<F> num = op.cls == CLS_DBL ? tangent_numerator<C>(A.x, fp_one<F>()) : fp_sub_lazy<F>(B.y, A.y);
  Fp<F> lam = fp_mul<F>(num, inv);
  Fp<F> x3 = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lam), A.x), B.x));
  Fp<F> y3 = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lam, fp_sub_lazy<F>(A.x, x3)), A.y));
  R.x = x3;
  R.y = y3;
  rinf = false;
}

template <class F>
__device__ __forceinline__ bool words_eq8(const uint32_t (&a)[8], const uint32_t (&b)[8]) {
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) d |= a[k] ^ b[k];
  return d == 0;
}

// a < b for 8-word little-endian integers
__device__ __forceinline__ bool words_lt8(const uint32_t (&a)[8], const uint32_t (&b)[8]) {
  bool lt = false, decided = false;
#pragma unroll
  for (int k = 7; k >= 0; k--) {
    if (!decided && a[k] != b[k]) {
      lt = a[k] < b[k];
      decided = true;
    }
  }
  return lt;
}

__device__ __forceinline__ bool words_zero8(const uint32_t (&a)[8]) {
  uint32_t o = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) o |= a[k];
  return o == 0;
}

// Loads request i, checks ranges and the public key, and computes
// w = s^-1 (one GAS inversion in F_n for the workgroup), u1 = e w and
// u2 = r w.  Dead or invalid requests continue with dummy values (r = s = 1,
// Q = G) so that every lane reaches every barrier; ok says which are real.
template <class C, int WG>
__device__ __forceinline__ void verify_prologue(const uint8_t* __restrict__ hashes,
                                                const uint32_t* __restrict__ pubkeys,
                                                const uint32_t* __restrict__ sigs, size_t i, bool live,
                                                Fp<typename OrderField<C>::type>* n_tot,
                                                Fp<typename OrderField<C>::type>* n_inv, uint32_t (&rw)[8],
                                                uint32_t (&u1)[8], uint32_t (&u2)[8], Affine<C>& Q, bool& ok) {
  using F = typename C::F;
  using N = typename OrderField<C>::type;
  uint32_t sw[8], ew[8], qx[8], qy[8];
  constexpr Words<8> n32 = N::P32;
  constexpr Words<8> p32 = F::P32;
  ok = live;
  if (live) {
    words_load<F>(sigs + i * 16, rw);
    words_load<F>(sigs + i * 16 + 8, sw);
    words_load<F>(pubkeys + i * 16, qx);
    words_load<F>(pubkeys + i * 16 + 8, qy);
    const uint8_t* h = hashes + i * 32;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint8_t* b = h + 28 - 4 * k;  // big-endian bytes, least significant word last
      ew[k] = (uint32_t(b[0]) << 24) | (uint32_t(b[1]) << 16) | (uint32_t(b[2]) << 8) | uint32_t(b[3]);
    }
    ok = !words_zero8(rw) && words_lt8(rw, n32.w) && !words_zero8(sw) && words_lt8(sw, n32.w) &&
         words_lt8(qx, p32.w) && words_lt8(qy, p32.w) && !(words_zero8(qx) && words_zero8(qy));
  }
  if (ok) {
    Q.x = fp_canonical<F>(fp_to_mont<F>(fp_from_words<F>(qx)));
    Q.y = fp_canonical<F>(fp_to_mont<F>(fp_from_words<F>(qy)));
    ok = affine_on_curve<C>(Q);
  }
  if (!ok) {
#pragma unroll
    for (int k = 0; k < 8; k++) rw[k] = sw[k] = ew[k] = 0;
    rw[0] = sw[0] = 1;
    constexpr Words<F::NL> gx = C::GX, gy = C::GY;
    Q.x = fp_from<F>(gx);
    Q.y = fp_from<F>(gy);
  }
  Fp<N> wm = wg_batch_inverse<N, WG, 3>(fp_to_mont<N>(fp_from_words<N>(sw)), n_tot, n_inv);
  fp_to_words<N>(fp_from_mont<N>(fp_mul<N>(fp_to_mont<N>(fp_from_words<N>(ew)), wm)), u1);
  fp_to_words<N>(fp_from_mont<N>(fp_mul<N>(fp_to_mont<N>(fp_from_words<N>(rw)), wm)), u2);
}

template <class C, int WG>
__global__ void __launch_bounds__(WG) k_verify(const uint8_t* __restrict__ hashes, const uint32_t* __restrict__ pubkeys,
                                               const uint32_t* __restrict__ sigs, size_t m,
                                               const uint32_t* __restrict__ gtab, uint8_t* __restrict__ valid) {
  using F = typename C::F;
  using N = typename OrderField<C>::type;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  __shared__ Fp<N> n_tot[WG / 64], n_inv[WG / 64];
  const size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  const bool live = i < m;
  constexpr Words<8> n32 = N::P32;
  uint32_t rw[8], u1[8], u2[8];
  Affine<C> Q;
  bool ok;
  verify_prologue<C, WG>(hashes, pubkeys, sigs, i, live, n_tot, n_inv, rw, u1, u2, Q, ok);

  // ---- the bit loop ----
  Affine<C> A1, A2, P = Q;
  bool i1 = true, i2 = true;
  A1.x = A1.y = A2.x = A2.y = fp_zero<F>();
  for (int j = 0; j < 256; j++) {
    const bool b1 = (u1[j >> 5] >> (j & 31)) & 1u;
    const bool b2 = (u2[j >> 5] >> (j & 31)) & 1u;
    const Affine<C> Gj = affine_load<C>(gtab + size_t(j) * PW);
    AffOp<C> oa, ob, oc;
    if (b1) {
      oa = plan_add<C>(A1, i1, Gj, false);
    } else {
      oa.cls = OP_NOP;
      oa.d = fp_one<F>();
    }
    if (b2) {
      ob = plan_add<C>(A2, i2, P, false);
    } else {
      ob.cls = OP_NOP;
      ob.d = fp_one<F>();
    }
    oc.cls = CLS_DBL;
    oc.d = fp_dbl<F>(P.y);
    const Fp<F> dab = fp_mul<F>(oa.d, ob.d);
    Fp<F> inv = wg_batch_inverse<F, WG, 4>(fp_mul<F>(dab, oc.d), s_tot, s_inv);
    const Fp<F> inv_c = fp_mul<F>(inv, dab);
    const Fp<F> inv_ab = fp_mul<F>(inv, oc.d);
    const Fp<F> inv_b = fp_mul<F>(inv_ab, oa.d);
    const Fp<F> inv_a = fp_mul<F>(inv_ab, ob.d);
    Affine<C> t;
    bool tinf;
    apply_add<C>(oa, A1, i1, Gj, false, inv_a, t, tinf);
    A1 = t;
    i1 = tinf;
    apply_add<C>(ob, A2, i2, P, false, inv_b, t, tinf);
    A2 = t;
    i2 = tinf;
    apply_add<C>(oc, P, false, P, false, inv_c, t, tinf);
    P = t;
  }
  // ---- R = A1 + A2 ----
  AffOp<C> of = plan_add<C>(A1, i1, A2, i2);
  Fp<F> inv = wg_batch_inverse<F, WG, 4>(of.d, s_tot, s_inv);
  Affine<C> R;
  bool rinf;
  apply_add<C>(of, A1, i1, A2, i2, inv, R, rinf);

  // ---- R.x mod n == r: R.x is below p < 2n, so R.x = r or R.x = r + n ----
  if (live) {
    bool good = ok && !rinf;
    if (good) {
      uint32_t xw[8];
      fp_to_words<F>(fp_from_mont<F>(R.x), xw);
      uint32_t rn[8];
      uint64_t cy = 0;
#pragma unroll
      for (int k = 0; k < 8; k++) {
        uint64_t v = uint64_t(rw[k]) + n32.w[k] + cy;
        rn[k] = uint32_t(v);
        cy = v >> 32;
      }
      good = words_eq8<F>(xw, rw) || (cy == 0 && words_eq8<F>(xw, rn));
    }
    valid[i] = good ? 1 : 0;
  }
}

// ---- latency form: one request per lane in XYZZ coordinates -----------------
//
// The loop above inverts once per scalar bit for the whole workgroup, so a
// launch costs 257 inversion latencies however few requests it holds.  This
// form keeps each request's sum in XYZZ coordinates on its own lane and
// inverts twice per launch (s mod n, and the table below), at about the same
// number of products per request:
//   u2 Q: 4-bit windows from the most significant end, four doublings and one
//         mixed addition of T[d] = d Q per window; T[2..15] are made on the
//         lane and normalised to affine with one Montgomery-trick chain and
//         one Gather-Apply-Scatter inversion;
//   u1 G: one mixed addition per byte of u1, of d 2^(8 j) G from a comb table
//         of 32 x 256 points made once per context;
//   R.x mod n = r without an inversion: x = X / ZZ, so the test is X = r ZZ,
//         or X = (r + n) ZZ when r + n < p.

constexpr int VT_N = 15;            // table entries d Q, d = 1..15
constexpr int VCOMB_WINDOWS = 32;
constexpr int VCOMB_ENTRIES = 256;  // entry 0 of each window is never read

// words per table entry: X, Y, ZZ, ZZZ, the chain prefix and a flag word,
// rounded up to whole 16-byte groups
template <class F>
constexpr int vt_slot() {
  return (5 * F::NL + 1 + 3) / 4 * 4;
}

// every access to a table slot is a 16-byte vector access (one access type
// for the whole scratch area)
template <int K>
__device__ __forceinline__ void vt_store(uint32_t* __restrict__ s, const uint32_t (&w)[K]) {
  static_assert(K % 4 == 0, "whole 16-byte groups");
  uint4* v = reinterpret_cast<uint4*>(s);
#pragma unroll
  for (int k = 0; k < K / 4; k++) v[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

template <int K>
__device__ __forceinline__ void vt_load(const uint32_t* __restrict__ s, uint32_t (&w)[K]) {
  static_assert(K % 4 == 0, "whole 16-byte groups");
  const uint4* v = reinterpret_cast<const uint4*>(s);
#pragma unroll
  for (int k = 0; k < K / 4; k++) {
    const uint4 t = v[k];
    w[4 * k] = t.x;
    w[4 * k + 1] = t.y;
    w[4 * k + 2] = t.z;
    w[4 * k + 3] = t.w;
  }
}

template <class F>
__device__ __forceinline__ void vt_pack(uint32_t* __restrict__ w, const Fp<F>& a) {
#pragma unroll
  for (int k = 0; k < F::NL; k++) w[k] = a.w[k];
}

template <class F>
__device__ __forceinline__ Fp<F> vt_unpack(const uint32_t* __restrict__ w) {
  Fp<F> a;
#pragma unroll
  for (int k = 0; k < F::NL; k++) a.w[k] = w[k];
  return a;
}

// an affine entry: x and y in the first 2 NL words of its slot, written and
// read as whole 16-byte groups
template <class F>
constexpr int vt_affine_words() {
  return (2 * F::NL + 3) / 4 * 4;
}

template <class C>
__device__ __forceinline__ void vt_put_affine(uint32_t* __restrict__ s, const Fp<typename C::F>& x,
                                              const Fp<typename C::F>& y) {
  constexpr int NL = C::F::NL;
  uint32_t w[vt_affine_words<typename C::F>()] = {};
  vt_pack(w, x);
  vt_pack(w + NL, y);
  vt_store(s, w);
}

template <class C>
__device__ __forceinline__ Affine<C> vt_get_affine(const uint32_t* __restrict__ s) {
  using F = typename C::F;
  uint32_t w[vt_affine_words<F>()];
  vt_load(s, w);
  Affine<C> a;
  a.x = vt_unpack<F>(w);
  a.y = vt_unpack<F>(w + F::NL);
  return a;
}

// the top S bits of a 256-bit value, which is then shifted left by S (the
// digits are read by shifting, so that no register array is indexed at run
// time: such an array would be placed in scratch or LDS memory)
template <int S>
__device__ __forceinline__ uint32_t take_top(uint32_t (&a)[8]) {
  const uint32_t d = a[7] >> (32 - S);
#pragma unroll
  for (int k = 7; k > 0; k--) a[k] = (a[k] << S) | (a[k - 1] >> (32 - S));
  a[0] <<= S;
  return d;
}

// the low S bits of a 256-bit value, which is then shifted right by S
template <int S>
__device__ __forceinline__ uint32_t take_low(uint32_t (&a)[8]) {
  const uint32_t d = a[0] & ((1u << S) - 1u);
#pragma unroll
  for (int k = 0; k < 7; k++) a[k] = (a[k] >> S) | (a[k + 1] << (32 - S));
  a[7] >>= S;
  return d;
}

// This lane's table T[d] = d Q (d = 1..15) as affine entries: made in XYZZ
// coordinates, then normalised with one Montgomery-trick chain over the ZZZ
// and one Gather-Apply-Scatter inversion for the workgroup (every lane must
// call it).  An entry that is O (Q of order at most 15, possible only off the
// prime-order subgroup) puts 1 into the chain and is stored as the infinity
// marker, which the mixed addition skips.  Q itself must not be O.
template <class C, int WG>
__device__ __forceinline__ void vt_build(uint32_t* __restrict__ tab, const Affine<C>& Q, Fp<typename C::F>* s_tot,
                                         Fp<typename C::F>* s_inv) {
  using F = typename C::F;
  constexpr int NL = F::NL;
  constexpr int SLOT = vt_slot<F>();
  static_assert(vt_affine_words<F>() <= SLOT, "affine entry inside its slot");
  XYZZ<C> T = xyzz_from_affine<C>(Q);
  Fp<F> pref = fp_one<F>();
#pragma unroll 1
  for (int d = 2; d <= VT_N; d++) {
    T = xyzz_add_affine_in<C>(T, Q);  // d = 2 takes the doubling case
    const bool inf = xyzz_is_inf<C>(T);
    const Fp<F> z = inf ? fp_one<F>() : T.ZZZ;
    uint32_t w[SLOT] = {};
    vt_pack(w, T.X);
    vt_pack(w + NL, T.Y);
    vt_pack(w + 2 * NL, T.ZZ);
    vt_pack(w + 3 * NL, z);
    vt_pack(w + 4 * NL, pref);
    w[5 * NL] = inf ? 1u : 0u;
    vt_store(tab + (d - 1) * SLOT, w);
    pref = fp_mul<F>(pref, z);
  }
  Fp<F> inv = wg_batch_inverse<F, WG, 4>(pref, s_tot, s_inv);
#pragma unroll 1
  for (int d = VT_N; d >= 2; d--) {
    uint32_t* sl = tab + (d - 1) * SLOT;
    uint32_t w[SLOT];
    vt_load(sl, w);
    const Fp<F> t = fp_mul<F>(inv, vt_unpack<F>(w + 4 * NL));  // 1 / ZZZ_d
    inv = fp_mul<F>(inv, vt_unpack<F>(w + 3 * NL));            // 1 / (ZZZ_2 ... ZZZ_(d-1))
    const Fp<F> iz = fp_mul<F>(vt_unpack<F>(w + 2 * NL), t);   // 1 / Z (ZZ = Z^2, ZZZ = Z^3)
    Fp<F> x = fp_canonical<F>(fp_mul<F>(vt_unpack<F>(w), fp_sqr<F>(iz)));
    const Fp<F> y = fp_canonical<F>(fp_mul<F>(vt_unpack<F>(w + NL), t));
    if (w[5 * NL]) x = fp_inf_marker<F>();
    vt_put_affine<C>(sl, x, y);
  }
  vt_put_affine<C>(tab, Q.x, Q.y);
}

// u Q from this lane's table: 4-bit windows from the most significant end,
// four doublings and one mixed addition each; u (256 bits) is consumed
template <class C>
__device__ __forceinline__ XYZZ<C> vt_mul(const uint32_t* __restrict__ tab, uint32_t (&u)[8]) {
  constexpr int SLOT = vt_slot<typename C::F>();
  XYZZ<C> A = xyzz_inf<C>();
#pragma unroll 1
  for (int w = 63; w >= 0; w--) {
    if (w != 63) {
#pragma unroll 1
      for (int k = 0; k < 4; k++) A = xyzz_dbl_in<C>(A);
    }
    const uint32_t d = take_top<4>(u);
    if (d != 0) A = xyzz_add_affine_in<C>(A, vt_get_affine<C>(tab + (d - 1) * SLOT));
  }
  return A;
}

// scratch: VT_N * vt_slot<F>() words per lane of the grid (dead lanes included)
template <class C, int WG>
__global__ void __launch_bounds__(WG) k_verify_xyzz(const uint8_t* __restrict__ hashes,
                                                    const uint32_t* __restrict__ pubkeys,
                                                    const uint32_t* __restrict__ sigs, size_t m,
                                                    const uint32_t* __restrict__ gcomb,
                                                    uint32_t* __restrict__ scratch, uint8_t* __restrict__ valid) {
  using F = typename C::F;
  using N = typename OrderField<C>::type;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  __shared__ Fp<N> n_tot[WG / 64], n_inv[WG / 64];
  const size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  const bool live = i < m;
  constexpr Words<8> n32 = N::P32;
  constexpr Words<8> p32 = F::P32;
  uint32_t rw[8], u1[8], u2[8];
  Affine<C> Q;
  bool ok;
  verify_prologue<C, WG>(hashes, pubkeys, sigs, i, live, n_tot, n_inv, rw, u1, u2, Q, ok);

  uint32_t* tab = scratch + i * size_t(VT_N * vt_slot<F>());
  vt_build<C, WG>(tab, Q, s_tot, s_inv);
  XYZZ<C> A = vt_mul<C>(tab, u2);  // A = u2 Q
  // ---- A += u1 G ----
#pragma unroll 1
  for (int j = 0; j < VCOMB_WINDOWS; j++) {
    const uint32_t d = take_low<8>(u1);
    if (d != 0) A = xyzz_add_affine_in<C>(A, affine_load<C>(gcomb + size_t(j * VCOMB_ENTRIES + d) * PW));
  }

  // ---- R.x mod n == r: R.x is below p < 2n, so R.x = r or R.x = r + n ----
  if (live) {
    bool good = ok && !xyzz_is_inf<C>(A);
    if (good) {
      const Fp<F> X = fp_canonical<F>(A.X);
      bool eq = fp_eq_canonical<F>(X, fp_canonical<F>(fp_mul<F>(fp_to_mont<F>(fp_from_words<F>(rw)), A.ZZ)));
      uint32_t rn[8];
      uint64_t cy = 0;
#pragma unroll
      for (int k = 0; k < 8; k++) {
        uint64_t v = uint64_t(rw[k]) + n32.w[k] + cy;
        rn[k] = uint32_t(v);
        cy = v >> 32;
      }
      if (!eq && cy == 0 && words_lt8(rn, p32.w))
        eq = fp_eq_canonical<F>(X, fp_canonical<F>(fp_mul<F>(fp_to_mont<F>(fp_from_words<F>(rn)), A.ZZ)));
      good = eq;
    }
    valid[i] = good ? 1 : 0;
  }
}

// ---- ECDSA signature generation ---------------------------------------------
//
// Per request: with 1 <= d, k < n, R = k G, r = R.x mod n and
// s = k^-1 (e + r d) mod n, e the hash read big-endian.  A request whose d or
// k is out of range, or whose r or s comes out zero, gets r = s = 0 (the
// caller draws another nonce).  The paper's signing workload is one
// fixed-point multiplication and one inversion mod n (Section 5.2): here k G
// is 32 mixed additions from the comb table in XYZZ coordinates on the lane,
// and 1 / ZZ (for R.x = X / ZZ) and k^-1 are one GAS inversion each per
// workgroup.
template <class C, int WG>
__global__ void __launch_bounds__(WG) k_sign(const uint8_t* __restrict__ hashes, const uint32_t* __restrict__ privkeys,
                                             const uint32_t* __restrict__ nonces, size_t m,
                                             const uint32_t* __restrict__ gcomb, uint32_t* __restrict__ sigs) {
  using F = typename C::F;
  using N = typename OrderField<C>::type;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  __shared__ Fp<N> n_tot[WG / 64], n_inv[WG / 64];
  const size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  const bool live = i < m;
  constexpr Words<8> n32 = N::P32;
  uint32_t dw[8], kw[8], ew[8];
  bool ok = live;
  if (live) {
    words_load<N>(privkeys + i * 8, dw);
    words_load<N>(nonces + i * 8, kw);
    const uint8_t* h = hashes + i * 32;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint8_t* b = h + 28 - 4 * k;  // big-endian bytes, least significant word last
      ew[k] = (uint32_t(b[0]) << 24) | (uint32_t(b[1]) << 16) | (uint32_t(b[2]) << 8) | uint32_t(b[3]);
    }
    ok = !words_zero8(dw) && words_lt8(dw, n32.w) && !words_zero8(kw) && words_lt8(kw, n32.w);
  }
  if (!ok) {  // dead or rejected requests continue with d = k = 1, e = 0
#pragma unroll
    for (int k = 0; k < 8; k++) dw[k] = kw[k] = ew[k] = 0;
    dw[0] = kw[0] = 1;
  }

  // ---- R = k G from the comb ----
  uint32_t kd[8];
#pragma unroll
  for (int k = 0; k < 8; k++) kd[k] = kw[k];
  XYZZ<C> A = xyzz_inf<C>();
#pragma unroll 1
  for (int j = 0; j < VCOMB_WINDOWS; j++) {
    const uint32_t d = take_low<8>(kd);
    if (d != 0) A = xyzz_add_affine_in<C>(A, affine_load<C>(gcomb + size_t(j * VCOMB_ENTRIES + d) * PW));
  }
  // 0 < k < n, so R != O and ZZ != 0
  const Fp<F> izz = wg_batch_inverse<F, WG, 4>(A.ZZ, s_tot, s_inv);
  uint32_t rw[8];
  fp_to_words<F>(fp_from_mont<F>(fp_canonical<F>(fp_mul<F>(A.X, izz))), rw);
  // r = R.x mod n: R.x < p < 2n
  if (!words_lt8(rw, n32.w)) {
    int64_t br = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const int64_t v = int64_t(rw[k]) - int64_t(n32.w[k]) + br;
      rw[k] = uint32_t(v);
      br = v >> 32;
    }
  }

  // ---- s = k^-1 (e + r d) mod n ----
  const Fp<N> kinv = wg_batch_inverse<N, WG, 3>(fp_to_mont<N>(fp_from_words<N>(kw)), n_tot, n_inv);
  const Fp<N> t = fp_add<N>(fp_to_mont<N>(fp_from_words<N>(ew)),
                            fp_mul<N>(fp_to_mont<N>(fp_from_words<N>(rw)), fp_to_mont<N>(fp_from_words<N>(dw))));
  uint32_t sw[8];
  fp_to_words<N>(fp_from_mont<N>(fp_mul<N>(t, kinv)), sw);
  if (live) {
    const bool good = ok && !words_zero8(rw) && !words_zero8(sw);
#pragma unroll
    for (int k = 0; k < 8; k++) {
      rw[k] = good ? rw[k] : 0u;
      sw[k] = good ? sw[k] : 0u;
    }
    words_store<N>(sigs + i * 16, rw);
    words_store<N>(sigs + i * 16 + 8, sw);
  }
}

// ---- batched unknown-point multiplication -----------------------------------
//
// out_i = k_i P_i for points known only at run time (the paper's UPMUL, the
// unknown-point half of its batch PMUL workload, Section 3.4 and Table 5),
// one request per lane: the table of d P_i and 4-bit windows of k_i as in
// the per-lane verification, then the result's 1 / (ZZ ZZZ) by one GAS
// inversion per workgroup.  pts are working-form affine points (the infinity
// marker for O); every k_i is a 256-bit integer, taken as is.
template <class C, int WG>
__global__ void __launch_bounds__(WG) k_pmul(const uint32_t* __restrict__ pts, const uint32_t* __restrict__ ks,
                                             size_t n, uint32_t* __restrict__ scratch, uint32_t* __restrict__ out,
                                             int out_mont) {
  using F = typename C::F;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  const size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  const bool live = i < n;
  Affine<C> P;
  uint32_t k[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool pinf = true;
  if (live) {
    P = affine_load<C>(pts + i * PW);
    pinf = fp_is_inf_marker<F>(P.x);
    load_scalar(ks + 8 * i, k);
  }
  if (pinf) {  // O, or a lane past the end: run on G, give O
    constexpr Words<F::NL> gx = C::GX, gy = C::GY;
    P.x = fp_from<F>(gx);
    P.y = fp_from<F>(gy);
  }
  uint32_t* tab = scratch + i * size_t(VT_N * vt_slot<F>());
  vt_build<C, WG>(tab, P, s_tot, s_inv);
  const XYZZ<C> A = vt_mul<C>(tab, k);
  store_xyzz_affine<C, WG>(A, pinf || xyzz_is_inf<C>(A), live, out + i * 2 * F::N32, out_mont, s_tot, s_inv);
}

// ---- batched unknown-point multiplication in affine coordinates ------------
//
// out_j = k_j P_j by the paper's batch UPMUL (Section 3.4, Algorithm 3): the
// scalar bits are walked from the least significant end; at bit i every
// request j has one point addition R_j = P_j + Q_j (P_j = 2^i P, Q_j the sum
// of the bits so far) and one doubling P_j <- 2 P_j, both affine.  Their two
// denominators t1 = 2 P_j.y (doubling) and t2 = P_j.x - Q_j.x (addition)
// enter one Montgomery-trick chain per lane, which walks the lane's requests;
// only the product T1 before both is kept per request (find-then-recompute:
// T1 t1 is recomputed from T1 and t1 in the decompress step), and the chain
// is inverted once per bit for the whole workgroup (GAS, Section 3.2).  The
// decompress step then finishes the addition first and the doubling second,
// each with its recovered inverse, and Q_j takes R_j when bit i of k_j is
// set: the addition is computed for every bit (a dummy one while Q_j is O),
// as the paper does for constant time.
//
// Request j of lane g is slot t of that lane, j = t T + g (T lanes in the
// grid), and its state lives in limb-major planes over the padded count
// J = T kper, so that a wave's accesses coalesce: P.x, P.y, Q.x, Q.y and the
// stored T1 (NL planes each), then the scalar (8 planes).  Exceptional
// additions (Q_j = O, Q_j = P_j, Q_j = -P_j) put 1 into the chain and are
// resolved in the decompress step; no curve here has a point of order 2, so
// 2^i P is never O and t1 is never 0.
template <class F>
constexpr int upmul_state_words() {
  return 5 * F::NL + 8;
}

enum : int { UP_ADD = 0, UP_COPY_P = 1, UP_TWICE = 2, UP_INF = 3 };

template <class C, int WG>
__global__ void __launch_bounds__(WG) k_upmul_affine(const uint32_t* __restrict__ pts, const uint32_t* __restrict__ ks,
                                                     size_t n, uint32_t kper, uint32_t* __restrict__ state,
                                                     uint32_t* __restrict__ out, int out_mont) {
  using F = typename C::F;
  constexpr int NL = F::NL;
  constexpr int N32 = F::N32;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  const size_t T = size_t(gridDim.x) * WG;
  const size_t J = T * kper;
  const size_t g = size_t(blockIdx.x) * WG + threadIdx.x;
  uint32_t* const px = state;
  uint32_t* const py = px + NL * J;
  uint32_t* const qx = py + NL * J;
  uint32_t* const qy = qx + NL * J;
  uint32_t* const mm = qy + NL * J;
  uint32_t* const sc = mm + NL * J;
  const Fp<F> one = fp_one<F>();
  constexpr Words<F::NL> gx = C::GX, gy = C::GY;

  // ---- state: P_j (G with a zero scalar for O and for padding), Q_j = O ----
  for (uint32_t t = 0; t < kper; t++) {
    const size_t j = size_t(t) * T + g;
    Affine<C> P;
    P.x = fp_from<F>(gx);
    P.y = fp_from<F>(gy);
    uint32_t k[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (j < n) {
      const Affine<C> A = affine_load<C>(pts + j * PW);
      if (!fp_is_inf_marker<F>(A.x)) {
        P = A;
        load_scalar(ks + 8 * j, k);
      }
    }
    fp_store_soa<F>(px + j, J, P.x);
    fp_store_soa<F>(py + j, J, P.y);
    fp_store_soa<F>(qx + j, J, fp_inf_marker<F>());
    fp_store_soa<F>(qy + j, J, fp_zero<F>());
#pragma unroll
    for (int w = 0; w < 8; w++) sc[size_t(w) * J + j] = k[w];
  }

  for (int i = 0; i < 256; i++) {
    // compress: M_j = T1 before request j, T1 <- T1 t1 t2
    Fp<F> acc = one;
    for (uint32_t t = 0; t < kper; t++) {
      const size_t j = size_t(t) * T + g;
      const Fp<F> Py = fp_load_soa<F>(py + j, J);
      const Fp<F> t1 = fp_dbl<F>(Py);
      const Fp<F> Px = fp_load_soa<F>(px + j, J);
      const Fp<F> Qx = fp_load_soa<F>(qx + j, J);
      Fp<F> t2 = one;
      if (!fp_is_inf_marker<F>(Qx) && !fp_eq_canonical<F>(Px, Qx)) t2 = fp_sub_lazy<F>(Px, Qx);
      fp_store_soa<F>(mm + j, J, acc);
      acc = fp_mul<F>(fp_mul<F>(acc, t1), t2);
    }
    Fp<F> inv = wg_batch_inverse<F, WG, 20>(acc, s_tot, s_inv);
    // decompress with the addition, then the doubling, of every request
    for (int t = int(kper) - 1; t >= 0; t--) {
      const size_t j = size_t(t) * T + g;
      const Fp<F> M = fp_load_soa<F>(mm + j, J);
      Affine<C> P, Q;
      P.x = fp_load_soa<F>(px + j, J);
      P.y = fp_load_soa<F>(py + j, J);
      Q.x = fp_load_soa<F>(qx + j, J);
      Q.y = fp_load_soa<F>(qy + j, J);
      const bool bit = (sc[size_t(i >> 5) * J + j] >> (i & 31)) & 1u;
      const Fp<F> t1 = fp_dbl<F>(P.y);
      int cls = UP_ADD;
      Fp<F> t2 = one;
      if (fp_is_inf_marker<F>(Q.x)) cls = UP_COPY_P;
      else if (fp_eq_canonical<F>(P.x, Q.x)) cls = fp_eq_canonical<F>(P.y, Q.y) ? UP_TWICE : UP_INF;
      else t2 = fp_sub_lazy<F>(P.x, Q.x);
      const Fp<F> T1t1 = fp_mul<F>(t1, M);   // the discarded product, recomputed
      const Fp<F> t2inv = fp_mul<F>(inv, T1t1);
      inv = fp_mul<F>(inv, t2);              // 1 / (T1 t1)
      const Fp<F> t1inv = fp_mul<F>(inv, M);
      inv = fp_mul<F>(inv, t1);              // 1 / T1: the previous request's total
      Affine<C> R = P;
      if (cls == UP_ADD) {
        const Fp<F> lam = fp_mul<F>(fp_sub_lazy<F>(P.y, Q.y), t2inv);
        R.x = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lam), P.x), Q.x));
        R.y = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lam, fp_sub_lazy<F>(P.x, R.x)), P.y));
      }
      // the doubling: lambda = (3 x^2 + a) / (2 y)
      const Fp<F> lamd = fp_mul<F>(tangent_numerator<C>(P.x, one), t1inv);
      Affine<C> D;
      D.x = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lamd), P.x), P.x));
      D.y = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lamd, fp_sub_lazy<F>(P.x, D.x)), P.y));
      if (cls == UP_TWICE) R = D;
      if (cls == UP_INF) {
        R.x = fp_inf_marker<F>();
        R.y = fp_zero<F>();
      }
      fp_store_soa<F>(px + j, J, D.x);
      fp_store_soa<F>(py + j, J, D.y);
      if (bit) {
        fp_store_soa<F>(qx + j, J, R.x);
        fp_store_soa<F>(qy + j, J, R.y);
      }
    }
  }

  // ---- results: Q_j in the boundary form ----
  constexpr Words<F::NL> rout = F::ROUT;
  Fp<F> k1 = fp_zero<F>();
  k1.w[0] = 1;
  const Fp<F> kf = out_mont ? fp_from<F>(rout) : k1;
  for (uint32_t t = 0; t < kper; t++) {
    const size_t j = size_t(t) * T + g;
    if (j >= n) break;
    const Fp<F> Qx = fp_load_soa<F>(qx + j, J);
    const bool qinf = fp_is_inf_marker<F>(Qx);
    uint32_t xw[N32], yw[N32];
    fp_to_words<F>(fp_canonical<F>(fp_mul<F>(Qx, kf)), xw);
    fp_to_words<F>(fp_canonical<F>(fp_mul<F>(fp_load_soa<F>(qy + j, J), kf)), yw);
#pragma unroll
    for (int w = 0; w < N32; w++) {
      xw[w] = qinf ? 0u : xw[w];
      yw[w] = qinf ? 0u : yw[w];
    }
    words_store<F>(out + j * 2 * N32, xw);
    words_store<F>(out + j * 2 * N32 + N32, yw);
  }
}

// ---- fixed-point multiplication from the comb -------------------------------
//
// out_i = k_i G for any 256-bit k_i: one mixed addition per byte of k_i, of
// d 2^(8 j) G from the context's comb table (the paper's FPMUL with a
// precomputed table, Section 2.1), in XYZZ coordinates on the lane, then the
// affine result by one GAS inversion per workgroup.
template <class C, int WG>
__global__ void __launch_bounds__(WG) k_fixed_base_comb(const uint32_t* __restrict__ ks, size_t n,
                                                        const uint32_t* __restrict__ gcomb, uint32_t* __restrict__ out,
                                                        int out_mont) {
  using F = typename C::F;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  const size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  const bool active = i < n;
  uint32_t k[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (active) load_scalar(ks + 8 * i, k);
  XYZZ<C> A = xyzz_inf<C>();
#pragma unroll 1
  for (int j = 0; j < VCOMB_WINDOWS; j++) {
    const uint32_t d = take_low<8>(k);
    if (d != 0) A = xyzz_add_affine_in<C>(A, affine_load<C>(gcomb + size_t(j * VCOMB_ENTRIES + d) * PW));
  }
  store_xyzz_affine<C, WG>(A, xyzz_is_inf<C>(A), active, out + i * 2 * F::N32, out_mont, s_tot, s_inv);
}

}  // namespace eccmi
