// Lane-parallel prime-field arithmetic for chains that run on one wave.
//
// The window combination is a single chain of about a hundred point
// doublings on one wave.  With one element per lane, a product costs the full
// limb-by-limb schedule of one lane while 60 lanes idle.  Here an element
// occupies a 16-lane row instead: lane j of the row holds limb j of the
// working form (radix 2^B, Montgomery R = 2^(B NL), the representation of
// field.h); lanes NL..15 hold 0.  A wave carries four independent elements,
// one per row, and one instruction stream computes four products.  Limbs move
// between lanes through DPP row operations (broadcast of one lane to its row,
// rotation inside the row, shift by one lane), never through LDS.
//
// Product (Section 2.2, Algorithm 2 with D = 2^B).  Lane j accumulates the
// product columns j and j + 16 in two 64-bit registers: for i = 0..NL-1 the
// limb a_i is broadcast to the row and b is rotated by i lanes, so that lane
// j multiplies a_i by b_{(j - i) mod 16}, which belongs to column j when
// j >= i and to column j + 16 otherwise.  The reduction then walks the
// columns i = 0..NL-1 in order: the broadcast column value plus the carry out
// of column i - 1 gives M_i = C_i q_inv mod 2^B; M_i q is added at columns
// i + m through a per-lane table of q's limbs rotated by i; the carry out of
// column i stays in a register.  Columns NL..2NL-1, rotated back to lanes
// 0..NL-1, plus the last carry are the result, brought to small limbs by two
// carry passes.
//
// Value conventions:
//   lp_mul inputs : limbs < 2^30 and a b < 36 p^2 (so that every 64-bit column
//                   and the Montgomery bound (a b + M q) / R < 2p hold for
//                   BN254, where R / p ~ 170, and BLS12-381, R / p ~ 2^11);
//   lp_mul output : limbs < 2^B + 2^9 below the top one, value < 2p;
//   lp_sub output : limbs <= 2^B below the top one, value < 2p (a - b + 8p,
//                   then the quotient by p estimated from the top limb is
//                   subtracted); lp_sub takes a < 8p with limbs below the
//                   top one < 4 2^B and b < 6p with limbs < 3 2^B - 3;
//   lp_canonical  : limbs < 2^B, value < p (the canonical form of field.h);
//   LpPoint Y     : as an lp_sub output, or (where lp_lazy_y holds) below 10p
//                   with limbs < 2^B + 16 (lp_sub_y).  The point formulas
//                   multiply it at most as (2Y)^2 < 400 p^2 and Y W < 20 p^2.
#pragma once
#include <type_traits>

#include "point.h"

namespace eccmi {

template <int I, int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, N>(fn);
  }
}

__device__ __forceinline__ uint32_t lane16() { return threadIdx.x & 15u; }
__device__ __forceinline__ uint32_t row4() { return (threadIdx.x >> 4) & 3u; }

// DPP moves inside 16-lane rows (lanes without a source read 0)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  return uint64_t(dpp32<CTRL>(uint32_t(v))) | (uint64_t(dpp32<CTRL>(uint32_t(v >> 32))) << 32);
}
constexpr int DPP_ROW_SHR(int n) { return 0x110 + n; }    // lane j <- lane j - n (0 below)
constexpr int DPP_ROW_ROR(int n) { return 0x120 + n; }    // lane j <- lane (j - n) mod 16
constexpr int DPP_ROW_BCAST(int n) { return 0x150 + n; }  // every lane <- lane n of its row

// 8p with every limb below the top one raised into [3 2^B - 3, 4 2^B - 3)
// by borrowing 3 from the next limb: a subtrahend with limbs below 3 2^B - 3
// and value below 6p leaves non-negative limbs in a - b + 8p
template <class F>
constexpr Words<F::NL> lp_sub_bias() {
  Words<F::NL> d{};
  uint64_t c = 0;
  for (int i = 0; i < F::NL; i++) {
    const uint64_t v = uint64_t(F::P.w[i]) * 8u + c;
    d.w[i] = i == F::NL - 1 ? uint32_t(v) : uint32_t(v & F::MASK);
    c = v >> F::B;
  }
  Words<F::NL> k{};
  for (int i = 0; i < F::NL; i++) {
    int64_t v = int64_t(d.w[i]);
    if (i < F::NL - 1) v += int64_t(3) << F::B;
    if (i > 0) v -= 3;
    k.w[i] = uint32_t(v);
  }
  return k;
}

// per-lane constants of one field
template <class F>
struct LpK {
  uint32_t p;           // lane j: limb j of p
  uint32_t bias;        // lane j: limb j of lp_sub_bias
  uint32_t plo[F::NL];  // lane j: p_{j-i} for j >= i, else 0
  uint32_t phi[F::NL];  // lane j: p_{j-i+16} for j < i, else 0
};

// lane j of each row: limb j of a constant (0 past NL)
template <class F>
__device__ __forceinline__ uint32_t lp_const(const Words<F::NL>& c) {
  const uint32_t j = lane16();
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) v = j == uint32_t(i) ? c.w[i] : v;
  return v;
}

template <class F>
__device__ __forceinline__ LpK<F> lp_consts() {
  constexpr Words<F::NL> P = F::P;
  constexpr Words<F::NL> BIAS = lp_sub_bias<F>();
  LpK<F> k;
  k.p = lp_const<F>(P);
  k.bias = lp_const<F>(BIAS);
  const uint32_t j = lane16();
  static_for<0, F::NL>([&](auto I) {
    constexpr int i = I;
    if constexpr (i == 0) {
      k.plo[0] = k.p;
      k.phi[0] = 0;
    } else {
      k.plo[i] = dpp32<DPP_ROW_SHR(i)>(k.p);
      const uint32_t r = dpp32<DPP_ROW_ROR(i)>(k.p);
      k.phi[i] = j < uint32_t(i) ? r : 0u;
    }
  });
  return k;
}

// one carry pass: limbs below the top one keep B bits and pass the rest up;
// the top limb (lane NL - 1) keeps everything; lanes past NL stay 0
template <class F>
__device__ __forceinline__ uint64_t lp_carry64(uint64_t v) {
  const uint32_t j = lane16();
  const bool top = j == uint32_t(F::NL - 1);
  const uint64_t c = top ? 0 : (v >> F::B);
  const uint64_t m = top ? v : (v & F::MASK);
  return m + dpp64<DPP_ROW_SHR(1)>(c);
}

template <class F>
__device__ __forceinline__ uint32_t lp_carry32(uint32_t v) {
  const uint32_t j = lane16();
  const bool top = j == uint32_t(F::NL - 1);
  const uint32_t c = top ? 0u : (v >> F::B);
  const uint32_t m = top ? v : (v & F::MASK);
  return m + dpp32<DPP_ROW_SHR(1)>(c);
}

// Montgomery product a b / R of the four row elements
template <class F>
__device__ __forceinline__ uint32_t lp_mul(uint32_t a, uint32_t b, const LpK<F>& k) {
  constexpr int NL = F::NL;
  const uint32_t j = lane16();
  uint64_t lo = 0, hi = 0;
  static_for<0, NL>([&](auto I) {
    constexpr int i = I;
    const uint32_t ai = dpp32<DPP_ROW_BCAST(i)>(a);
    if constexpr (i == 0) {
      lo = uint64_t(ai) * b;
    } else {
      const uint32_t br = dpp32<DPP_ROW_ROR(i)>(b);
      const uint32_t ml = j >= uint32_t(i) ? ai : 0u;
      lo += uint64_t(ml) * br;
      hi += uint64_t(ai - ml) * br;
    }
  });
  constexpr uint32_t P0 = F::P.w[0];
  uint64_t carry = 0;
  static_for<0, NL>([&](auto I) {
    constexpr int i = I;
    const uint64_t ci = dpp64<DPP_ROW_BCAST(i)>(lo) + carry;
    const uint32_t q = (uint32_t(ci) * F::QINV) & F::MASK;
    lo += uint64_t(q) * k.plo[i];
    hi += uint64_t(q) * k.phi[i];
    carry = (ci + uint64_t(q) * P0) >> F::B;
  });
  // lane r <- column NL + r: low columns of lanes NL..15, then high columns
  constexpr int ROT = 16 - NL;
  const uint64_t rl = dpp64<DPP_ROW_ROR(ROT)>(lo);
  const uint64_t rh = dpp64<DPP_ROW_ROR(ROT)>(hi);
  uint64_t r = j + uint32_t(NL) < 16u ? rl : rh;
  if (j == 0) r += carry;
  if (j >= uint32_t(NL)) r = 0;
  r = lp_carry64<F>(r);
  return uint32_t(lp_carry64<F>(r));
}

__device__ __forceinline__ uint32_t lp_add(uint32_t a, uint32_t b) { return a + b; }

// value < 16p with limbs below the top one < 2^(B+3) -> value < 2p, limbs <= 2^B
template <class F>
__device__ __forceinline__ uint32_t lp_reduce(uint32_t v, const LpK<F>& k) {
  constexpr uint32_t PTOP = F::P.w[F::NL - 1];
  constexpr uint32_t QR = uint32_t((uint64_t(1) << 32) / (uint64_t(PTOP) + 1));
  v = lp_carry32<F>(v);
  // q <= top / (PTOP + 1) <= floor(v / p), and v - q p < 2p
  const uint32_t t = dpp32<DPP_ROW_BCAST(F::NL - 1)>(v);
  const uint32_t q = __umulhi(t, QR);
  int64_t d = int64_t(v) - int64_t(uint64_t(q) * k.p);
  // signed carries until every limb below the top one is in [0, 2^B)
  const uint32_t j = lane16();
  const bool top = j == uint32_t(F::NL - 1);
  for (;;) {
    const int64_t c = top ? 0 : (d >> F::B);
    if (__ballot(c != 0) == 0) break;
    const int64_t m = top ? d : (d & int64_t(F::MASK));
    d = m + int64_t(dpp64<DPP_ROW_SHR(1)>(uint64_t(c)));
  }
  return uint32_t(d);
}

// a - b (a < 8p with limbs below the top one < 4 2^B, b < 6p with limbs
// below the top one < 3 2^B - 3: a + 8p - b then has non-negative limbs below
// 2^(B+3), the top one included, and a value below 16p, the domain of
// lp_reduce)
template <class F>
__device__ __forceinline__ uint32_t lp_sub(uint32_t a, uint32_t b, const LpK<F>& k) {
  return lp_reduce<F>(a + k.bias - b, k);
}

// bit length of p, and whether R / p >= 2^10: then the largest product an
// unreduced Y enters, (2Y)^2 < 400 p^2, still has (a b + M q) / R < 2p
template <class F>
constexpr int lp_p_bits() {
  uint32_t t = F::P.w[F::NL - 1];
  int b = 0;
  while (t) {
    b++;
    t >>= 1;
  }
  return F::B * (F::NL - 1) + b;
}
template <class F>
constexpr bool lp_lazy_y() {
  return F::B * F::NL - lp_p_bits<F>() >= 10;
}

// a - b for a Y coordinate (a, b product outputs): where lp_lazy_y holds,
// a + 8p - b after one carry pass (value below 10p, limbs below 2^B + 16),
// without the quotient and the signed carries of lp_sub
template <class F>
__device__ __forceinline__ uint32_t lp_sub_y(uint32_t a, uint32_t b, const LpK<F>& k) {
  if constexpr (lp_lazy_y<F>()) {
    return lp_carry32<F>(a + k.bias - b);
  } else {
    return lp_sub<F>(a, b, k);
  }
}

// canonical form (limbs < 2^B, value < p) of a value < 2p with limbs < 2^31
template <class F>
__device__ __forceinline__ uint32_t lp_canonical(uint32_t v, const LpK<F>& k) {
  const uint32_t j = lane16();
  const bool top = j == uint32_t(F::NL - 1);
  for (;;) {
    const uint32_t c = top ? 0u : (v >> F::B);
    if (__ballot(c != 0) == 0) break;
    v = (top ? v : (v & F::MASK)) + dpp32<DPP_ROW_SHR(1)>(c);
  }
  // v >= p: the highest limb where v and p differ has v's larger
  const uint32_t sh = row4() * 16u;
  const uint32_t gt = uint32_t(__ballot(v > k.p) >> sh) & 0xFFFFu;
  const uint32_t lt = uint32_t(__ballot(v < k.p) >> sh) & 0xFFFFu;
  if (gt >= lt) {
    int32_t d = int32_t(v) - int32_t(k.p);
    for (;;) {
      const int32_t c = top ? 0 : (d >> F::B);
      if (__ballot(c != 0) == 0) break;
      d = (top ? d : (d & int32_t(F::MASK))) + int32_t(dpp32<DPP_ROW_SHR(1)>(uint32_t(c)));
    }
    v = uint32_t(d);
  }
  return v;
}

// the value is 0 mod p (all four rows hold the same element: wave-uniform)
template <class F>
__device__ __forceinline__ bool lp_is_zero(uint32_t v, const LpK<F>& k) {
  return __ballot(lp_canonical<F>(v, k) != 0) == 0;
}

// element r of a wave whose rows hold a0..a3
__device__ __forceinline__ uint32_t lp_rows(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3) {
  const uint32_t r = row4();
  return r == 0 ? a0 : r == 1 ? a1 : r == 2 ? a2 : a3;
}

// row r's element in every row
__device__ __forceinline__ uint32_t lp_take(uint32_t v, int r) {
  // rows move between registers without LDS: v_permlane32_swap of v with
  // itself leaves rows (0 1 0 1) and (2 3 2 3), and v_permlane16_swap of one
  // of those with itself leaves (x x x x) for its even and its odd row
  const auto h = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  const uint32_t hv = r < 2 ? h[0] : h[1];
  const auto q = __builtin_amdgcn_permlane16_swap(hv, hv, false, false);
  return (r & 1) ? q[1] : q[0];
}

// working-form words of one coordinate (lane j reads limb j) and back
template <class F>
__device__ __forceinline__ uint32_t lp_load(const uint32_t* p) {
  const uint32_t j = lane16();
  return j < uint32_t(F::NL) ? p[j] : 0u;
}

// the element of row 0 as a per-lane field element (every lane the same)
template <class F>
__device__ __forceinline__ Fp<F> lp_to_fp(uint32_t v) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = uint32_t(__shfl(int(v), i, 64));
  return r;
}

// ---- XYZZ points with every coordinate replicated in all four rows --------

template <class C>
struct LpPoint {
  uint32_t X, Y, ZZ, ZZZ;
  bool inf;  // wave-uniform
};

// dbl-2008-s-1 (a = 0) in three product levels:
// [U^2, X^2] -> [U V, X V, V ZZ, M^2] -> [M (S - X3), W Y, W ZZZ]
template <class C>
__device__ __forceinline__ LpPoint<C> lp_dbl(const LpPoint<C>& P, const LpK<typename C::F>& k) {
  using F = typename C::F;
  static_assert(!C::A_IS_MINUS3, "the lane-parallel doubling is written for a = 0");
  if (P.inf) return P;
  const uint32_t U = lp_add(P.Y, P.Y);
  uint32_t z = lp_mul<F>(lp_rows(U, P.X, U, P.X), lp_rows(U, P.X, U, P.X), k);
  const uint32_t V = lp_take(z, 0), XX = lp_take(z, 1);
  const uint32_t M = lp_carry32<F>(XX + XX + XX);
  z = lp_mul<F>(lp_rows(U, P.X, V, M), lp_rows(V, V, P.ZZ, M), k);
  const uint32_t W = lp_take(z, 0), S = lp_take(z, 1), ZZ3 = lp_take(z, 2), MM = lp_take(z, 3);
  // X3 = M^2 - 2S (row 0) and S - X3 = 3S - M^2 (the other rows) in one
  // reduction: 3S < 6p has limbs below 3 (2^B + 2^9) < 4 2^B
  const bool r0 = row4() == 0u;
  const uint32_t S2 = S + S;
  const uint32_t d = lp_sub<F>(r0 ? MM : S2 + S, r0 ? S2 : MM, k);
  const uint32_t X3 = lp_take(d, 0), T = lp_take(d, 1);
  z = lp_mul<F>(lp_rows(M, W, W, W), lp_rows(T, P.Y, P.ZZZ, P.ZZZ), k);
  LpPoint<C> R;
  R.X = X3;
  R.Y = lp_sub_y<F>(lp_take(z, 0), lp_take(z, 1), k);
  R.ZZ = ZZ3;
  R.ZZZ = lp_take(z, 2);
  R.inf = false;
  return R;
}

// add-2008-s in four product levels:
// [X1 ZZ2, X2 ZZ1, Y1 ZZZ2, Y2 ZZZ1] -> [P^2, R^2, ZZ1 ZZ2, ZZZ1 ZZZ2]
//   -> [P PP, U1 PP, (ZZ1 ZZ2) PP] -> [R (Q - X3), S1 PPP, (ZZZ1 ZZZ2) PPP]
template <class C>
__device__ __forceinline__ LpPoint<C> lp_add_pts(const LpPoint<C>& A, const LpPoint<C>& B,
                                                 const LpK<typename C::F>& k) {
  using F = typename C::F;
  if (A.inf) return B;
  if (B.inf) return A;
  uint32_t z = lp_mul<F>(lp_rows(A.X, B.X, A.Y, B.Y), lp_rows(B.ZZ, A.ZZ, B.ZZZ, A.ZZZ), k);
  // rows (U1, U2, S1, S2) -> (U1 U1 S1 S1) and (U2 U2 S2 S2): one reduction
  // gives P = U2 - U1 in rows 0-1 and R = S2 - S1 in rows 2-3
  const auto e = __builtin_amdgcn_permlane16_swap(z, z, false, false);
  const auto us1 = __builtin_amdgcn_permlane32_swap(e[0], e[0], false, false);
  const uint32_t U1 = us1[0], S1 = us1[1];
  const uint32_t d = lp_sub<F>(e[1], e[0], k);
  const auto pr = __builtin_amdgcn_permlane32_swap(d, d, false, false);
  const uint32_t P = pr[0], R = pr[1];
  if (lp_is_zero<F>(P, k)) {
    if (lp_is_zero<F>(R, k)) return lp_dbl<C>(A, k);
    LpPoint<C> O = A;
    O.inf = true;
    return O;
  }
  z = lp_mul<F>(lp_rows(P, R, A.ZZ, A.ZZZ), lp_rows(P, R, B.ZZ, B.ZZZ), k);
  const uint32_t PP = lp_take(z, 0), RR = lp_take(z, 1), Zf = lp_take(z, 2), Zzf = lp_take(z, 3);
  z = lp_mul<F>(lp_rows(P, U1, Zf, Zf), PP, k);
  const uint32_t PPP = lp_take(z, 0), Q = lp_take(z, 1), ZZ3 = lp_take(z, 2);
  // X3 = R^2 - (PPP + 2Q) (row 0) and Q - X3 = (3Q + PPP) - R^2 (the other
  // rows) in one reduction; one carry pass first brings the limbs of the
  // sums (values below 6p and 8p) under 2^B + 16
  const bool r0 = row4() == 0u;
  const uint32_t Q2 = Q + Q;
  const uint32_t c = lp_carry32<F>(r0 ? PPP + Q2 : Q2 + Q + PPP);
  const uint32_t x = lp_sub<F>(r0 ? RR : c, r0 ? c : RR, k);
  const uint32_t X3 = lp_take(x, 0), T = lp_take(x, 1);
  z = lp_mul<F>(lp_rows(R, S1, Zzf, Zzf), lp_rows(T, PPP, PPP, PPP), k);
  LpPoint<C> O;
  O.X = X3;
  O.Y = lp_sub_y<F>(lp_take(z, 0), lp_take(z, 1), k);
  O.ZZ = ZZ3;
  O.ZZZ = lp_take(z, 2);
  O.inf = false;
  return O;
}

template <class C>
__device__ __forceinline__ LpPoint<C> lp_point_load(const uint32_t* p, const LpK<typename C::F>& k) {
  using F = typename C::F;
  constexpr int CW = F::CW;
  LpPoint<C> P;
  P.X = lp_load<F>(p);
  P.Y = lp_load<F>(p + CW);
  P.ZZ = lp_load<F>(p + 2 * CW);
  P.ZZZ = lp_load<F>(p + 3 * CW);
  P.inf = lp_is_zero<F>(P.ZZ, k);
  return P;
}

// canonical coordinates in the XYZZ storage layout (infinity: ZZ = ZZZ = 0)
template <class C>
__device__ __forceinline__ void lp_point_store(uint32_t* p, const LpPoint<C>& P, const LpK<typename C::F>& k) {
  using F = typename C::F;
  constexpr int CW = F::CW;
  constexpr Words<F::NL> ONE = F::ONE;
  uint32_t X = lp_canonical<F>(P.X, k), Y = lp_canonical<F>(lp_reduce<F>(P.Y, k), k);
  uint32_t ZZ = lp_canonical<F>(P.ZZ, k), ZZZ = lp_canonical<F>(P.ZZZ, k);
  if (P.inf) {
    X = Y = lp_const<F>(ONE);
    ZZ = ZZZ = 0;
  }
  const uint32_t j = threadIdx.x & 63u;
  if (j < uint32_t(F::NL)) {
    p[j] = X;
    p[CW + j] = Y;
    p[2 * CW + j] = ZZ;
    p[3 * CW + j] = ZZZ;
  }
}

// the point as a per-lane XYZZ value with canonical coordinates
template <class C>
__device__ __forceinline__ XYZZ<C> lp_point_to_xyzz(const LpPoint<C>& P, const LpK<typename C::F>& k) {
  using F = typename C::F;
  if (P.inf) return xyzz_inf<C>();
  XYZZ<C> R;
  R.X = lp_to_fp<F>(lp_canonical<F>(P.X, k));
  R.Y = lp_to_fp<F>(lp_canonical<F>(lp_reduce<F>(P.Y, k), k));
  R.ZZ = lp_to_fp<F>(lp_canonical<F>(P.ZZ, k));
  R.ZZZ = lp_to_fp<F>(lp_canonical<F>(P.ZZZ, k));
  return R;
}

}  // namespace eccmi
