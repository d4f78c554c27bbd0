// Point representations used on the device.
//
// * Affine (x, y) in Montgomery form: the form of the batched additions of
//   Section 3 (Eqns 2-3 and the tangent slope for doubling).  Stored points
//   use the sentinel x = all-ones words for the point at infinity: it is not a
//   canonical coordinate (every prime here is below 2^(32N) - 1).
// * XYZZ (X, Y, ZZ, ZZZ) with x = X/ZZ, y = Y/ZZZ and ZZ^3 = ZZZ^2, used where
//   additions form a dependent chain and cannot be batched (bucket reduction,
//   window combination, per-lane scalar multiplication).  Formulas are the
//   published ones for this system (add-2008-s, madd-2008-s, dbl-2008-s-1 of
//   the Explicit-Formulas Database), written out below with their special
//   cases.
#pragma once
#include "field.h"
#include "inverse.h"

namespace eccmi {

template <class C>
struct Affine {
  Fp<typename C::F> x, y;
};

template <class C>
struct XYZZ {
  Fp<typename C::F> X, Y, ZZ, ZZZ;  // ZZ = 0 encodes the point at infinity
};

template <class F>
__device__ __forceinline__ Fp<F> fp_inf_marker() {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::N; i++) r.w[i] = 0xffffffffu;
  return r;
}

template <class F>
__device__ __forceinline__ bool fp_is_inf_marker(const Fp<F>& x) {
  uint32_t a = 0xffffffffu;
#pragma unroll
  for (int i = 0; i < F::N; i++) a &= x.w[i];
  return a == 0xffffffffu;
}

template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_inf() {
  using F = typename C::F;
  XYZZ<C> r;
  r.X = fp_one<F>();
  r.Y = fp_one<F>();
  r.ZZ = fp_zero<F>();
  r.ZZZ = fp_zero<F>();
  return r;
}

template <class C>
__device__ __forceinline__ bool xyzz_is_inf(const XYZZ<C>& P) {
  return fp_is_zero<typename C::F>(P.ZZ);
}

template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_from_affine(const Affine<C>& a) {
  using F = typename C::F;
  if (fp_is_inf_marker<F>(a.x)) return xyzz_inf<C>();
  XYZZ<C> r;
  r.X = a.x;
  r.Y = a.y;
  r.ZZ = fp_one<F>();
  r.ZZZ = fp_one<F>();
  return r;
}

// 3 x^2 + a zz^2 (a = 0 or -3)
template <class C>
__device__ __forceinline__ Fp<typename C::F> tangent_numerator(const Fp<typename C::F>& x,
                                                               const Fp<typename C::F>& zz) {
  using F = typename C::F;
  Fp<F> xx = fp_sqr<F>(x);
  Fp<F> m = fp_add<F>(fp_add<F>(xx, xx), xx);
  if constexpr (C::A_IS_MINUS3) {
    Fp<F> z4 = fp_sqr<F>(zz);
    Fp<F> t = fp_add<F>(fp_add<F>(z4, z4), z4);
    m = fp_sub<F>(m, t);
  }
  return m;
}

// dbl-2008-s-1: U = 2Y, V = U^2, W = U V, S = X V, M = 3X^2 + a ZZ^2,
// X3 = M^2 - 2S, Y3 = M (S - X3) - W Y, ZZ3 = V ZZ, ZZZ3 = W ZZZ.
template <class C>
__device__ __noinline__ XYZZ<C> xyzz_dbl(const XYZZ<C>& P) {
  using F = typename C::F;
  if (xyzz_is_inf<C>(P)) return P;
  Fp<F> U = fp_dbl<F>(P.Y);
  Fp<F> V = fp_sqr<F>(U);
  Fp<F> W = fp_mul<F>(U, V);
  Fp<F> S = fp_mul<F>(P.X, V);
  Fp<F> M = tangent_numerator<C>(P.X, P.ZZ);
  XYZZ<C> R;
  R.X = fp_sub<F>(fp_sqr<F>(M), fp_dbl<F>(S));
  R.Y = fp_sub<F>(fp_mul<F>(M, fp_sub<F>(S, R.X)), fp_mul<F>(W, P.Y));
  R.ZZ = fp_mul<F>(V, P.ZZ);
  R.ZZZ = fp_mul<F>(W, P.ZZZ);
  return R;
}

// madd-2008-s: P (XYZZ) + Q (affine, ZZ = ZZZ = 1):
// U2 = X2 ZZ1, S2 = Y2 ZZZ1, P = U2 - X1, R = S2 - Y1, PP = P^2, PPP = P PP,
// Q = X1 PP, X3 = R^2 - PPP - 2Q, Y3 = R (Q - X3) - Y1 PPP, ZZ3 = ZZ1 PP,
// ZZZ3 = ZZZ1 PPP.
template <class C>
__device__ __noinline__ XYZZ<C> xyzz_add_affine(const XYZZ<C>& A, const Affine<C>& B) {
  using F = typename C::F;
  if (fp_is_inf_marker<F>(B.x)) return A;
  if (xyzz_is_inf<C>(A)) return xyzz_from_affine<C>(B);
  Fp<F> U2 = fp_mul<F>(B.x, A.ZZ);
  Fp<F> S2 = fp_mul<F>(B.y, A.ZZZ);
  Fp<F> P = fp_sub<F>(U2, A.X);
  Fp<F> R = fp_sub<F>(S2, A.Y);
  if (fp_is_zero<F>(P)) {
    if (fp_is_zero<F>(R)) return xyzz_dbl<C>(A);
    return xyzz_inf<C>();
  }
  Fp<F> PP = fp_sqr<F>(P);
  Fp<F> PPP = fp_mul<F>(P, PP);
  Fp<F> Q = fp_mul<F>(A.X, PP);
  XYZZ<C> O;
  O.X = fp_sub<F>(fp_sub<F>(fp_sqr<F>(R), PPP), fp_dbl<F>(Q));
  O.Y = fp_sub<F>(fp_mul<F>(R, fp_sub<F>(Q, O.X)), fp_mul<F>(A.Y, PPP));
  O.ZZ = fp_mul<F>(A.ZZ, PP);
  O.ZZZ = fp_mul<F>(A.ZZZ, PPP);
  return O;
}

// add-2008-s: U1 = X1 ZZ2, U2 = X2 ZZ1, S1 = Y1 ZZZ2, S2 = Y2 ZZZ1,
// P = U2 - U1, R = S2 - S1, PP = P^2, PPP = P PP, Q = U1 PP,
// X3 = R^2 - PPP - 2Q, Y3 = R (Q - X3) - S1 PPP, ZZ3 = ZZ1 ZZ2 PP,
// ZZZ3 = ZZZ1 ZZZ2 PPP.
template <class C>
__device__ __noinline__ XYZZ<C> xyzz_add(const XYZZ<C>& A, const XYZZ<C>& B) {
  using F = typename C::F;
  if (xyzz_is_inf<C>(A)) return B;
  if (xyzz_is_inf<C>(B)) return A;
  Fp<F> U1 = fp_mul<F>(A.X, B.ZZ);
  Fp<F> U2 = fp_mul<F>(B.X, A.ZZ);
  Fp<F> S1 = fp_mul<F>(A.Y, B.ZZZ);
  Fp<F> S2 = fp_mul<F>(B.Y, A.ZZZ);
  Fp<F> P = fp_sub<F>(U2, U1);
  Fp<F> R = fp_sub<F>(S2, S1);
  if (fp_is_zero<F>(P)) {
    if (fp_is_zero<F>(R)) return xyzz_dbl<C>(A);
    return xyzz_inf<C>();
  }
  Fp<F> PP = fp_sqr<F>(P);
  Fp<F> PPP = fp_mul<F>(P, PP);
  Fp<F> Q = fp_mul<F>(U1, PP);
  XYZZ<C> O;
  O.X = fp_sub<F>(fp_sub<F>(fp_sqr<F>(R), PPP), fp_dbl<F>(Q));
  O.Y = fp_sub<F>(fp_mul<F>(R, fp_sub<F>(Q, O.X)), fp_mul<F>(S1, PPP));
  O.ZZ = fp_mul<F>(fp_mul<F>(A.ZZ, B.ZZ), PP);
  O.ZZZ = fp_mul<F>(fp_mul<F>(A.ZZZ, B.ZZZ), PPP);
  return O;
}

template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_neg(const XYZZ<C>& A) {
  XYZZ<C> r = A;
  r.Y = fp_neg<typename C::F>(A.Y);
  return r;
}

// k P for a small non-negative integer k (double-and-add from the top bit)
template <class C>
__device__ __noinline__ XYZZ<C> xyzz_mul_small(const XYZZ<C>& P, uint32_t k) {
  XYZZ<C> acc = xyzz_inf<C>();
  for (int b = 31; b >= 0; b--) {
    acc = xyzz_dbl<C>(acc);
    if ((k >> b) & 1u) acc = xyzz_add<C>(acc, P);
  }
  return acc;
}

// Normalise to affine on one wave-uniform value: one inversion of ZZ ZZZ.
template <class C>
__device__ __noinline__ Affine<C> xyzz_to_affine_uniform(const XYZZ<C>& P) {
  using F = typename C::F;
  Affine<C> a;
  if (xyzz_is_inf<C>(P)) {
    a.x = fp_inf_marker<F>();
    a.y = fp_zero<F>();
    return a;
  }
  Fp<F> t = fp_inv_uniform<F>(fp_mul<F>(P.ZZ, P.ZZZ));
  Fp<F> izz = fp_mul<F>(t, P.ZZZ);   // 1/ZZ
  Fp<F> izzz = fp_mul<F>(t, P.ZZ);   // 1/ZZZ
  a.x = fp_mul<F>(P.X, izz);
  a.y = fp_mul<F>(P.Y, izzz);
  return a;
}

template <class C>
__device__ __forceinline__ void xyzz_store(uint32_t* __restrict__ p, const XYZZ<C>& P) {
  using F = typename C::F;
  constexpr int N = F::N;
  fp_store<F>(p, P.X);
  fp_store<F>(p + N, P.Y);
  fp_store<F>(p + 2 * N, P.ZZ);
  fp_store<F>(p + 3 * N, P.ZZZ);
}

template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_load(const uint32_t* __restrict__ p) {
  using F = typename C::F;
  constexpr int N = F::N;
  XYZZ<C> P;
  P.X = fp_load<F>(p);
  P.Y = fp_load<F>(p + N);
  P.ZZ = fp_load<F>(p + 2 * N);
  P.ZZZ = fp_load<F>(p + 3 * N);
  return P;
}

template <class C>
__device__ __forceinline__ Affine<C> affine_load(const uint32_t* __restrict__ p) {
  using F = typename C::F;
  Affine<C> a;
  a.x = fp_load<F>(p);
  a.y = fp_load<F>(p + F::N);
  return a;
}

template <class C>
__device__ __forceinline__ void affine_store(uint32_t* __restrict__ p, const Affine<C>& a) {
  using F = typename C::F;
  fp_store<F>(p, a.x);
  fp_store<F>(p + F::N, a.y);
}

// y^2 == x^3 + a x + b (Montgomery-form coordinates)
template <class C>
__device__ __forceinline__ bool affine_on_curve(const Affine<C>& P) {
  using F = typename C::F;
  constexpr Words<F::N> b = C::B_MONT;
  Fp<F> lhs = fp_sqr<F>(P.y);
  Fp<F> rhs = fp_mul<F>(fp_sqr<F>(P.x), P.x);
  if constexpr (C::A_IS_MINUS3) {
    rhs = fp_sub<F>(rhs, fp_add<F>(fp_add<F>(P.x, P.x), P.x));
  }
  rhs = fp_add<F>(rhs, fp_from<F>(b));
  return fp_eq<F>(lhs, rhs);
}

}  // namespace eccmi
