// Point representations used on the device.
//
// * Affine (x, y) in Montgomery form: the form of the batched additions of
//   Section 3 (Eqns 2-3 and the tangent slope for doubling).  Stored points
//   are canonical and use the sentinel x = all-ones limbs for the point at
//   infinity: no normalised limb has its top bit set.
// * XYZZ (X, Y, ZZ, ZZZ) with x = X/ZZ, y = Y/ZZZ and ZZ^3 = ZZZ^2, used where
//   additions form a dependent chain and cannot be batched (bucket reduction,
//   window combination, per-lane scalar multiplication).  Formulas are the
//   published ones for this system (add-2008-s, madd-2008-s, dbl-2008-s-1 of
//   the Explicit-Formulas Database), written out below with their special
//   cases.  XYZZ coordinates are semi-reduced.
//
// Storage: a coordinate takes F::CW words; an affine point 2 CW, an XYZZ
// point 4 CW.
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

template <class C>
constexpr int affine_words() {
  return 2 * C::F::CW;
}
template <class C>
constexpr int xyzz_words() {
  return 4 * C::F::CW;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_inf_marker() {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = 0xffffffffu;
  return r;
}

// a stored (normalised) coordinate never has bit 31 set in its first limb
template <class F>
__device__ __forceinline__ bool fp_is_inf_marker(const Fp<F>& x) {
  return (x.w[0] >> 31) != 0;
}

// p - y for canonical 0 < y < p: canonical
template <class F>
__device__ __forceinline__ Fp<F> fp_neg_canonical(const Fp<F>& y) {
  constexpr Words<F::NL> p = F::P;
  Fp<F> r;
  int32_t br = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    int32_t v = int32_t(p.w[i]) - int32_t(y.w[i]) + br;
    br = v >> F::B;
    r.w[i] = uint32_t(v) & F::MASK;
  }
  return r;
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

// 3 x^2 + a zz^2 (a = 0 or -3), semi-reduced; for a = -3 it is
// 3 (x - zz)(x + zz), one product instead of two squarings
template <class C>
__device__ __forceinline__ Fp<typename C::F> tangent_numerator(const Fp<typename C::F>& x,
                                                               const Fp<typename C::F>& zz) {
  using F = typename C::F;
  Fp<F> t;
  if constexpr (C::A_IS_MINUS3) {
    t = fp_mul<F>(fp_add<F>(x, zz), fp_sub_lazy<F>(x, zz));
  } else {
    t = fp_sqr<F>(x);
  }
  return fp_add<F>(fp_add<F>(t, t), t);
}

// dbl-2008-s-1: U = 2Y, V = U^2, W = U V, S = X V, M = 3X^2 + a ZZ^2,
// X3 = M^2 - 2S, Y3 = M (S - X3) - W Y, ZZ3 = V ZZ, ZZZ3 = W ZZZ.
template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_dbl_in(const XYZZ<C>& P) {
  using F = typename C::F;
  if (xyzz_is_inf<C>(P)) return P;
  Fp<F> U = fp_dbl<F>(P.Y);
  Fp<F> V = fp_sqr<F>(U);
  Fp<F> W = fp_mul<F>(U, V);
  Fp<F> S = fp_mul<F>(P.X, V);
  Fp<F> M = tangent_numerator<C>(P.X, P.ZZ);
  XYZZ<C> R;
  R.X = fp_sub<F>(fp_sqr<F>(M), fp_dbl<F>(S));
  R.Y = fp_sub<F>(fp_mul<F>(M, fp_sub_lazy<F>(S, R.X)), fp_mul<F>(W, P.Y));
  R.ZZ = fp_mul<F>(V, P.ZZ);
  R.ZZZ = fp_mul<F>(W, P.ZZZ);
  return R;
}

template <class C>
__device__ __noinline__ XYZZ<C> xyzz_dbl(const XYZZ<C>& P) {
  return xyzz_dbl_in<C>(P);
}

// madd-2008-s: P (XYZZ) + Q (affine, ZZ = ZZZ = 1):
// U2 = X2 ZZ1, S2 = Y2 ZZZ1, P = U2 - X1, R = S2 - Y1, PP = P^2, PPP = P PP,
// Q = X1 PP, X3 = R^2 - PPP - 2Q, Y3 = R (Q - X3) - Y1 PPP, ZZ3 = ZZ1 PP,
// ZZZ3 = ZZZ1 PPP.
template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_add_affine_in(const XYZZ<C>& A, const Affine<C>& B) {
  using F = typename C::F;
  if (fp_is_inf_marker<F>(B.x)) return A;
  if (xyzz_is_inf<C>(A)) return xyzz_from_affine<C>(B);
  Fp<F> U2 = fp_mul<F>(B.x, A.ZZ);
  Fp<F> S2 = fp_mul<F>(B.y, A.ZZZ);
  Fp<F> P = fp_sub<F>(U2, A.X);
  Fp<F> R = fp_sub<F>(S2, A.Y);
  bool dbl = false;
  if (fp_is_zero<F>(P)) {
    if (!fp_is_zero<F>(R)) return xyzz_inf<C>();
    // A = B: dbl-2008-s-1 is this tail with P = 2 Y1 (PP = V, PPP = W,
    // Q = S), R = M = 3 X1^2 + a ZZ1^2, and no PPP term in X3
    dbl = true;
    P = fp_dbl<F>(A.Y);
    R = tangent_numerator<C>(A.X, A.ZZ);
  }
  Fp<F> PP = fp_sqr<F>(P);
  Fp<F> PPP = fp_mul<F>(P, PP);
  Fp<F> Q = fp_mul<F>(A.X, PP);
  XYZZ<C> O;
  Fp<F> RR = fp_sqr<F>(R);
  if (!dbl) RR = fp_sub<F>(RR, PPP);
  O.X = fp_sub<F>(RR, fp_dbl<F>(Q));
  O.Y = fp_sub<F>(fp_mul<F>(R, fp_sub_lazy<F>(Q, O.X)), fp_mul<F>(A.Y, PPP));
  O.ZZ = fp_mul<F>(A.ZZ, PP);
  O.ZZZ = fp_mul<F>(A.ZZZ, PPP);
  return O;
}

template <class C>
__device__ __noinline__ XYZZ<C> xyzz_add_affine(const XYZZ<C>& A, const Affine<C>& B) {
  return xyzz_add_affine_in<C>(A, B);
}

// add-2008-s: U1 = X1 ZZ2, U2 = X2 ZZ1, S1 = Y1 ZZZ2, S2 = Y2 ZZZ1,
// P = U2 - U1, R = S2 - S1, PP = P^2, PPP = P PP, Q = U1 PP,
// X3 = R^2 - PPP - 2Q, Y3 = R (Q - X3) - S1 PPP, ZZ3 = ZZ1 ZZ2 PP,
// ZZZ3 = ZZZ1 ZZZ2 PPP.
template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_add_in(const XYZZ<C>& A, const XYZZ<C>& B) {
  using F = typename C::F;
  if (xyzz_is_inf<C>(A)) return B;
  if (xyzz_is_inf<C>(B)) return A;
  Fp<F> U1 = fp_mul<F>(A.X, B.ZZ);
  Fp<F> U2 = fp_mul<F>(B.X, A.ZZ);
  Fp<F> S1 = fp_mul<F>(A.Y, B.ZZZ);
  Fp<F> S2 = fp_mul<F>(B.Y, A.ZZZ);
  Fp<F> P = fp_sub<F>(U2, U1);
  Fp<F> R = fp_sub<F>(S2, S1);
  Fp<F> Zf, Zzf;  // the factors of ZZ3 / PP and ZZZ3 / PPP
  bool dbl = false;
  if (fp_is_zero<F>(P)) {
    if (!fp_is_zero<F>(R)) return xyzz_inf<C>();
    // A = B: dbl-2008-s-1 of A is this tail with U1 = X1, S1 = Y1,
    // P = 2 Y1, R = M = 3 X1^2 + a ZZ1^2, no PPP term in X3, and ZZ1, ZZZ1
    // as the factors of ZZ3 and ZZZ3
    dbl = true;
    U1 = A.X;
    S1 = A.Y;
    P = fp_dbl<F>(A.Y);
    R = tangent_numerator<C>(A.X, A.ZZ);
    Zf = A.ZZ;
    Zzf = A.ZZZ;
  } else {
    Zf = fp_mul<F>(A.ZZ, B.ZZ);
    Zzf = fp_mul<F>(A.ZZZ, B.ZZZ);
  }
  Fp<F> PP = fp_sqr<F>(P);
  Fp<F> PPP = fp_mul<F>(P, PP);
  Fp<F> Q = fp_mul<F>(U1, PP);
  XYZZ<C> O;
  Fp<F> RR = fp_sqr<F>(R);
  if (!dbl) RR = fp_sub<F>(RR, PPP);
  O.X = fp_sub<F>(RR, fp_dbl<F>(Q));
  O.Y = fp_sub<F>(fp_mul<F>(R, fp_sub_lazy<F>(Q, O.X)), fp_mul<F>(S1, PPP));
  O.ZZ = fp_mul<F>(Zf, PP);
  O.ZZZ = fp_mul<F>(Zzf, PPP);
  return O;
}

template <class C>
__device__ __noinline__ XYZZ<C> xyzz_add(const XYZZ<C>& A, const XYZZ<C>& B) {
  return xyzz_add_in<C>(A, B);
}

template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_neg(const XYZZ<C>& A) {
  XYZZ<C> r = A;
  r.Y = fp_neg<typename C::F>(A.Y);
  return r;
}

// The _in forms are inlined where a chain of point operations is hot and
// latency-bound (the bucket reduction): a call with points passed by value
// would move most of them through the stack.  The plain forms are separate
// functions that keep code size down elsewhere.

// ---- one wave evaluating one chain of point operations ----------------------
// The operands below are wave-uniform; the independent products of each step
// of a formula run on different lanes (lane k computes product k) and are
// read back into every lane, so a formula costs one product latency per level
// of its dependency graph rather than one per product.

template <class F, int K>
__device__ __forceinline__ void par_mul(const Fp<F> (&a)[K], const Fp<F> (&b)[K], Fp<F> (&r)[K]) {
  const int lane = threadIdx.x & 63;
  Fp<F> x = a[0], y = b[0];
#pragma unroll
  for (int k = 1; k < K; k++) {
#pragma unroll
    for (int i = 0; i < F::NL; i++) {
      x.w[i] = lane == k ? a[k].w[i] : x.w[i];
      y.w[i] = lane == k ? b[k].w[i] : y.w[i];
    }
  }
  Fp<F> z = fp_mul<F>(x, y);
  // read back through the lane crossbar rather than into scalar registers:
  // the following additions and subtractions then stay on the vector unit,
  // where a 14-limb carry chain is several times faster than on the scalar one
#pragma unroll
  for (int k = 0; k < K; k++) {
#pragma unroll
    for (int i = 0; i < F::NL; i++) r[k].w[i] = __shfl(z.w[i], k, 64);
  }
}

// dbl-2008-s-1 in three product levels:
// [U^2, X^2 (, ZZ^2)] -> [U V, X V, V ZZ, M^2] -> [W Y, W ZZZ, M (S - X3)]
template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_dbl_wave(const XYZZ<C>& P) {
  using F = typename C::F;
  if (xyzz_is_inf<C>(P)) return P;
  Fp<F> U = fp_dbl<F>(P.Y);
  Fp<F> M;
  Fp<F> V;
  if constexpr (C::A_IS_MINUS3) {
    Fp<F> r1[3];
    par_mul<F, 3>({U, P.X, P.ZZ}, {U, P.X, P.ZZ}, r1);
    V = r1[0];
    M = fp_sub<F>(fp_add<F>(fp_add<F>(r1[1], r1[1]), r1[1]), fp_add<F>(fp_add<F>(r1[2], r1[2]), r1[2]));
  } else {
    Fp<F> r1[2];
    par_mul<F, 2>({U, P.X}, {U, P.X}, r1);
    V = r1[0];
    M = fp_add<F>(fp_add<F>(r1[1], r1[1]), r1[1]);
  }
  Fp<F> r2[4];
  par_mul<F, 4>({U, P.X, V, M}, {V, V, P.ZZ, M}, r2);
  const Fp<F> W = r2[0], S = r2[1];
  XYZZ<C> R;
  R.ZZ = r2[2];
  R.X = fp_sub<F>(r2[3], fp_dbl<F>(S));
  Fp<F> r3[3];
  par_mul<F, 3>({W, W, M}, {P.Y, P.ZZZ, fp_sub<F>(S, R.X)}, r3);
  R.ZZZ = r3[1];
  R.Y = fp_sub<F>(r3[2], r3[0]);
  return R;
}

// add-2008-s in four product levels:
// [X1 ZZ2, X2 ZZ1, Y1 ZZZ2, Y2 ZZZ1, ZZ1 ZZ2, ZZZ1 ZZZ2] -> [P^2, R^2]
// -> [P PP, U1 PP, ZZ1 ZZ2 PP] -> [S1 PPP, R (Q - X3), ZZZ1 ZZZ2 PPP]
template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_add_wave(const XYZZ<C>& A, const XYZZ<C>& B) {
  using F = typename C::F;
  if (xyzz_is_inf<C>(A)) return B;
  if (xyzz_is_inf<C>(B)) return A;
  Fp<F> r1[6];
  par_mul<F, 6>({A.X, B.X, A.Y, B.Y, A.ZZ, A.ZZZ}, {B.ZZ, A.ZZ, B.ZZZ, A.ZZZ, B.ZZ, B.ZZZ}, r1);
  const Fp<F> U1 = r1[0], S1 = r1[2];
  Fp<F> P = fp_sub<F>(r1[1], U1);
  Fp<F> R = fp_sub<F>(r1[3], S1);
  if (fp_is_zero<F>(P)) {
    if (fp_is_zero<F>(R)) return xyzz_dbl_wave<C>(A);
    return xyzz_inf<C>();
  }
  Fp<F> r2[2];
  par_mul<F, 2>({P, R}, {P, R}, r2);
  const Fp<F> PP = r2[0];
  Fp<F> r3[3];
  par_mul<F, 3>({P, U1, r1[4]}, {PP, PP, PP}, r3);
  const Fp<F> PPP = r3[0], Q = r3[1];
  XYZZ<C> O;
  O.ZZ = r3[2];
  O.X = fp_sub<F>(fp_sub<F>(r2[1], PPP), fp_dbl<F>(Q));
  Fp<F> r4[3];
  par_mul<F, 3>({S1, R, r1[5]}, {PPP, fp_sub<F>(Q, O.X), PPP}, r4);
  O.ZZZ = r4[2];
  O.Y = fp_sub<F>(r4[1], r4[0]);
  return O;
}

// Normalise to canonical affine on one wave-uniform value: one inversion of
// ZZ ZZZ.  Infinity becomes the marker.
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
  Fp<F> izz = fp_mul<F>(t, P.ZZZ);  // 1/ZZ
  Fp<F> izzz = fp_mul<F>(t, P.ZZ);  // 1/ZZZ
  a.x = fp_canonical<F>(fp_mul<F>(P.X, izz));
  a.y = fp_canonical<F>(fp_mul<F>(P.Y, izzz));
  return a;
}

template <class C>
__device__ __forceinline__ void xyzz_store(uint32_t* __restrict__ p, const XYZZ<C>& P) {
  using F = typename C::F;
  constexpr int CW = F::CW;
  fp_store<F>(p, P.X);
  fp_store<F>(p + CW, P.Y);
  fp_store<F>(p + 2 * CW, P.ZZ);
  fp_store<F>(p + 3 * CW, P.ZZZ);
}

template <class C>
__device__ __forceinline__ XYZZ<C> xyzz_load(const uint32_t* __restrict__ p) {
  using F = typename C::F;
  constexpr int CW = F::CW;
  XYZZ<C> P;
  P.X = fp_load<F>(p);
  P.Y = fp_load<F>(p + CW);
  P.ZZ = fp_load<F>(p + 2 * CW);
  P.ZZZ = fp_load<F>(p + 3 * CW);
  return P;
}

template <class C>
__device__ __forceinline__ Affine<C> affine_load(const uint32_t* __restrict__ p) {
  using F = typename C::F;
  Affine<C> a;
  a.x = fp_load<F>(p);
  a.y = fp_load<F>(p + F::CW);
  return a;
}

template <class C>
__device__ __forceinline__ void affine_store(uint32_t* __restrict__ p, const Affine<C>& a) {
  using F = typename C::F;
  fp_store<F>(p, a.x);
  fp_store<F>(p + F::CW, a.y);
}

// y^2 == x^3 + a x + b (Montgomery-form coordinates, semi-reduced)
template <class C>
__device__ __forceinline__ bool affine_on_curve(const Affine<C>& P) {
  using F = typename C::F;
  constexpr Words<F::NL> b = C::B_MONT;
  Fp<F> lhs = fp_sqr<F>(P.y);
  Fp<F> rhs = fp_mul<F>(fp_sqr<F>(P.x), P.x);
  if constexpr (C::A_IS_MINUS3) {
    rhs = fp_sub<F>(rhs, fp_add<F>(fp_add<F>(P.x, P.x), P.x));
  }
  rhs = fp_add<F>(rhs, fp_from<F>(b));
  return fp_eq<F>(lhs, rhs);
}

}  // namespace eccmi
