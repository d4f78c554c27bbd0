// Single-lane field inversion for the "apply" step of the batch inversion
// (Section 3.2).  Section 2.2 names two methods: Fermat (x^(q-2), branch-free,
// hundreds of multiplications) and binary extended Euclid (about three times
// faster but branchy, hence avoided there for data-parallel lanes).  Here the
// inversion runs once per workgroup on wave-uniform values, so branching costs
// nothing and the binary method is used: written over wave-uniform operands it
// compiles to scalar-unit instructions and leaves the vector unit to the other
// waves on the compute unit.
#pragma once
#include "field.h"

namespace eccmi {

template <int N>
struct UInt {
  uint32_t w[N];
};

template <int N>
__device__ __forceinline__ bool ui_is_one(const UInt<N>& a) {
  uint32_t o = a.w[0] ^ 1u;
#pragma unroll
  for (int i = 1; i < N; i++) o |= a.w[i];
  return o == 0;
}

template <int N>
__device__ __forceinline__ bool ui_ge(const UInt<N>& a, const UInt<N>& b) {
  // a >= b  <=>  a - b does not borrow
  uint32_t br = 0;
#pragma unroll
  for (int i = 0; i < N; i++) {
    uint64_t d = uint64_t(a.w[i]) - b.w[i] - br;
    br = uint32_t(d >> 63);
  }
  return br == 0;
}

template <int N>
__device__ __forceinline__ void ui_sub(UInt<N>& a, const UInt<N>& b) {
  uint32_t br = 0;
#pragma unroll
  for (int i = 0; i < N; i++) {
    uint64_t d = uint64_t(a.w[i]) - b.w[i] - br;
    a.w[i] = uint32_t(d);
    br = uint32_t(d >> 63);
  }
}

template <int N>
__device__ __forceinline__ void ui_shr1(UInt<N>& a, uint32_t top) {
#pragma unroll
  for (int i = 0; i < N - 1; i++) a.w[i] = (a.w[i] >> 1) | (a.w[i + 1] << 31);
  a.w[N - 1] = (a.w[N - 1] >> 1) | (top << 31);
}

// x / 2 mod p for x < p
template <class F>
__device__ __forceinline__ void ui_half_mod(UInt<F::N>& x) {
  constexpr int N = F::N;
  constexpr Words<N> p = F::P;
  if (x.w[0] & 1u) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < N; i++) {
      uint64_t s = uint64_t(x.w[i]) + p.w[i] + c;
      x.w[i] = uint32_t(s);
      c = uint32_t(s >> 32);
    }
    ui_shr1<N>(x, c);
  } else {
    ui_shr1<N>(x, 0);
  }
}

// x - y mod p for x, y < p
template <class F>
__device__ __forceinline__ void ui_sub_mod(UInt<F::N>& x, const UInt<F::N>& y) {
  constexpr int N = F::N;
  constexpr Words<N> p = F::P;
  uint32_t br = 0;
#pragma unroll
  for (int i = 0; i < N; i++) {
    uint64_t d = uint64_t(x.w[i]) - y.w[i] - br;
    x.w[i] = uint32_t(d);
    br = uint32_t(d >> 63);
  }
  if (br) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < N; i++) {
      uint64_t s = uint64_t(x.w[i]) + p.w[i] + c;
      x.w[i] = uint32_t(s);
      c = uint32_t(s >> 32);
    }
  }
}

template <int N>
__device__ __forceinline__ bool ui_is_zero(const UInt<N>& a) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < N; i++) o |= a.w[i];
  return o == 0;
}

// a^-1 mod p for 0 < a < p (plain integers, no Montgomery factor); 0 for
// a = 0.  Binary extended Euclid with invariants x1 a = u and x2 a = v
// (mod p).  Every subtraction of two odd values is followed by at least one
// halving, so at most 2 * 32N rounds run; the bound also ends the loop for
// inputs outside [1, p), whose result is then meaningless but finite.
template <class F>
__device__ UInt<F::N> ui_inverse(const UInt<F::N>& a) {
  constexpr int N = F::N;
  constexpr Words<N> pw = F::P;
  UInt<N> u = a, v, x1, x2;
#pragma unroll
  for (int i = 0; i < N; i++) {
    v.w[i] = pw.w[i];
    x1.w[i] = 0;
    x2.w[i] = 0;
  }
  if (ui_is_zero<N>(u)) return x1;
  x1.w[0] = 1;
  for (int round = 0; round < 2 * 32 * N + 8; round++) {
    if (ui_is_one<N>(u) || ui_is_one<N>(v) || ui_is_zero<N>(u) || ui_is_zero<N>(v)) break;
    while ((u.w[0] & 1u) == 0 && !ui_is_zero<N>(u)) {
      ui_shr1<N>(u, 0);
      ui_half_mod<F>(x1);
    }
    while ((v.w[0] & 1u) == 0 && !ui_is_zero<N>(v)) {
      ui_shr1<N>(v, 0);
      ui_half_mod<F>(x2);
    }
    if (ui_ge<N>(u, v)) {
      ui_sub<N>(u, v);
      ui_sub_mod<F>(x1, x2);
    } else {
      ui_sub<N>(v, u);
      ui_sub_mod<F>(x2, x1);
    }
  }
  return ui_is_one<N>(u) ? x1 : x2;
}

// Inverse of a Montgomery-form element x R (x != 0), returned as x^-1 R:
// the binary method gives (x R)^-1 = x^-1 R^-1, and one Montgomery product with
// R^3 restores the factor: x^-1 R^-1 R^3 R^-1 = x^-1 R.
template <class F>
__device__ __noinline__ Fp<F> fp_inv_uniform(const Fp<F>& xr) {
  constexpr int N = F::N;
  UInt<N> a;
#pragma unroll
  for (int i = 0; i < N; i++) a.w[i] = __builtin_amdgcn_readfirstlane(xr.w[i]);
  UInt<N> ia = ui_inverse<F>(a);
  Fp<F> t;
#pragma unroll
  for (int i = 0; i < N; i++) t.w[i] = ia.w[i];
  constexpr Words<N> r3 = F::R3;
  return fp_mul<F>(t, fp_from<F>(r3));
}

}  // namespace eccmi
