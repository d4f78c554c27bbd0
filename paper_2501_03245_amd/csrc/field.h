// Prime-field arithmetic in Montgomery form on 32-bit words (D = 2^32 in the
// notation of Section 2.2), one field element per lane.
//
// Multiplication follows Algorithm 2 (Montgomery multiplication: m^2 word
// products for a*b, then m reduction rows M_i = C_i q_inv mod D, C += M_i q
// D^i, final conditional subtraction with c >= q, not c > q) with its loops
// reordered column by column ("finely integrated product scanning"): each
// output column accumulates its a_i b_j and M_i q_j products in a 96-bit
// accumulator.  On gfx950 each word product is one v_mad_u64_u32 into the low
// 64 bits plus one v_addc_co_u32 of its carry-out into the third word; the
// 2m^2 + m multiply-adds of Section 4.1 are issued exactly once each.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "curves.h"

namespace eccmi {

template <class F>
struct Fp {
  uint32_t w[F::N];
};

template <class F>
__device__ __forceinline__ Fp<F> fp_from(const Words<F::N>& c) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::N; i++) r.w[i] = c.w[i];
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_zero() {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::N; i++) r.w[i] = 0;
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_one() {
  constexpr Words<F::N> one = F::ONE;
  return fp_from<F>(one);
}

template <class F>
__device__ __forceinline__ bool fp_is_zero(const Fp<F>& a) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < F::N; i++) o |= a.w[i];
  return o == 0;
}

template <class F>
__device__ __forceinline__ bool fp_eq(const Fp<F>& a, const Fp<F>& b) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < F::N; i++) o |= a.w[i] ^ b.w[i];
  return o == 0;
}

// ---- carry chains ----------------------------------------------------------
// Carries travel in explicit SGPR-pair lane masks so that the compiler can
// schedule freely without an unseen VCC dependency between statements.

__device__ __forceinline__ uint32_t add_co(uint32_t a, uint32_t b, uint64_t& c) {
  uint32_t r;
  asm("v_add_co_u32_e64 %0, %1, %2, %3" : "=v"(r), "=s"(c) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ uint32_t addc_co(uint32_t a, uint32_t b, uint64_t& c) {
  uint32_t r;
  uint64_t ci = c;
  asm("v_addc_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(r), "=s"(c) : "v"(a), "v"(b), "s"(ci));
  return r;
}
__device__ __forceinline__ uint32_t sub_co(uint32_t a, uint32_t b, uint64_t& c) {
  uint32_t r;
  asm("v_sub_co_u32_e64 %0, %1, %2, %3" : "=v"(r), "=s"(c) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ uint32_t subb_co(uint32_t a, uint32_t b, uint64_t& c) {
  uint32_t r;
  uint64_t ci = c;
  asm("v_subb_co_u32_e64 %0, %1, %2, %3, %4" : "=v"(r), "=s"(c) : "v"(a), "v"(b), "s"(ci));
  return r;
}
// value of the carry for this lane (0 or 1)
__device__ __forceinline__ uint32_t carry_bit(uint64_t c) {
  uint32_t r;
  asm("v_cndmask_b32_e64 %0, 0, 1, %1" : "=v"(r) : "s"(c));
  return r;
}

// r = a - p if a >= p else a, for a < 2p given as N words plus a top carry word
template <class F>
__device__ __forceinline__ void fp_reduce_once(Fp<F>& r, const Fp<F>& a, uint32_t top) {
  constexpr Words<F::N> p = F::P;
  Fp<F> d;
  uint64_t c;
  d.w[0] = sub_co(a.w[0], p.w[0], c);
#pragma unroll
  for (int i = 1; i < F::N; i++) d.w[i] = subb_co(a.w[i], p.w[i], c);
  uint32_t borrow = carry_bit(c);
  // keep a when (top:a) < p, i.e. the subtraction borrowed past the top word
  bool keep = borrow > top;
#pragma unroll
  for (int i = 0; i < F::N; i++) r.w[i] = keep ? a.w[i] : d.w[i];
}

template <class F>
__device__ __forceinline__ Fp<F> fp_add(const Fp<F>& a, const Fp<F>& b) {
  Fp<F> s, r;
  uint64_t c;
  s.w[0] = add_co(a.w[0], b.w[0], c);
#pragma unroll
  for (int i = 1; i < F::N; i++) s.w[i] = addc_co(a.w[i], b.w[i], c);
  fp_reduce_once<F>(r, s, carry_bit(c));
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_sub(const Fp<F>& a, const Fp<F>& b) {
  constexpr Words<F::N> p = F::P;
  Fp<F> d, r;
  uint64_t c;
  d.w[0] = sub_co(a.w[0], b.w[0], c);
#pragma unroll
  for (int i = 1; i < F::N; i++) d.w[i] = subb_co(a.w[i], b.w[i], c);
  // add p back when the subtraction borrowed
  uint32_t mask = 0u - carry_bit(c);
  uint64_t c2;
  r.w[0] = add_co(d.w[0], p.w[0] & mask, c2);
#pragma unroll
  for (int i = 1; i < F::N; i++) r.w[i] = addc_co(d.w[i], p.w[i] & mask, c2);
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_neg(const Fp<F>& a) {
  return fp_sub<F>(fp_zero<F>(), a);
}

template <class F>
__device__ __forceinline__ Fp<F> fp_dbl(const Fp<F>& a) {
  return fp_add<F>(a, a);
}

// ---- Montgomery multiplication ---------------------------------------------

// (t2:acc) += a * b ; a, b in VGPRs
__device__ __forceinline__ void mac_vv(uint64_t& acc, uint32_t& t2, uint32_t a, uint32_t b) {
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
      : "+v"(acc), "+v"(t2)
      : "v"(a), "v"(b)
      : "vcc");
}
// (t2:acc) += a * k ; k a uniform constant held in an SGPR
__device__ __forceinline__ void mac_vs(uint64_t& acc, uint32_t& t2, uint32_t a, uint32_t k) {
  asm("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\t"
      "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
      : "+v"(acc), "+v"(t2)
      : "v"(a), "s"(k)
      : "vcc");
}

// Montgomery product a b R^-1 mod p, canonical output in [0, p) for inputs < p.
template <class F>
__device__ __forceinline__ Fp<F> fp_mul(const Fp<F>& a, const Fp<F>& b) {
  constexpr int N = F::N;
  constexpr Words<N> q = F::P;
  constexpr uint32_t qinv = F::QINV;
  uint32_t m[N];
  Fp<F> r;
  uint64_t acc = 0;
  uint32_t t2 = 0;
#pragma unroll
  for (int k = 0; k < N; k++) {
#pragma unroll
    for (int i = 0; i <= k; i++) mac_vv(acc, t2, a.w[i], b.w[k - i]);
#pragma unroll
    for (int i = 0; i < k; i++) mac_vs(acc, t2, m[i], q.w[k - i]);
    m[k] = uint32_t(acc) * qinv;
    mac_vs(acc, t2, m[k], q.w[0]);  // clears the low word
    acc = (acc >> 32) | (uint64_t(t2) << 32);
    t2 = 0;
  }
#pragma unroll
  for (int k = N; k < 2 * N - 1; k++) {
#pragma unroll
    for (int i = k - N + 1; i < N; i++) mac_vv(acc, t2, a.w[i], b.w[k - i]);
#pragma unroll
    for (int i = k - N + 1; i < N; i++) mac_vs(acc, t2, m[i], q.w[k - i]);
    r.w[k - N] = uint32_t(acc);
    acc = (acc >> 32) | (uint64_t(t2) << 32);
    t2 = 0;
  }
  r.w[N - 1] = uint32_t(acc);
  // value < 2p: one conditional subtraction (the "c >= q" test of Algorithm 2)
  Fp<F> out;
  fp_reduce_once<F>(out, r, uint32_t(acc >> 32));
  return out;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_sqr(const Fp<F>& a) {
  return fp_mul<F>(a, a);
}

template <class F>
__device__ __forceinline__ Fp<F> fp_to_mont(const Fp<F>& a) {
  constexpr Words<F::N> r2 = F::R2;
  return fp_mul<F>(a, fp_from<F>(r2));
}

template <class F>
__device__ __forceinline__ Fp<F> fp_from_mont(const Fp<F>& a) {
  Fp<F> one = fp_zero<F>();
  one.w[0] = 1;
  return fp_mul<F>(a, one);
}

// canonical check: a < p
template <class F>
__device__ __forceinline__ bool fp_lt_p(const Fp<F>& a) {
  constexpr Words<F::N> p = F::P;
  uint64_t c;
  (void)sub_co(a.w[0], p.w[0], c);
#pragma unroll
  for (int i = 1; i < F::N; i++) (void)subb_co(a.w[i], p.w[i], c);
  return carry_bit(c) != 0;
}

// ---- loads and stores of array-of-structures elements ---------------------
// An element is N consecutive 32-bit words; N is a multiple of 4, so it is
// moved as N/4 16-byte vectors.

template <class F>
__device__ __forceinline__ Fp<F> fp_load(const uint32_t* __restrict__ p) {
  Fp<F> r;
  const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int i = 0; i < F::N / 4; i++) {
    uint4 t = v[i];
    r.w[4 * i] = t.x;
    r.w[4 * i + 1] = t.y;
    r.w[4 * i + 2] = t.z;
    r.w[4 * i + 3] = t.w;
  }
  return r;
}

template <class F>
__device__ __forceinline__ void fp_store(uint32_t* __restrict__ p, const Fp<F>& a) {
  uint4* v = reinterpret_cast<uint4*>(p);
#pragma unroll
  for (int i = 0; i < F::N / 4; i++) v[i] = make_uint4(a.w[4 * i], a.w[4 * i + 1], a.w[4 * i + 2], a.w[4 * i + 3]);
}

// structure-of-arrays access: word i of element e lives at p[i * stride + e]
template <class F>
__device__ __forceinline__ Fp<F> fp_load_soa(const uint32_t* __restrict__ p, size_t stride) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::N; i++) r.w[i] = p[i * stride];
  return r;
}

template <class F>
__device__ __forceinline__ void fp_store_soa(uint32_t* __restrict__ p, size_t stride, const Fp<F>& a) {
#pragma unroll
  for (int i = 0; i < F::N; i++) p[i * stride] = a.w[i];
}

}  // namespace eccmi
