// Prime-field arithmetic in Montgomery form, one field element per lane.
//
// Working form: NL limbs of B bits (B = 28 or 29) held in 32-bit registers,
// R = 2^(B NL).  Section 2.2 writes an element as sum x_i D^i with D a machine
// word; here D = 2^B is kept below the register width so that every word
// product (at most 2^58..2^62) and every column of Algorithm 2 fits a 64-bit
// accumulator.  Each product is then a single v_mad_u64_u32 into that
// accumulator with no carry flag: on gfx950 the carry-out form of the VALU
// (VOP3b) issues at about half the rate of a plain multiply-add and needs
// wait states before its carry is read, so a carry-free column beats the
// 2^32 radix despite the extra limb products.
//
// Multiplication is Algorithm 2 (integer product, then reduction rows
// M_i = C_i q_inv mod D and C += M_i q D^i, then a conditional subtraction)
// with its two loops interleaved column by column: column k collects
// a_i b_{k-i} and M_i q_{k-i} for all i, M_k is taken from the low limb of the
// column, and the column's carry moves to the next one.
//
// Value conventions (all functions state theirs):
//   normalised: every limb < 2^B;
//   lazy      : limbs < 2^(B+2), produced only as a multiplication operand;
//   semi-reduced values lie in [0, 2p); canonical values in [0, p).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "curves.h"

namespace eccmi {

template <class F>
struct Fp {
  uint32_t w[F::NL];
};

template <class F>
__device__ __forceinline__ Fp<F> fp_from(const Words<F::NL>& c) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = c.w[i];
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_zero() {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = 0;
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_one() {
  constexpr Words<F::NL> one = F::ONE;
  return fp_from<F>(one);
}

// ---- limb-level helpers --------------------------------------------------

// carry propagation of non-negative limbs (each < 2^31) to normalised limbs
template <class F>
__device__ __forceinline__ Fp<F> fp_normalize(const Fp<F>& a) {
  Fp<F> r;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < F::NL - 1; i++) {
    uint32_t t = a.w[i] + c;
    r.w[i] = t & F::MASK;
    c = t >> F::B;
  }
  r.w[F::NL - 1] = a.w[F::NL - 1] + c;
  return r;
}

// a - K if a >= K else a, for normalised a and a normalised constant K
template <class F>
__device__ __forceinline__ Fp<F> fp_cond_sub(const Fp<F>& a, const Words<F::NL>& K) {
  Fp<F> t;
  int32_t br = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    int32_t v = int32_t(a.w[i]) - int32_t(K.w[i]) + br;
    br = v >> F::B;  // 0 or -1
    t.w[i] = uint32_t(v) & F::MASK;
  }
  // the top limb keeps its full width (values are below 2^(B NL))
  bool keep = br < 0;
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = keep ? a.w[i] : t.w[i];
  return r;
}

// canonical form of a normalised semi-reduced value
template <class F>
__device__ __forceinline__ Fp<F> fp_canonical(const Fp<F>& a) {
  constexpr Words<F::NL> p = F::P;
  return fp_cond_sub<F>(a, p);
}

// ---- additive operations ---------------------------------------------------

// a + b as a lazy multiplication operand (limbs < 2^(B+1)), value a + b
template <class F>
__device__ __forceinline__ Fp<F> fp_add_lazy(const Fp<F>& a, const Fp<F>& b) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = a.w[i] + b.w[i];
  return r;
}

// a - b + 4p as a lazy multiplication operand: limbs < 2^(B+2), value in
// (2p, 6p) for normalised a, b below 2p.  For B = 29 the limbs are carried
// back to normalised form so that the product's columns stay within 64 bits.
template <class F>
__device__ __forceinline__ Fp<F> fp_sub_lazy(const Fp<F>& a, const Fp<F>& b) {
  constexpr Words<F::NL> kp = F::KP;
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = a.w[i] + kp.w[i] - b.w[i];
  if constexpr (F::B > 28) r = fp_normalize<F>(r);
  return r;
}

// (a + b) mod 2p: normalised, semi-reduced, for a, b semi-reduced
template <class F>
__device__ __forceinline__ Fp<F> fp_add(const Fp<F>& a, const Fp<F>& b) {
  constexpr Words<F::NL> p2 = F::P2;
  return fp_cond_sub<F>(fp_normalize<F>(fp_add_lazy<F>(a, b)), p2);
}

// (a - b) mod 2p: normalised, semi-reduced, for a, b semi-reduced
template <class F>
__device__ __forceinline__ Fp<F> fp_sub(const Fp<F>& a, const Fp<F>& b) {
  constexpr Words<F::NL> p2 = F::P2;
  // signed limb differences, carried with arithmetic shifts: value in (-2p, 2p)
  int32_t d[F::NL];
  int32_t c = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    int32_t v = int32_t(a.w[i]) - int32_t(b.w[i]) + c;
    if (i < F::NL - 1) {
      c = v >> F::B;
      v &= int32_t(F::MASK);
    }
    d[i] = v;
  }
  // negative iff the top limb is negative: then add 2p
  uint32_t mask = d[F::NL - 1] < 0 ? 0xffffffffu : 0u;
  Fp<F> r;
  uint32_t cc = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) {
    uint32_t t = uint32_t(d[i]) + (p2.w[i] & mask) + cc;
    if (i < F::NL - 1) {
      cc = t >> F::B;
      t &= F::MASK;
    }
    r.w[i] = t;
  }
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

// ---- comparisons (any semi-reduced operands) --------------------------------

template <class F>
__device__ __forceinline__ bool fp_is_zero(const Fp<F>& a) {
  Fp<F> c = fp_canonical<F>(a);
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) o |= c.w[i];
  return o == 0;
}

// equality of two canonical values (no reduction)
template <class F>
__device__ __forceinline__ bool fp_eq_canonical(const Fp<F>& a, const Fp<F>& b) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < F::NL; i++) o |= a.w[i] ^ b.w[i];
  return o == 0;
}

template <class F>
__device__ __forceinline__ bool fp_eq(const Fp<F>& a, const Fp<F>& b) {
  return fp_eq_canonical<F>(fp_canonical<F>(a), fp_canonical<F>(b));
}

// ---- Montgomery reduction for a sparse prime (Section 4.2) ------------------
//
// When p = -1 mod 2^B, q_inv = 1 and the multiple m_k of p that clears column
// k is the column's own low B bits.  Adding m_k p then takes one term per
// nonzero balanced digit of p instead of NL products, and the lowest digit
// (-1) cancels exactly the bits that the shift drops, so it costs nothing.
// For secp256r1, p = 2^256 - 2^224 + 2^192 + 2^96 - 1 has the radix-2^28
// digits -1, 2^12 (limb 3), 2^24 (limb 6), -1 (limb 8) and 16 (limb 9): four
// multiply-adds per column in place of ten and the q_inv product.  A column
// may go negative on the way, so the carry shifts arithmetically; every m_k,
// and so the result, equals that of the generic reduction bit for bit.

// the nonzero digits of p above the lowest one, in scalar registers
template <class F>
__device__ __forceinline__ void sparse_digits(int32_t (&dq)[F::NL]) {
  constexpr Digits<F::NL> sd = F::SD;
#pragma unroll
  for (int j = 0; j < F::NL; j++) {
    dq[j] = sd.d[j];
    if (j > 0 && sd.d[j] != 0) asm("" : "+s"(dq[j]));
  }
}

// acc += sum over i in [lo, hi) of m_i d_(k - i), skipping zero digits
template <class F>
__device__ __forceinline__ void sparse_terms(uint64_t& acc, const uint32_t (&m)[F::NL], const int32_t (&dq)[F::NL],
                                             int k, int lo, int hi) {
  constexpr Digits<F::NL> sd = F::SD;
#pragma unroll
  for (int i = lo; i < hi; i++) {
    const int32_t d = sd.d[k - i];
    if (d > 0) acc += uint64_t(m[i]) * uint32_t(dq[k - i]);
    if (d < 0) acc += uint64_t(int64_t(int32_t(m[i])) * int64_t(dq[k - i]));
  }
}

template <class F>
__device__ __forceinline__ Fp<F> fp_mul_sparse(const Fp<F>& a, const Fp<F>& b) {
  constexpr int NL = F::NL;
  constexpr int B = F::B;
  int32_t dq[NL];
  sparse_digits<F>(dq);
  uint32_t m[NL];
  Fp<F> r;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NL; k++) {
#pragma unroll
    for (int i = 0; i <= k; i++) acc += uint64_t(a.w[i]) * b.w[k - i];
    sparse_terms<F>(acc, m, dq, k, 0, k);
    m[k] = uint32_t(acc) & F::MASK;
    acc = uint64_t(int64_t(acc) >> B);
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; k++) {
#pragma unroll
    for (int i = k - NL + 1; i < NL; i++) acc += uint64_t(a.w[i]) * b.w[k - i];
    sparse_terms<F>(acc, m, dq, k, k - NL + 1, NL);
    r.w[k - NL] = uint32_t(acc) & F::MASK;
    acc = uint64_t(int64_t(acc) >> B);
  }
  r.w[NL - 1] = uint32_t(acc);
  return r;
}

template <class F>
__device__ __forceinline__ Fp<F> fp_sqr_sparse(const Fp<F>& a) {
  constexpr int NL = F::NL;
  constexpr int B = F::B;
  int32_t dq[NL];
  sparse_digits<F>(dq);
  uint32_t a2[NL];
#pragma unroll
  for (int j = 0; j < NL; j++) a2[j] = a.w[j] << 1;
  uint32_t m[NL];
  Fp<F> r;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NL; k++) {
#pragma unroll
    for (int i = 0; 2 * i < k; i++) acc += uint64_t(a.w[i]) * a2[k - i];
    if ((k & 1) == 0) acc += uint64_t(a.w[k / 2]) * a.w[k / 2];
    sparse_terms<F>(acc, m, dq, k, 0, k);
    m[k] = uint32_t(acc) & F::MASK;
    acc = uint64_t(int64_t(acc) >> B);
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; k++) {
#pragma unroll
    for (int i = k - NL + 1; 2 * i < k; i++) acc += uint64_t(a.w[i]) * a2[k - i];
    if ((k & 1) == 0) acc += uint64_t(a.w[k / 2]) * a.w[k / 2];
    sparse_terms<F>(acc, m, dq, k, k - NL + 1, NL);
    r.w[k - NL] = uint32_t(acc) & F::MASK;
    acc = uint64_t(int64_t(acc) >> B);
  }
  r.w[NL - 1] = uint32_t(acc);
  return r;
}

// ---- Montgomery multiplication ---------------------------------------------

// a b R^-1 mod p: normalised, semi-reduced.  Requires one operand normalised,
// the other normalised or lazy, and a b < R p (true for one operand < 2p and
// the other < 6p).
template <class F>
__device__ __forceinline__ Fp<F> fp_mul(const Fp<F>& a, const Fp<F>& b) {
  if constexpr (F::SPARSE) return fp_mul_sparse<F>(a, b);
  constexpr int NL = F::NL;
  constexpr int B = F::B;
  constexpr Words<NL> qc = F::P;
  // modulus limbs and q_inv in scalar registers; the empty asm keeps the
  // compiler from rebuilding the constants at every use
  uint32_t q[NL];
#pragma unroll
  for (int j = 0; j < NL; j++) {
    q[j] = qc.w[j];
    asm("" : "+s"(q[j]));
  }
  uint32_t qinv = F::QINV;
  asm("" : "+s"(qinv));
  uint32_t m[NL];
  Fp<F> r;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NL; k++) {
#pragma unroll
    for (int i = 0; i <= k; i++) acc += uint64_t(a.w[i]) * b.w[k - i];
#pragma unroll
    for (int i = 0; i < k; i++) acc += uint64_t(m[i]) * q[k - i];
    m[k] = (uint32_t(acc) * qinv) & F::MASK;
    acc += uint64_t(m[k]) * q[0];  // clears the low B bits
    acc >>= B;
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; k++) {
#pragma unroll
    for (int i = k - NL + 1; i < NL; i++) acc += uint64_t(a.w[i]) * b.w[k - i];
#pragma unroll
    for (int i = k - NL + 1; i < NL; i++) acc += uint64_t(m[i]) * q[k - i];
    r.w[k - NL] = uint32_t(acc) & F::MASK;
    acc >>= B;
  }
  r.w[NL - 1] = uint32_t(acc);
  return r;
}

// a^2 R^-1 mod p: normalised, semi-reduced, for a normalised a < 2p.  The
// integer product takes each cross term a_i a_j (i < j) once, against the
// doubled limb 2 a_j, plus the squares a_i^2: NL (NL + 1) / 2 limb products
// instead of NL^2; the reduction is that of fp_mul.
template <class F>
__device__ __forceinline__ Fp<F> fp_sqr(const Fp<F>& a) {
  if constexpr (F::SPARSE) return fp_sqr_sparse<F>(a);
  constexpr int NL = F::NL;
  constexpr int B = F::B;
  constexpr Words<NL> qc = F::P;
  uint32_t q[NL];
#pragma unroll
  for (int j = 0; j < NL; j++) {
    q[j] = qc.w[j];
    asm("" : "+s"(q[j]));
  }
  uint32_t qinv = F::QINV;
  asm("" : "+s"(qinv));
  uint32_t a2[NL];
#pragma unroll
  for (int j = 0; j < NL; j++) a2[j] = a.w[j] << 1;
  uint32_t m[NL];
  Fp<F> r;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NL; k++) {
#pragma unroll
    for (int i = 0; 2 * i < k; i++) acc += uint64_t(a.w[i]) * a2[k - i];
    if ((k & 1) == 0) acc += uint64_t(a.w[k / 2]) * a.w[k / 2];
#pragma unroll
    for (int i = 0; i < k; i++) acc += uint64_t(m[i]) * q[k - i];
    m[k] = (uint32_t(acc) * qinv) & F::MASK;
    acc += uint64_t(m[k]) * q[0];  // clears the low B bits
    acc >>= B;
  }
#pragma unroll
  for (int k = NL; k < 2 * NL - 1; k++) {
#pragma unroll
    for (int i = k - NL + 1; 2 * i < k; i++) acc += uint64_t(a.w[i]) * a2[k - i];
    if ((k & 1) == 0) acc += uint64_t(a.w[k / 2]) * a.w[k / 2];
#pragma unroll
    for (int i = k - NL + 1; i < NL; i++) acc += uint64_t(m[i]) * q[k - i];
    r.w[k - NL] = uint32_t(acc) & F::MASK;
    acc >>= B;
  }
  r.w[NL - 1] = uint32_t(acc);
  return r;
}

// ---- conversions between the I/O words and the working form -----------------

// canonical N32-word integer -> B-bit limbs (no Montgomery factor)
template <class F>
__device__ __forceinline__ Fp<F> fp_from_words(const uint32_t (&x)[F::N32]) {
  Fp<F> r;
#pragma unroll
  for (int k = 0; k < F::NL; k++) {
    constexpr int B = F::B;
    const int bit = B * k;
    const int w = bit >> 5, s = bit & 31;
    uint32_t lo = w < F::N32 ? x[w] : 0u;
    uint32_t hi = (w + 1) < F::N32 ? x[w + 1] : 0u;
    uint32_t v = s ? ((lo >> s) | (hi << (32 - s))) : lo;
    r.w[k] = v & F::MASK;
  }
  return r;
}

// normalised limbs of a value < 2^(32 N32) -> N32 words
template <class F>
__device__ __forceinline__ void fp_to_words(const Fp<F>& a, uint32_t (&x)[F::N32]) {
#pragma unroll
  for (int w = 0; w < F::N32; w++) {
    constexpr int B = F::B;
    const int bit = 32 * w;
    const int k = bit / B, s = bit % B;
    uint32_t v = a.w[k] >> s;
    if (k + 1 < F::NL) v |= a.w[k + 1] << (B - s);
    if (k + 2 < F::NL && 2 * B - s < 32) v |= a.w[k + 2] << (2 * B - s);
    x[w] = v;
  }
}

// canonical words -> Montgomery working form (x R mod p, semi-reduced)
template <class F>
__device__ __forceinline__ Fp<F> fp_to_mont(const Fp<F>& a) {
  constexpr Words<F::NL> r2 = F::R2;
  return fp_mul<F>(a, fp_from<F>(r2));
}

// Montgomery working form -> canonical plain value
template <class F>
__device__ __forceinline__ Fp<F> fp_from_mont(const Fp<F>& a) {
  Fp<F> one = fp_zero<F>();
  one.w[0] = 1;
  return fp_canonical<F>(fp_mul<F>(a, one));
}

// x < p for canonical-range checks of I/O words
template <class F>
__device__ __forceinline__ bool words_lt_p(const uint32_t (&x)[F::N32]) {
  constexpr Words<F::N32> p = F::P32;
  bool lt = false, decided = false;
#pragma unroll
  for (int i = F::N32 - 1; i >= 0; i--) {
    if (!decided && x[i] != p.w[i]) {
      lt = x[i] < p.w[i];
      decided = true;
    }
  }
  return lt;
}

// ---- loads and stores --------------------------------------------------------
// A stored coordinate occupies CW words (NL limbs then padding), a multiple of
// four so that it moves as 16-byte vectors.

template <class F>
__device__ __forceinline__ Fp<F> fp_load(const uint32_t* __restrict__ p) {
  Fp<F> r;
  const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int i = 0; i < F::CW / 4; i++) {
    uint4 t = v[i];
    if (4 * i < F::NL) r.w[4 * i] = t.x;
    if (4 * i + 1 < F::NL) r.w[4 * i + 1] = t.y;
    if (4 * i + 2 < F::NL) r.w[4 * i + 2] = t.z;
    if (4 * i + 3 < F::NL) r.w[4 * i + 3] = t.w;
  }
  return r;
}

template <class F>
__device__ __forceinline__ void fp_store(uint32_t* __restrict__ p, const Fp<F>& a) {
  uint4* v = reinterpret_cast<uint4*>(p);
#pragma unroll
  for (int i = 0; i < F::CW / 4; i++) {
    uint32_t e[4];
#pragma unroll
    for (int j = 0; j < 4; j++) e[j] = (4 * i + j < F::NL) ? a.w[4 * i + j] : 0u;
    v[i] = make_uint4(e[0], e[1], e[2], e[3]);
  }
}

// structure-of-arrays access: limb i of element e lives at p[i * stride + e]
template <class F>
__device__ __forceinline__ Fp<F> fp_load_soa(const uint32_t* __restrict__ p, size_t stride) {
  Fp<F> r;
#pragma unroll
  for (int i = 0; i < F::NL; i++) r.w[i] = p[i * stride];
  return r;
}

template <class F>
__device__ __forceinline__ void fp_store_soa(uint32_t* __restrict__ p, size_t stride, const Fp<F>& a) {
#pragma unroll
  for (int i = 0; i < F::NL; i++) p[i * stride] = a.w[i];
}

// I/O words of one coordinate (N32 words, u64 limbs in memory)
template <class F>
__device__ __forceinline__ void words_load(const uint32_t* __restrict__ p, uint32_t (&x)[F::N32]) {
  const uint4* v = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int i = 0; i < F::N32 / 4; i++) {
    uint4 t = v[i];
    x[4 * i] = t.x;
    x[4 * i + 1] = t.y;
    x[4 * i + 2] = t.z;
    x[4 * i + 3] = t.w;
  }
}

template <class F>
__device__ __forceinline__ void words_store(uint32_t* __restrict__ p, const uint32_t (&x)[F::N32]) {
  uint4* v = reinterpret_cast<uint4*>(p);
#pragma unroll
  for (int i = 0; i < F::N32 / 4; i++) v[i] = make_uint4(x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]);
}

}  // namespace eccmi
