// Single-lane field inversion for the "apply" step of the batch inversion
// (Section 3.2).  Section 2.2 names two families: Fermat's x^(q-2) (hundreds
// of multiplications) and the extended-Euclid/binary-GCD family (cheaper but
// branchy, hence avoided there for data-parallel lanes).  Here one lane
// inverts the product of a whole workgroup, so data-dependent control flow is
// harmless and a GCD method is used: the divstep iteration of Bernstein and
// Yang ("Fast constant-time gcd computation and modular inversion", 2019), in
// batches of 30 divsteps whose decisions depend only on the low bits of f and
// g; each batch yields a 2x2 matrix that is then applied to the full values.
//
//   divstep(delta, f, g) = (1 - delta, g, (g - f)/2)        if delta > 0, g odd
//                          (1 + delta, f, (g + (g mod 2) f)/2) otherwise
// Starting from (1, p, x) the iteration reaches g = 0 with f = +-1; tracking
// d, e with f = d x and g = e x (mod p) gives x^-1 = +-d.
//
// Big values use 30-bit limbs in signed 32-bit registers (lower limbs in
// [0, 2^30), the top limb signed), so every limb product fits one
// v_mad_i64_i32.
#pragma once
#include "field.h"

namespace eccmi {

template <class F>
struct Inv30 {
  static constexpr int L = (32 * F::N32 + 2 + 29) / 30;  // limbs for +-2^(32 N32 + 1)
  static constexpr Words<L> P = to_limbs<L, 30, F::N32>(F::P32);
  // p^-1 mod 2^30 (p odd)
  static constexpr uint32_t PINV = (0u - neg_inv_bits(F::P32.w[0], 30)) & ((1u << 30) - 1u);
};

constexpr int32_t M30 = (1 << 30) - 1;

// (a, b) <- ((u a + v b) / 2^30, (q a + r b) / 2^30), exact divisions
template <int L>
__host__ __device__ __forceinline__ void lin30_exact(int32_t* a, int32_t* b, int32_t u, int32_t v, int32_t q, int32_t r) {
  int64_t ca = int64_t(u) * a[0] + int64_t(v) * b[0];
  int64_t cb = int64_t(q) * a[0] + int64_t(r) * b[0];
  ca >>= 30;
  cb >>= 30;
#pragma unroll
  for (int i = 1; i < L; i++) {
    ca += int64_t(u) * a[i] + int64_t(v) * b[i];
    cb += int64_t(q) * a[i] + int64_t(r) * b[i];
    a[i - 1] = int32_t(ca & M30);
    b[i - 1] = int32_t(cb & M30);
    ca >>= 30;
    cb >>= 30;
  }
  a[L - 1] = int32_t(ca);
  b[L - 1] = int32_t(cb);
}

// (d, e) <- ((u d + v e) / 2^30, (q d + r e) / 2^30) mod p: a multiple of p
// chosen from the low limb makes each combination divisible by 2^30
template <class F>
__host__ __device__ __forceinline__ void lin30_mod(int32_t* d, int32_t* e, int32_t u, int32_t v, int32_t q, int32_t r) {
  using I = Inv30<F>;
  constexpr int L = I::L;
  constexpr Words<L> p = I::P;
  constexpr uint32_t pinv = I::PINV;
  int64_t cd = int64_t(u) * d[0] + int64_t(v) * e[0];
  int64_t ce = int64_t(q) * d[0] + int64_t(r) * e[0];
  // md = -cd / p mod 2^30, taken in (-2^29, 2^29] to keep |d| growing slowly
  int32_t md = int32_t((uint32_t(0) - uint32_t(cd) * pinv) & uint32_t(M30));
  int32_t me = int32_t((uint32_t(0) - uint32_t(ce) * pinv) & uint32_t(M30));
  if (md > (1 << 29)) md -= (1 << 30);
  if (me > (1 << 29)) me -= (1 << 30);
  cd += int64_t(md) * int32_t(p.w[0]);
  ce += int64_t(me) * int32_t(p.w[0]);
  cd >>= 30;
  ce >>= 30;
#pragma unroll
  for (int i = 1; i < L; i++) {
    cd += int64_t(u) * d[i] + int64_t(v) * e[i] + int64_t(md) * int32_t(p.w[i]);
    ce += int64_t(q) * d[i] + int64_t(r) * e[i] + int64_t(me) * int32_t(p.w[i]);
    d[i - 1] = int32_t(cd & M30);
    e[i - 1] = int32_t(ce & M30);
    cd >>= 30;
    ce >>= 30;
  }
  d[L - 1] = int32_t(cd);
  e[L - 1] = int32_t(ce);
}

template <int L>
__host__ __device__ __forceinline__ bool s30_is_zero(const int32_t* a) {
  int32_t o = 0;
#pragma unroll
  for (int i = 0; i < L; i++) o |= a[i];
  return o == 0;
}

// carry the lower limbs into [0, 2^30); the sign then sits in the top limb
template <int L>
__host__ __device__ __forceinline__ void s30_carry(int32_t* a) {
#pragma unroll
  for (int i = 0; i < L - 1; i++) {
    int32_t c = a[i] >> 30;
    a[i] &= M30;
    a[i + 1] += c;
  }
}

template <class F>
__host__ __device__ __forceinline__ void s30_add_p(int32_t* a, int sign) {
  using I = Inv30<F>;
  constexpr Words<I::L> p = I::P;
#pragma unroll
  for (int i = 0; i < I::L; i++) a[i] += sign * int32_t(p.w[i]);
  s30_carry<I::L>(a);
}

// a >= p for a non-negative carried value
template <class F>
__host__ __device__ __forceinline__ bool s30_ge_p(const int32_t* a) {
  using I = Inv30<F>;
  constexpr Words<I::L> p = I::P;
  bool ge = true, decided = false;
#pragma unroll
  for (int i = I::L - 1; i >= 0; i--) {
    if (!decided && a[i] != int32_t(p.w[i])) {
      ge = a[i] > int32_t(p.w[i]);
      decided = true;
    }
  }
  return ge;
}

// x^-1 mod p for a canonical 0 < x < p given as N32 words (0 for x = 0).
// Runs in the calling lane; the batch loop ends when g reaches 0, with a cap
// far above the known divstep bounds so that any input terminates.
template <class F>
__host__ __device__ __forceinline__ void inverse_words_inline(const uint32_t* x, uint32_t* out) {
  using I = Inv30<F>;
  constexpr int L = I::L;
  constexpr Words<L> p = I::P;
  int32_t f[L], g[L], d[L], e[L];
#pragma unroll
  for (int k = 0; k < L; k++) {
    int bit = 30 * k, wi = bit >> 5, s = bit & 31;
    uint64_t v = wi < F::N32 ? x[wi] : 0u;
    if (wi + 1 < F::N32) v |= uint64_t(x[wi + 1]) << 32;
    g[k] = int32_t((v >> s) & uint64_t(M30));
    f[k] = int32_t(p.w[k]);
    d[k] = 0;
    e[k] = 0;
  }
  e[0] = 1;
  int32_t delta = 1;
  for (int batch = 0; batch < 200 && !s30_is_zero<L>(g); batch++) {
    // 30 divsteps on the low 32 bits of f and g (exact for the parities used)
    uint32_t fl = uint32_t(f[0]) | (uint32_t(f[1]) << 30);
    uint32_t gl = uint32_t(g[0]) | (uint32_t(g[1]) << 30);
    int32_t u = 1, v = 0, q = 0, r = 1;  // 2^j (f_j, g_j) = (u f + v g, q f + r g)
    // branch-free divstep: when g is odd and delta > 0, first swap
    // (delta, f, g, u, v, q, r) -> (-delta, g, -f, q, r, -u, -v); then
    // delta += 1, g += f (g odd), g /= 2, with (q, r) += (u, v) (g odd) and
    // (u, v) doubled, which keeps 2^j (f, g) = (u f0 + v g0, q f0 + r g0)
#pragma unroll
    for (int j = 0; j < 30; j++) {
      const uint32_t odd = 0u - (gl & 1u);
      const uint32_t swp = odd & uint32_t(int32_t(-delta) >> 31);  // g odd and delta > 0
      const uint32_t nf = (gl & swp) | (fl & ~swp);
      const uint32_t ng = ((0u - fl) & swp) | (gl & ~swp);
      const int32_t nu = int32_t((uint32_t(q) & swp) | (uint32_t(u) & ~swp));
      const int32_t nv = int32_t((uint32_t(r) & swp) | (uint32_t(v) & ~swp));
      const int32_t nq = int32_t((uint32_t(-u) & swp) | (uint32_t(q) & ~swp));
      const int32_t nr = int32_t((uint32_t(-v) & swp) | (uint32_t(r) & ~swp));
      delta = int32_t((uint32_t(-delta) & swp) | (uint32_t(delta) & ~swp)) + 1;
      fl = nf;
      gl = (ng + (nf & odd)) >> 1;
      q = nq + int32_t(uint32_t(nu) & odd);
      r = nr + int32_t(uint32_t(nv) & odd);
      u = nu * 2;
      v = nv * 2;
    }
    lin30_exact<L>(f, g, u, v, q, r);
    lin30_mod<F>(d, e, u, v, q, r);
  }
  // f = +-1: x^-1 = sign(f) d mod p
  s30_carry<L>(f);
  s30_carry<L>(d);
  if (f[L - 1] < 0) {
    for (int i = 0; i < L; i++) d[i] = -d[i];
    s30_carry<L>(d);
  }
  for (int it = 0; it < 64 && d[L - 1] < 0; it++) s30_add_p<F>(d, 1);
  for (int it = 0; it < 64 && s30_ge_p<F>(d); it++) s30_add_p<F>(d, -1);
#pragma unroll
  for (int wi = 0; wi < F::N32; wi++) {
    int bit = 32 * wi, k = bit / 30, s = bit % 30;
    uint64_t v = uint32_t(d[k]) >> s;
    if (k + 1 < L) v |= uint64_t(uint32_t(d[k + 1])) << (30 - s);
    if (k + 2 < L) v |= uint64_t(uint32_t(d[k + 2])) << (60 - s);
    out[wi] = uint32_t(v);
  }
}

// The same as a separate function of the calling lane (per-lane inversions).
// V only makes distinct copies of the function, so that each copy is compiled
// under the register budget of the kernels that call it.
template <class F, int V = 0>
__host__ __device__ __noinline__ void inverse_words(const uint32_t* x, uint32_t* out) {
  inverse_words_inline<F>(x, out);
}

// Inverse of a Montgomery-form element x R (x != 0), returned as x^-1 R:
// the GCD gives (x R)^-1 = x^-1 R^-1, and one Montgomery product with R^3
// restores the factor: x^-1 R^-1 R^3 R^-1 = x^-1 R.  Every lane returns the
// inverse of lane 0's argument.
// The GCD of a wave-uniform operand split between the two units of a CU:
// the 30-divstep batches, which need only the low 32 bits of f and g and
// branch on every step, run on the scalar unit; the application of each
// batch's matrix to the long f, g, d, e (64-bit multiply-adds) runs on the
// vector unit, whose multiply-add is several times faster.  The long values
// start from an opaque per-lane zero so that they are kept in vector
// registers; every lane holds the same values.
template <class F>
__device__ __forceinline__ void inverse_words_split(const uint32_t* x, uint32_t* out) {
  using I = Inv30<F>;
  constexpr int L = I::L;
  constexpr Words<L> p = I::P;
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  int32_t f[L], g[L], d[L], e[L];
#pragma unroll
  for (int k = 0; k < L; k++) {
    int bit = 30 * k, wi = bit >> 5, s = bit & 31;
    uint64_t v = wi < F::N32 ? x[wi] : 0u;
    if (wi + 1 < F::N32) v |= uint64_t(x[wi + 1]) << 32;
    g[k] = int32_t(uint32_t((v >> s) & uint64_t(M30)) + z);
    f[k] = int32_t(p.w[k] + z);
    d[k] = int32_t(z);
    e[k] = int32_t(z);
  }
  e[0] = 1;
  int32_t delta = 1;
  for (int batch = 0; batch < 200; batch++) {
    uint32_t gor = 0;
#pragma unroll
    for (int k = 0; k < L; k++) gor |= uint32_t(g[k]);
    if (__builtin_amdgcn_readfirstlane(gor) == 0) break;
    uint32_t fl = __builtin_amdgcn_readfirstlane(uint32_t(f[0]) | (uint32_t(f[1]) << 30));
    uint32_t gl = __builtin_amdgcn_readfirstlane(uint32_t(g[0]) | (uint32_t(g[1]) << 30));
    int32_t u = 1, v = 0, q = 0, r = 1;
#pragma unroll
    for (int j = 0; j < 30; j++) {
      const uint32_t odd = 0u - (gl & 1u);
      const uint32_t swp = odd & uint32_t(int32_t(-delta) >> 31);
      const uint32_t nf = (gl & swp) | (fl & ~swp);
      const uint32_t ng = ((0u - fl) & swp) | (gl & ~swp);
      const int32_t nu = int32_t((uint32_t(q) & swp) | (uint32_t(u) & ~swp));
      const int32_t nv = int32_t((uint32_t(r) & swp) | (uint32_t(v) & ~swp));
      const int32_t nq = int32_t((uint32_t(-u) & swp) | (uint32_t(q) & ~swp));
      const int32_t nr = int32_t((uint32_t(-v) & swp) | (uint32_t(r) & ~swp));
      delta = int32_t((uint32_t(-delta) & swp) | (uint32_t(delta) & ~swp)) + 1;
      fl = nf;
      gl = (ng + (nf & odd)) >> 1;
      q = nq + int32_t(uint32_t(nu) & odd);
      r = nr + int32_t(uint32_t(nv) & odd);
      u = nu * 2;
      v = nv * 2;
    }
    lin30_exact<L>(f, g, u, v, q, r);
    lin30_mod<F>(d, e, u, v, q, r);
  }
  s30_carry<L>(f);
  s30_carry<L>(d);
  if (f[L - 1] < 0) {
    for (int i = 0; i < L; i++) d[i] = -d[i];
    s30_carry<L>(d);
  }
  for (int it = 0; it < 64 && d[L - 1] < 0; it++) s30_add_p<F>(d, 1);
  for (int it = 0; it < 64 && s30_ge_p<F>(d); it++) s30_add_p<F>(d, -1);
#pragma unroll
  for (int wi = 0; wi < F::N32; wi++) {
    int bit = 32 * wi, k = bit / 30, s = bit % 30;
    uint64_t v = uint32_t(d[k]) >> s;
    if (k + 1 < L) v |= uint64_t(uint32_t(d[k + 1])) << (30 - s);
    if (k + 2 < L) v |= uint64_t(uint32_t(d[k + 2])) << (60 - s);
    out[wi] = uint32_t(v);
  }
}

template <class F, int V = 0>
__device__ __noinline__ Fp<F> fp_inv_uniform(const Fp<F>& xr) {
  constexpr int N = F::N32;
  uint32_t w[N], iw[N];
  fp_to_words<F>(fp_canonical<F>(xr), w);
#pragma unroll
  for (int i = 0; i < N; i++) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  inverse_words_split<F>(w, iw);
#pragma unroll
  for (int i = 0; i < N; i++) iw[i] = __builtin_amdgcn_readfirstlane(iw[i]);
  constexpr Words<F::NL> r3 = F::R3;
  // the final product on the vector unit as well
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  Fp<F> a = fp_from_words<F>(iw);
#pragma unroll
  for (int i = 0; i < F::NL; i++) a.w[i] += z;
  return fp_mul<F>(a, fp_from<F>(r3));
}

}  // namespace eccmi
