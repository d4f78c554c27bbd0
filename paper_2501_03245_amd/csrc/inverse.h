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
// ---- the GCD of one wave-uniform operand, spread over the wave ---------------
// The 30-divstep batches need only the low 32 bits of f and g and branch on
// every step: they run on the scalar unit.  Each batch's matrix is then
// applied to the long f, g, d, e with one 30-bit limb per lane (lane k holds
// limb k): every lane forms its 64-bit combination at once, and the carries
// move up one lane per pass until none is left, instead of a serial carry
// chain through all limbs.  The exact division by 2^30 is a shift down by one
// lane.

// value of lane k - 1 in lane k (lane 0 of each row of 16 gets 0)
__device__ __forceinline__ int64_t lanes_up1(int64_t v) {
  const int32_t lo = __builtin_amdgcn_update_dpp(0, int32_t(uint64_t(v)), 0x111, 0xf, 0xf, true);
  const int32_t hi = __builtin_amdgcn_update_dpp(0, int32_t(uint64_t(v) >> 32), 0x111, 0xf, 0xf, true);
  return int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
}

// value of lane k + 1 in lane k (lane 15 of each row gets 0)
__device__ __forceinline__ int32_t lanes_down1(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x101, 0xf, 0xf, true);
}

// two carry passes over four lane-distributed values at once (lane k:
// coefficient of 2^(30 k); lanes 0 .. L - 2 keep 30 bits, lane L - 1 the
// rest).  From |v| < 2^62 this leaves lanes 0 .. L - 2 in [-8, 2^30 + 8):
// not normalised, but small enough for the next matrix products, and every
// lane but the top one a multiple of 2^30 in value, so that the low words
// and the division by 2^30 stay exact
template <int L>
__device__ __forceinline__ void lanes_carry2x4(int64_t (&v)[4], int lane) {
  const bool low = lane < L - 1;
#pragma unroll
  for (int pass = 0; pass < 2; pass++) {
    int64_t c[4];
#pragma unroll
    for (int t = 0; t < 4; t++) c[t] = low ? (v[t] >> 30) : 0;
#pragma unroll
    for (int t = 0; t < 4; t++) v[t] = (low ? (v[t] & int64_t(M30)) : v[t]) + lanes_up1(c[t]);
  }
}

template <class F>
__device__ __forceinline__ void inverse_wave(const uint32_t* x, uint32_t* out) {
  using I = Inv30<F>;
  constexpr int L = I::L;
  static_assert(L + 1 <= 16, "limbs (and the carry-out lane) must fit one DPP row");
  constexpr Words<L> p = I::P;
  constexpr uint32_t pinv = I::PINV;
  const int lane = threadIdx.x & 63;
  int32_t pk = 0, gk = 0;
#pragma unroll
  for (int k = 0; k < L; k++) {
    int bit = 30 * k, wi = bit >> 5, s = bit & 31;
    uint64_t v = wi < F::N32 ? x[wi] : 0u;
    if (wi + 1 < F::N32) v |= uint64_t(x[wi + 1]) << 32;
    if (lane == k) {
      pk = int32_t(p.w[k]);
      gk = int32_t((v >> s) & uint64_t(M30));
    }
  }
  int32_t fk = pk, dk = 0, ek = lane == 0 ? 1 : 0;
  int32_t delta = 1;
  for (int batch = 0; batch < 200; batch++) {
    // g = 0 ends the loop (its limbs are only partly carried, so zero limbs
    // may come a batch late; batches with g = 0 change nothing)
    if (__builtin_amdgcn_ballot_w64(gk != 0) == 0) break;
    // low 32 bits of f and g (a sum: lanes 0 and 1 are not normalised)
    uint32_t fl = uint32_t(__builtin_amdgcn_readlane(fk, 0)) + (uint32_t(__builtin_amdgcn_readlane(fk, 1)) << 30);
    uint32_t gl = uint32_t(__builtin_amdgcn_readlane(gk, 0)) + (uint32_t(__builtin_amdgcn_readlane(gk, 1)) << 30);
    int32_t u = 1, v = 0, q = 0, r = 1;  // 2^j (f_j, g_j) = (u f + v g, q f + r g)
    // 30 divsteps in variable time: a run of halvings of an even g at once
    // (trailing zeros, capped at the steps left), a swap when g is odd and
    // delta > 0, then up to min(1 - delta, steps left, 6) additions of f
    // merged into one: g += w f with w = -g / f mod 2^bits, where
    // 1 / f = f (2 - f^2) mod 64 for odd f
    int32_t left = 30;
    for (int guard = 0; guard < 64; guard++) {
      const int32_t z = __builtin_ctz(gl | (1u << left));
      gl >>= z;
      u = int32_t(uint32_t(u) << z);
      v = int32_t(uint32_t(v) << z);
      delta += z;
      left -= z;
      if (left == 0) break;
      if (delta > 0) {
        delta = -delta;
        const uint32_t tf = fl;
        fl = gl;
        gl = 0u - tf;
        const int32_t tu = u, tv = v;
        u = q;
        v = r;
        q = -tu;
        r = -tv;
      }
      int32_t bits = 1 - delta;
      if (bits > left) bits = left;
      if (bits > 6) bits = 6;
      const uint32_t w = (gl * fl * (fl * fl - 2u)) & ((1u << bits) - 1u);
      gl += fl * w;
      q += int32_t(uint32_t(u) * w);
      r += int32_t(uint32_t(v) * w);
    }
    // (f, g) <- M (f, g) / 2^30, exact
    int64_t cf = int64_t(u) * fk + int64_t(v) * gk;
    int64_t cg = int64_t(q) * fk + int64_t(r) * gk;
    // (d, e) <- (M (d, e) + (md, me) p) / 2^30, the multiples of p chosen
    // from the low limb (lane 0) so that the division is exact
    int64_t cd = int64_t(u) * dk + int64_t(v) * ek;
    int64_t ce = int64_t(q) * dk + int64_t(r) * ek;
    const uint32_t lo_d = uint32_t(__builtin_amdgcn_readlane(int32_t(uint64_t(cd)), 0));
    const uint32_t lo_e = uint32_t(__builtin_amdgcn_readlane(int32_t(uint64_t(ce)), 0));
    int32_t md = int32_t((0u - lo_d * pinv) & uint32_t(M30));
    int32_t me = int32_t((0u - lo_e * pinv) & uint32_t(M30));
    if (md > (1 << 29)) md -= (1 << 30);
    if (me > (1 << 29)) me -= (1 << 30);
    cd += int64_t(md) * pk;
    ce += int64_t(me) * pk;
    // carried over L + 1 lanes (lane L takes the signed carry-out), then
    // shifted down one lane: lanes 0 .. L - 1 hold the quotient's limbs
    int64_t c4[4] = {cf, cg, cd, ce};
    lanes_carry2x4<L + 1>(c4, lane);
    fk = lanes_down1(int32_t(c4[0]));
    gk = lanes_down1(int32_t(c4[1]));
    dk = lanes_down1(int32_t(c4[2]));
    ek = lanes_down1(int32_t(c4[3]));
  }
  // f = +-1: x^-1 = sign(f) d mod p, finished on the scalar unit
  int32_t f[L], d[L];
#pragma unroll
  for (int k = 0; k < L; k++) {
    f[k] = __builtin_amdgcn_readlane(fk, k);
    d[k] = __builtin_amdgcn_readlane(dk, k);
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
__device__ __noinline__ Fp<F> fp_inv_uniform(Fp<F> xr) {  // by value: the argument travels in registers
  constexpr int N = F::N32;
  uint32_t w[N], iw[N];
  fp_to_words<F>(fp_canonical<F>(xr), w);
#pragma unroll
  for (int i = 0; i < N; i++) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  inverse_wave<F>(w, iw);
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
