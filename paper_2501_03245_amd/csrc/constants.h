// Compile-time derivation of the Montgomery constants of each prime field.
//
// Only the primes, curve coefficients and generators are written down (as the
// published hexadecimal strings); everything else (R mod p, R^2, R^3, the
// per-word Montgomery factor q_inv = -p^-1 mod 2^32 of Algorithm 2) is
// computed here by constexpr arithmetic on 32-bit words.
#pragma once
#include <cstdint>

namespace eccmi {

template <int N>
struct Words {
  uint32_t w[N];
};

template <int N>
constexpr Words<N> hex_words(const char* s) {
  Words<N> r{};
  int len = 0;
  while (s[len]) len++;
  for (int i = 0; i < len; i++) {
    char ch = s[len - 1 - i];
    uint32_t v = (ch >= '0' && ch <= '9') ? uint32_t(ch - '0')
                 : (ch >= 'a' && ch <= 'f') ? uint32_t(ch - 'a' + 10)
                                            : uint32_t(ch - 'A' + 10);
    r.w[i / 8] |= v << (4 * (i % 8));
  }
  return r;
}

template <int N>
constexpr bool words_ge(const Words<N>& a, const Words<N>& b) {
  for (int i = N - 1; i >= 0; i--) {
    if (a.w[i] != b.w[i]) return a.w[i] > b.w[i];
  }
  return true;
}

template <int N>
constexpr Words<N> words_sub(const Words<N>& a, const Words<N>& b) {
  Words<N> r{};
  uint64_t br = 0;
  for (int i = 0; i < N; i++) {
    uint64_t d = uint64_t(a.w[i]) - b.w[i] - br;
    r.w[i] = uint32_t(d);
    br = (d >> 63) & 1;
  }
  return r;
}

// (2 x) mod p for x < p
template <int N>
constexpr Words<N> dbl_mod(const Words<N>& x, const Words<N>& p) {
  Words<N> r{};
  uint32_t carry = 0;
  for (int i = 0; i < N; i++) {
    r.w[i] = (x.w[i] << 1) | carry;
    carry = x.w[i] >> 31;
  }
  if (carry || words_ge(r, p)) r = words_sub(r, p);
  return r;
}

// 2^e mod p by repeated doubling
template <int N>
constexpr Words<N> pow2_mod(int e, const Words<N>& p) {
  Words<N> r{};
  r.w[0] = 1;
  if (words_ge(r, p)) r = words_sub(r, p);
  for (int i = 0; i < e; i++) r = dbl_mod(r, p);
  return r;
}

// (a * b) mod p, schoolbook shift-and-add (constexpr use only)
template <int N>
constexpr Words<N> mul_mod(const Words<N>& a, const Words<N>& b, const Words<N>& p) {
  Words<N> acc{};
  for (int bit = 32 * N - 1; bit >= 0; bit--) {
    acc = dbl_mod(acc, p);
    if ((b.w[bit / 32] >> (bit % 32)) & 1) {
      // acc = acc + a mod p
      Words<N> s{};
      uint64_t c = 0;
      for (int i = 0; i < N; i++) {
        uint64_t t = uint64_t(acc.w[i]) + a.w[i] + c;
        s.w[i] = uint32_t(t);
        c = t >> 32;
      }
      if (c || words_ge(s, p)) s = words_sub(s, p);
      acc = s;
    }
  }
  return acc;
}

// -p^-1 mod 2^32 by Newton iteration x <- x (2 - p x)
constexpr uint32_t neg_inv32(uint32_t p0) {
  uint32_t x = 1;
  for (int i = 0; i < 6; i++) x = x * (2u - p0 * x);
  return 0u - x;
}

template <int N>
constexpr Words<N> small_words(uint32_t v) {
  Words<N> r{};
  r.w[0] = v;
  return r;
}

// x 2^rbits mod p (to Montgomery form with R = 2^rbits) for a constant x < p
template <int N>
constexpr Words<N> to_mont_bits(const Words<N>& x, const Words<N>& p, int rbits) {
  return mul_mod(x, pow2_mod<N>(rbits, p), p);
}

}  // namespace eccmi

namespace eccmi {

// ---- limb representation in radix 2^B ------------------------------------

// B-bit limbs of a K-word integer (limb k holds bits [B k, B k + B))
template <int NL, int B, int K>
constexpr Words<NL> to_limbs(const Words<K>& x) {
  Words<NL> r{};
  for (int k = 0; k < NL; k++) {
    int bit = B * k;
    uint64_t v = 0;
    for (int j = 0; j < 2; j++) {  // B <= 32 bits from bit (bit % 32) span two words
      int w = bit / 32 + j;
      if (w < K) v |= uint64_t(x.w[w]) << (32 * j);
    }
    v >>= (bit % 32);
    r.w[k] = uint32_t(v & ((uint64_t(1) << B) - 1));
  }
  return r;
}

// x * 2^s for a K-word integer (bits shifted out of the top are lost)
template <int K>
constexpr Words<K> shl_words(const Words<K>& x, int s) {
  Words<K> r{};
  for (int i = K - 1; i >= 0; i--) {
    uint64_t v = 0;
    int src = i * 32 - s;  // bit index in x of r's word i low bit
    for (int b = 0; b < 32; b++) {
      int sb = src + b;
      if (sb >= 0 && sb < 32 * K && ((x.w[sb / 32] >> (sb % 32)) & 1u)) v |= uint64_t(1) << b;
    }
    r.w[i] = uint32_t(v);
  }
  return r;
}

template <int K, int N>
constexpr Words<K> widen(const Words<N>& x) {
  Words<K> r{};
  for (int i = 0; i < N && i < K; i++) r.w[i] = x.w[i];
  return r;
}

// -p^-1 mod 2^B
constexpr uint32_t neg_inv_bits(uint32_t p0, int B) {
  uint32_t x = 1;
  for (int i = 0; i < 6; i++) x = x * (2u - p0 * x);
  return (0u - x) & ((B == 32) ? 0xffffffffu : ((1u << B) - 1u));
}

// A multiple of p written with every limb below the top one at least 2^B
// (limb i gains 2^B, limb i + 1 loses 1): subtracting any normalised value
// from it limb by limb never goes negative.  Value unchanged.
template <int NL, int B>
constexpr Words<NL> redundant_limbs(const Words<NL>& v) {
  Words<NL> r = v;
  for (int i = 0; i + 1 < NL; i++) {
    r.w[i] += (1u << B);
    r.w[i + 1] -= 1u;
  }
  return r;
}

// Balanced radix-2^B digits of a value held in NL limbs: every digit but the
// top one lies in (-2^(B-1), 2^(B-1)], a digit above that range borrowing
// 2^B from the next.  The value is sum d_i 2^(B i), unchanged.
template <int N>
struct Digits {
  int32_t d[N];
};

template <int NL, int B>
constexpr Digits<NL> balanced_digits(const Words<NL>& v) {
  Digits<NL> r{};
  int64_t carry = 0;
  for (int i = 0; i < NL; i++) {
    int64_t t = int64_t(v.w[i]) + carry;
    carry = 0;
    if (i + 1 < NL && t > (int64_t(1) << (B - 1))) {
      t -= int64_t(1) << B;
      carry = 1;
    }
    r.d[i] = int32_t(t);
  }
  return r;
}

template <int NL>
constexpr int nonzero_digits(const Digits<NL>& x) {
  int c = 0;
  for (int i = 0; i < NL; i++) c += x.d[i] != 0;
  return c;
}

}  // namespace eccmi
