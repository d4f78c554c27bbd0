// Curve and field parameter sets (short Weierstrass y^2 = x^3 + a x + b,
// Section 2.1 Eqn 1).  The paper evaluates SM2 only; this library serves
// BN254 G1 and BLS12-381 G1 (MSM) and secp256r1 (ECDSA verification) with the
// published parameters.  Derived Montgomery constants come from constants.h.
#pragma once
#include "constants.h"

namespace eccmi {

// A prime field in two representations:
//  * I/O form: N32 little-endian 32-bit words, canonical in [0, p);
//  * working form: NL limbs of B bits (radix 2^B, B < 32) in 32-bit registers,
//    Montgomery form with R = 2^(B NL).  The unused top bits of every limb let
//    sums and products accumulate without carry flags.
template <int N32_, int NL_, int B_, const char* P_HEX>
struct PrimeField {
  static constexpr int N32 = N32_;
  static constexpr int NL = NL_;
  static constexpr int B = B_;
  static constexpr int CW = (NL + 3) / 4 * 4;  // stored words per coordinate (16-byte multiple)
  static constexpr uint32_t MASK = (1u << B) - 1u;
  static constexpr Words<N32> P32 = hex_words<N32>(P_HEX);
  static constexpr Words<NL> P = to_limbs<NL, B, N32>(P32);
  static constexpr Words<NL> P2 = to_limbs<NL, B, N32 + 1>(shl_words<N32 + 1>(widen<N32 + 1, N32>(P32), 1));
  static constexpr Words<NL> P4 = to_limbs<NL, B, N32 + 1>(shl_words<N32 + 1>(widen<N32 + 1, N32>(P32), 2));
  static constexpr Words<NL> KP = redundant_limbs<NL, B>(P4);  // 4p, lower limbs >= 2^B
  static constexpr uint32_t QINV = neg_inv_bits(P.w[0], B);  // -p^-1 mod 2^B
  // balanced digits of p; a prime with p = -1 mod 2^B (q_inv = 1) and at most
  // NL / 2 nonzero digits takes the sparse Montgomery reduction of field.h
  static constexpr Digits<NL> SD = balanced_digits<NL, B>(P);
  static constexpr bool SPARSE = QINV == 1u && SD.d[0] == -1 && nonzero_digits<NL>(SD) <= NL / 2;
  static constexpr int RBITS = NL * B;
  static constexpr Words<NL> ONE = to_limbs<NL, B, N32>(pow2_mod<N32>(RBITS, P32));     // R mod p
  static constexpr Words<NL> R2 = to_limbs<NL, B, N32>(pow2_mod<N32>(2 * RBITS, P32));  // R^2 mod p
  static constexpr Words<NL> R3 = to_limbs<NL, B, N32>(pow2_mod<N32>(3 * RBITS, P32));  // R^3 mod p
  // the boundary's Montgomery form uses R' = 2^(32 N32): converting x R' to
  // x R is a Montgomery product with R^2 / R', and back with R' (plain)
  static constexpr Words<NL> RIN = to_limbs<NL, B, N32>(pow2_mod<N32>(2 * RBITS - 32 * N32, P32));
  static constexpr Words<NL> ROUT = to_limbs<NL, B, N32>(pow2_mod<N32>(32 * N32, P32));
};

inline constexpr char BN254_P[] = "30644e72e131a029b85045b68181585d97816a916871ca8d3c208c16d87cfd47";
inline constexpr char BN254_R[] = "30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001";
inline constexpr char BLS_P[] =
    "1a0111ea397fe69a4b1ba7b6434bacd764774b84f38512bf6730d2a0f6b0f6241eabfffeb153ffffb9feffffffffaaab";
inline constexpr char BLS_R[] = "73eda753299d7d483339d80809a1d80553bda402fffe5bfeffffffff00000001";
inline constexpr char BLS_GX[] =
    "17f1d3a73197d7942695638c4fa9ac0fc3688c4f9774b905a14e3a3f171bac586c55e83ff97a1aeffb3af00adb22c6bb";
inline constexpr char BLS_GY[] =
    "08b3f481e3aaa0f1a09e30ed741d8ae4fcf5e095d5d00af600db18cb2c04b3edd03cc744a2888ae40caa232946c5e7e1";
inline constexpr char P256_P[] = "ffffffff00000001000000000000000000000000ffffffffffffffffffffffff";
inline constexpr char P256_N[] = "ffffffff00000000ffffffffffffffffbce6faada7179e84f3b9cac2fc632551";
inline constexpr char P256_B[] = "5ac635d8aa3a93e7b3ebbd55769886bc651d06b0cc53b0f63bce3c3e27d2604b";
inline constexpr char P256_GX[] = "6b17d1f2e12c4247f8bce6e563a440f277037d812deb33a0f4a13945d898c296";
inline constexpr char P256_GY[] = "4fe342e2fe1a7f9b8ee7eb4a7c0f9e162bce33576b315ececbb6406837bf51f5";

// BN254: 9 limbs of 29 bits (R = 2^261); BLS12-381: 14 limbs of 28 bits
// (R = 2^392); secp256r1: 10 limbs of 28 bits (R = 2^280).  In each case
// 12 p < R, so a Montgomery product with one operand below 2p and the other
// below 6p lands below 2p.
using FpBN254 = PrimeField<8, 9, 29, BN254_P>;
using FpBLS = PrimeField<12, 14, 28, BLS_P>;
using FpP256 = PrimeField<8, 10, 28, P256_P>;
using FnP256 = PrimeField<8, 10, 28, P256_N>;

// SM2 (GB/T 32918.5), the curve of the paper's evaluation: its prime
// 2^256 - 2^224 - 2^96 + 2^64 - 1 is the one Section 4.2's reduction is built
// for, and takes the sparse reduction of field.h (radix-2^28 digits -1,
// 2^8 D^2, -2^12 D^3, -D^8, 16 D^9)
inline constexpr char SM2_P[] = "fffffffeffffffffffffffffffffffffffffffff00000000ffffffffffffffff";
inline constexpr char SM2_N[] = "fffffffeffffffffffffffffffffffff7203df6b21c6052b53bbf40939d54123";
inline constexpr char SM2_B[] = "28e9fa9e9d9f5e344d5a9e4bcf6509a7f39789f515ab8f92ddbcbd414d940e93";
inline constexpr char SM2_GX[] = "32c4ae2c1f1981195f9904466a39c9948fe30bbff2660be1715a4589334c74c7";
inline constexpr char SM2_GY[] = "bc3736a2f4f6779c59bdcee36b692153d0a9877cc62a474002df32e52139f0a0";
using FpSM2 = PrimeField<8, 10, 28, SM2_P>;
using FnSM2 = PrimeField<8, 10, 28, SM2_N>;

template <class F_, int ID_, const char* B_HEX, const char* GX_HEX, const char* GY_HEX, const char* R_HEX,
          bool A_IS_MINUS3_, int SCALAR_BITS_>
struct Curve {
  using F = F_;
  static constexpr int ID = ID_;
  static constexpr int NL = F::NL;
  static constexpr int N32 = F::N32;
  static constexpr int LIMBS64 = F::N32 / 2;         // boundary limbs per coordinate
  static constexpr bool A_IS_MINUS3 = A_IS_MINUS3_;  // otherwise a = 0
  static constexpr Words<NL> B_MONT = to_limbs<NL, F::B, N32>(to_mont_bits<N32>(hex_words<N32>(B_HEX), F::P32, F::RBITS));
  static constexpr Words<NL> GX = to_limbs<NL, F::B, N32>(to_mont_bits<N32>(hex_words<N32>(GX_HEX), F::P32, F::RBITS));
  static constexpr Words<NL> GY = to_limbs<NL, F::B, N32>(to_mont_bits<N32>(hex_words<N32>(GY_HEX), F::P32, F::RBITS));
  static constexpr Words<8> ORDER = hex_words<8>(R_HEX);  // group order r (256-bit words)
  static constexpr int SCALAR_BITS = SCALAR_BITS_;        // bit length of r
};

inline constexpr char BN254_B[] = "3";
inline constexpr char BN254_GX[] = "1";
inline constexpr char BN254_GY[] = "2";
inline constexpr char BLS_B[] = "4";

using BN254 = Curve<FpBN254, 1, BN254_B, BN254_GX, BN254_GY, BN254_R, false, 254>;
using BLS12_381 = Curve<FpBLS, 2, BLS_B, BLS_GX, BLS_GY, BLS_R, false, 255>;
using P256 = Curve<FpP256, 3, P256_B, P256_GX, P256_GY, P256_N, true, 256>;
using SM2 = Curve<FpSM2, 4, SM2_B, SM2_GX, SM2_GY, SM2_N, true, 256>;

// the field of scalars mod the group order n, for the curves that sign and
// verify (ECDSA)
template <class C>
struct OrderField;
template <>
struct OrderField<P256> {
  using type = FnP256;
};
template <>
struct OrderField<SM2> {
  using type = FnSM2;
};

// Endomorphism split (Gallant-Lambert-Vanstone).  On BN254 and BLS12-381
// (a = 0) the map (x, y) -> (beta x, y), beta a cube root of unity mod p, acts
// on the order-r subgroup as multiplication by lambda, a cube root of unity
// mod r (beta and lambda below are the pair that match on the generator).  A
// scalar k is written k = k1 + lambda k2 (mod r) by Babai rounding against a
// reduced basis v1 = (A1, B1), v2 = (A2, B2) of the lattice
// {(x, y) : x + lambda y = 0 mod r}, whose determinant is +-r:
//   c1 = round(k G1 / 2^320), c2 = round(k G2 / 2^320),
//   G1 = round(2^320 |B2| / r), G2 = round(2^320 |B1| / r)
// (for both curves the rounding coefficients k B2 / det and -k B1 / det are
// non-negative), then k1 = k - c1 A1 - c2 A2, k2 = -c1 B1 - c2 B2, so that
// |k1|, |k2| < 2^BITS.  The basis entries are 192-bit two's complement
// (three 64-bit words, least significant first).
template <class C>
struct Glv {
  static constexpr bool HAS = false;
};

inline constexpr char BN254_BETA[] = "59e26bcea0d48bacd4f263f1acdb5c4f5763473177fffffe";
inline constexpr char BLS_BETA[] =
    "1a0111ea397fe699ec02408663d4de85aa0d857d89759ad4897d29650fb85f9b409427eb4f49fffd8bfd00000000aaac";

template <>
struct Glv<BN254> {
  using F = BN254::F;
  static constexpr bool HAS = true;
  static constexpr int BITS = 126;
  static constexpr Words<F::NL> BETA =
      to_limbs<F::NL, F::B, F::N32>(to_mont_bits<F::N32>(hex_words<F::N32>(BN254_BETA), F::P32, F::RBITS));
  static constexpr uint64_t A1[3] = {0x89d3256894d213e3ull, 0x0ull, 0x0ull};
  static constexpr uint64_t B1[3] = {0x7dee441482b0eed8ull, 0x90b27db71147a603ull, 0xffffffffffffffffull};
  static constexpr uint64_t A2[3] = {0x0be4e1541221250bull, 0x6f4d8248eeb859fdull, 0x0ull};
  static constexpr uint64_t B2[3] = {0x89d3256894d213e3ull, 0x0ull, 0x0ull};
  static constexpr uint64_t G1[4] = {0x6eb9c714773a6ef3ull, 0xd91d232ec7e0b3d7ull, 0x2ull, 0x0ull};
  static constexpr uint64_t G2[4] = {0xa5e38cfb5eaa26daull, 0x7a7bd9d4391eb18dull, 0x4ccef014a773d2cfull, 0x2ull};
};

// BLS12-381: lambda = z^2 - 1 for the curve parameter z, r = lambda^2 + lambda + 1,
// basis v1 = (1, lambda + 1), v2 = (lambda, -1)
template <>
struct Glv<BLS12_381> {
  using F = BLS12_381::F;
  static constexpr bool HAS = true;
  static constexpr int BITS = 127;
  static constexpr Words<F::NL> BETA =
      to_limbs<F::NL, F::B, F::N32>(to_mont_bits<F::N32>(hex_words<F::N32>(BLS_BETA), F::P32, F::RBITS));
  static constexpr uint64_t A1[3] = {0x1ull, 0x0ull, 0x0ull};
  static constexpr uint64_t B1[3] = {0x0000000100000000ull, 0xac45a4010001a402ull, 0x0ull};
  static constexpr uint64_t A2[3] = {0x00000000ffffffffull, 0xac45a4010001a402ull, 0x0ull};
  static constexpr uint64_t B2[3] = {0xffffffffffffffffull, 0xffffffffffffffffull, 0xffffffffffffffffull};
  static constexpr uint64_t G1[4] = {0x355094edfede377cull, 0x2ull, 0x0ull, 0x0ull};
  static constexpr uint64_t G2[4] = {0x389f49a7268bf7a4ull, 0x63f6e522f6cfee30ull, 0x7c6becf1e01faaddull, 0x1ull};
};

}  // namespace eccmi
