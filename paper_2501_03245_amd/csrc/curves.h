// Curve and field parameter sets (short Weierstrass y^2 = x^3 + a x + b,
// Section 2.1 Eqn 1).  The paper evaluates SM2 only; this library serves
// BN254 G1 and BLS12-381 G1 (MSM) and secp256r1 (ECDSA verification) with the
// published parameters.  Derived Montgomery constants come from constants.h.
#pragma once
#include "constants.h"

namespace eccmi {

template <int N_, const char* P_HEX>
struct PrimeField {
  static constexpr int N = N_;                         // 32-bit words per element
  static constexpr Words<N> P = hex_words<N>(P_HEX);
  static constexpr uint32_t QINV = neg_inv32(P.w[0]);  // -p^-1 mod 2^32
  static constexpr Words<N> ONE = pow2_mod<N>(32 * N, P);   // R mod p
  static constexpr Words<N> R2 = pow2_mod<N>(64 * N, P);    // R^2 mod p
  static constexpr Words<N> R3 = pow2_mod<N>(96 * N, P);    // R^3 mod p
  static constexpr bool HEADROOM = has_headroom<N>(P);      // 4p < R
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
inline constexpr char ONE_HEX[] = "1";
inline constexpr char TWO_HEX[] = "2";
inline constexpr char THREE_HEX[] = "3";
inline constexpr char FOUR_HEX[] = "4";

using FpBN254 = PrimeField<8, BN254_P>;
using FpBLS = PrimeField<12, BLS_P>;
using FpP256 = PrimeField<8, P256_P>;
using FnP256 = PrimeField<8, P256_N>;

template <class F_, int ID_, const char* B_HEX, const char* GX_HEX, const char* GY_HEX, const char* R_HEX,
          bool A_IS_MINUS3_, int SCALAR_BITS_>
struct Curve {
  using F = F_;
  static constexpr int ID = ID_;
  static constexpr int N = F::N;
  static constexpr int LIMBS64 = F::N / 2;          // boundary limbs per coordinate
  static constexpr bool A_IS_MINUS3 = A_IS_MINUS3_;  // otherwise a = 0
  static constexpr Words<N> B_MONT = to_mont_const<N>(hex_words<N>(B_HEX), F::P);
  static constexpr Words<N> A_MONT =
      A_IS_MINUS3_ ? to_mont_const<N>(neg_const<N>(small_words<N>(3), F::P), F::P) : Words<N>{};
  static constexpr Words<N> GX = to_mont_const<N>(hex_words<N>(GX_HEX), F::P);
  static constexpr Words<N> GY = to_mont_const<N>(hex_words<N>(GY_HEX), F::P);
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

}  // namespace eccmi
