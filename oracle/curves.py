"""Curve parameter sets used by the oracle (short Weierstrass y^2 = x^3 + a x + b,
Section 2.1, Eqn 1).

The paper evaluates only SM2; the workloads here use the standard curves
below, SM2 among them.  Constants are the published ones (BN254 as used by
Ethereum's alt_bn128 precompiles, BLS12-381 from the Zcash/IETF
pairing-friendly-curves drafts, secp256r1 from NIST FIPS 186 / SEC 2, SM2 from
GB/T 32918.5).  They are pinned in the tests by independent facts: the BN and
BLS primes are re-derived from their curve-family polynomials, the P-256 and
SM2 primes from the sparse forms the paper and the standards state, the
generator lies on the curve, and order * G is the identity.
"""

from dataclasses import dataclass


@dataclass(frozen=True)
class Curve:
    name: str
    cid: int            # identifier used by the C oracle and the library ABI
    p: int              # field prime
    a: int
    b: int
    r: int              # prime order of the generator's subgroup
    gx: int
    gy: int
    limbs: int          # 64-bit limbs per coordinate

    @property
    def scalar_bits(self) -> int:
        return self.r.bit_length()


BN254 = Curve(
    name="bn254",
    cid=1,
    p=0x30644E72E131A029B85045B68181585D97816A916871CA8D3C208C16D87CFD47,
    a=0,
    b=3,
    r=0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001,
    gx=1,
    gy=2,
    limbs=4,
)

BLS12_381 = Curve(
    name="bls12_381",
    cid=2,
    p=int(
        "1a0111ea397fe69a4b1ba7b6434bacd764774b84f38512bf6730d2a0f6b0f624"
        "1eabfffeb153ffffb9feffffffffaaab", 16),
    a=0,
    b=4,
    r=0x73EDA753299D7D483339D80809A1D80553BDA402FFFE5BFEFFFFFFFF00000001,
    gx=int(
        "17f1d3a73197d7942695638c4fa9ac0fc3688c4f9774b905a14e3a3f171bac58"
        "6c55e83ff97a1aeffb3af00adb22c6bb", 16),
    gy=int(
        "08b3f481e3aaa0f1a09e30ed741d8ae4fcf5e095d5d00af600db18cb2c04b3ed"
        "d03cc744a2888ae40caa232946c5e7e1", 16),
    limbs=6,
)

SECP256R1 = Curve(
    name="secp256r1",
    cid=3,
    p=(1 << 256) - (1 << 224) + (1 << 192) + (1 << 96) - 1,
    a=((1 << 256) - (1 << 224) + (1 << 192) + (1 << 96) - 1) - 3,
    b=0x5AC635D8AA3A93E7B3EBBD55769886BC651D06B0CC53B0F63BCE3C3E27D2604B,
    r=0xFFFFFFFF00000000FFFFFFFFFFFFFFFFBCE6FAADA7179E84F3B9CAC2FC632551,
    gx=0x6B17D1F2E12C4247F8BCE6E563A440F277037D812DEB33A0F4A13945D898C296,
    gy=0x4FE342E2FE1A7F9B8EE7EB4A7C0F9E162BCE33576B315ECECBB6406837BF51F5,
    limbs=4,
)

# SM2 (the curve of the paper's evaluation, Section 5): published parameters
# of the Chinese standard GB/T 32918.5; p = 2^256 - 2^224 - 2^96 + 2^64 - 1,
# a = -3, cofactor 1
SM2 = Curve(
    name="sm2",
    cid=4,
    p=(1 << 256) - (1 << 224) - (1 << 96) + (1 << 64) - 1,
    a=((1 << 256) - (1 << 224) - (1 << 96) + (1 << 64) - 1) - 3,
    b=0x28E9FA9E9D9F5E344D5A9E4BCF6509A7F39789F515AB8F92DDBCBD414D940E93,
    r=0xFFFFFFFEFFFFFFFFFFFFFFFFFFFFFFFF7203DF6B21C6052B53BBF40939D54123,
    gx=0x32C4AE2C1F1981195F9904466A39C9948FE30BBFF2660BE1715A4589334C74C7,
    gy=0xBC3736A2F4F6779C59BDCEE36B692153D0A9877CC62A474002DF32E52139F0A0,
    limbs=4,
)

CURVES = {c.name: c for c in (BN254, BLS12_381, SECP256R1, SM2)}
BY_ID = {c.cid: c for c in (BN254, BLS12_381, SECP256R1, SM2)}
