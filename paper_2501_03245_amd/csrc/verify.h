// Batched ECDSA verification on secp256r1.
//
// Per request: valid iff 1 <= r, s < n, Q is a curve point other than O, and
// with w = s^-1, u1 = e w, u2 = r w (mod n), R = u1 G + u2 Q is not O and
// R.x mod n = r.  The paper counts a verification as one fixed-point and one
// unknown-point multiplication (Section 5.2); here both run in one loop over
// the scalar bits from the least significant end, as in its batch PMUL
// (Section 3.3, Algorithm 4):
//
//   step j:  A1 <- A1 + 2^j G   if bit j of u1     (fixed point, table)
//            A2 <- A2 + P       if bit j of u2     (unknown point)
//            P  <- 2 P                              (P = 2^j Q)
//
// All three are affine operations whose denominators go into one
// Montgomery-trick chain per lane, inverted once per step for the whole
// workgroup (Gather-Apply-Scatter, Section 3.2).  The inverse of s mod n is
// batched the same way in F_n.  Finally R = A1 + A2 is one more batched step.
// One request per lane; lanes past the end run dummy requests so that every
// lane reaches every workgroup barrier.
#pragma once
#include "kernels.h"

namespace eccmi {

enum : int { OP_NOP = 5 };  // alongside CLS_ADD .. CLS_COPY2

template <class C>
struct AffOp {
  int cls;
  Fp<typename C::F> d;  // denominator put into the chain (1 when none is needed)
};

// affine A + B with A, B canonical (infinity flags ia, ib)
template <class C>
__device__ __forceinline__ AffOp<C> plan_add(const Affine<C>& A, bool ia, const Affine<C>& B, bool ib) {
  using F = typename C::F;
  AffOp<C> op;
  op.d = fp_one<F>();
  if (ia && ib) {
    op.cls = CLS_INF;
  } else if (ia) {
    op.cls = CLS_COPY2;
  } else if (ib) {
    op.cls = CLS_COPY1;
  } else if (fp_eq_canonical<F>(A.x, B.x)) {
    if (fp_eq_canonical<F>(A.y, B.y)) {
      op.cls = CLS_DBL;  // y != 0: these curves have no point of order 2
      op.d = fp_dbl<F>(A.y);
    } else {
      op.cls = CLS_INF;
    }
  } else {
    op.cls = CLS_ADD;
    op.d = fp_sub<F>(B.x, A.x);  // normalised: two denominators are multiplied together
  }
  return op;
}

// result of a planned addition given inv = 1 / op.d; canonical output
template <class C>
__device__ __forceinline__ void apply_add(const AffOp<C>& op, const Affine<C>& A, bool ia, const Affine<C>& B, bool ib,
                                          const Fp<typename C::F>& inv, Affine<C>& R, bool& rinf) {
  using F = typename C::F;
  if (op.cls == OP_NOP) {
    R = A;
    rinf = ia;
    return;
  }
  if (op.cls == CLS_INF) {
    rinf = true;
    R = A;
    return;
  }
  if (op.cls == CLS_COPY1) {
    R = A;
    rinf = false;
    return;
  }
  if (op.cls == CLS_COPY2) {
    R = B;
    rinf = false;
    return;
  }
  Fp<F> num = op.cls == CLS_DBL ? tangent_numerator<C>(A.x, fp_one<F>()) : fp_sub_lazy<F>(B.y, A.y);
  Fp<F> lam = fp_mul<F>(num, inv);
  Fp<F> x3 = fp_canonical<F>(fp_sub<F>(fp_sub<F>(fp_sqr<F>(lam), A.x), B.x));
  Fp<F> y3 = fp_canonical<F>(fp_sub<F>(fp_mul<F>(lam, fp_sub_lazy<F>(A.x, x3)), A.y));
  R.x = x3;
  R.y = y3;
  rinf = false;
}

template <class F>
__device__ __forceinline__ bool words_eq8(const uint32_t (&a)[8], const uint32_t (&b)[8]) {
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) d |= a[k] ^ b[k];
  return d == 0;
}

// a < b for 8-word little-endian integers
__device__ __forceinline__ bool words_lt8(const uint32_t (&a)[8], const uint32_t (&b)[8]) {
  bool lt = false, decided = false;
#pragma unroll
  for (int k = 7; k >= 0; k--) {
    if (!decided && a[k] != b[k]) {
      lt = a[k] < b[k];
      decided = true;
    }
  }
  return lt;
}

__device__ __forceinline__ bool words_zero8(const uint32_t (&a)[8]) {
  uint32_t o = 0;
#pragma unroll
  for (int k = 0; k < 8; k++) o |= a[k];
  return o == 0;
}

template <int WG>
__global__ void __launch_bounds__(WG) k_verify(const uint8_t* __restrict__ hashes, const uint32_t* __restrict__ pubkeys,
                                               const uint32_t* __restrict__ sigs, size_t m,
                                               const uint32_t* __restrict__ gtab, uint8_t* __restrict__ valid) {
  using C = P256;
  using F = FpP256;
  using N = FnP256;
  constexpr int PW = affine_words<C>();
  __shared__ Fp<F> s_tot[WG / 64], s_inv[WG / 64];
  __shared__ Fp<N> n_tot[WG / 64], n_inv[WG / 64];
  const size_t i = size_t(blockIdx.x) * WG + threadIdx.x;
  const bool live = i < m;

  // ---- load and range checks (dead or invalid requests continue with
  // dummy values: r = s = 1, Q = G) ----
  uint32_t rw[8], sw[8], ew[8], qx[8], qy[8];
  constexpr Words<8> n32 = N::P32;
  constexpr Words<8> p32 = F::P32;
  bool ok = live;
  if (live) {
    words_load<F>(sigs + i * 16, rw);
    words_load<F>(sigs + i * 16 + 8, sw);
    words_load<F>(pubkeys + i * 16, qx);
    words_load<F>(pubkeys + i * 16 + 8, qy);
    const uint8_t* h = hashes + i * 32;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint8_t* b = h + 28 - 4 * k;  // big-endian bytes, least significant word last
      ew[k] = (uint32_t(b[0]) << 24) | (uint32_t(b[1]) << 16) | (uint32_t(b[2]) << 8) | uint32_t(b[3]);
    }
    ok = !words_zero8(rw) && words_lt8(rw, n32.w) && !words_zero8(sw) && words_lt8(sw, n32.w) &&
         words_lt8(qx, p32.w) && words_lt8(qy, p32.w) && !(words_zero8(qx) && words_zero8(qy));
  }
  Affine<C> Q;
  if (ok) {
    Q.x = fp_canonical<F>(fp_to_mont<F>(fp_from_words<F>(qx)));
    Q.y = fp_canonical<F>(fp_to_mont<F>(fp_from_words<F>(qy)));
    ok = affine_on_curve<C>(Q);
  }
  if (!ok) {
#pragma unroll
    for (int k = 0; k < 8; k++) rw[k] = sw[k] = ew[k] = 0;
    rw[0] = sw[0] = 1;
    constexpr Words<F::NL> gx = C::GX, gy = C::GY;
    Q.x = fp_from<F>(gx);
    Q.y = fp_from<F>(gy);
  }

  // ---- w = s^-1, u1 = e w, u2 = r w (mod n), batched inversion in F_n ----
  Fp<N> wm = wg_batch_inverse<N, WG, 3>(fp_to_mont<N>(fp_from_words<N>(sw)), n_tot, n_inv);
  uint32_t u1[8], u2[8];
  fp_to_words<N>(fp_from_mont<N>(fp_mul<N>(fp_to_mont<N>(fp_from_words<N>(ew)), wm)), u1);
  fp_to_words<N>(fp_from_mont<N>(fp_mul<N>(fp_to_mont<N>(fp_from_words<N>(rw)), wm)), u2);

  // ---- the bit loop ----
  Affine<C> A1, A2, P = Q;
  bool i1 = true, i2 = true;
  A1.x = A1.y = A2.x = A2.y = fp_zero<F>();
  for (int j = 0; j < 256; j++) {
    const bool b1 = (u1[j >> 5] >> (j & 31)) & 1u;
    const bool b2 = (u2[j >> 5] >> (j & 31)) & 1u;
    const Affine<C> Gj = affine_load<C>(gtab + size_t(j) * PW);
    AffOp<C> oa, ob, oc;
    if (b1) {
      oa = plan_add<C>(A1, i1, Gj, false);
    } else {
      oa.cls = OP_NOP;
      oa.d = fp_one<F>();
    }
    if (b2) {
      ob = plan_add<C>(A2, i2, P, false);
    } else {
      ob.cls = OP_NOP;
      ob.d = fp_one<F>();
    }
    oc.cls = CLS_DBL;
    oc.d = fp_dbl<F>(P.y);
    const Fp<F> dab = fp_mul<F>(oa.d, ob.d);
    Fp<F> inv = wg_batch_inverse<F, WG, 4>(fp_mul<F>(dab, oc.d), s_tot, s_inv);
    const Fp<F> inv_c = fp_mul<F>(inv, dab);
    const Fp<F> inv_ab = fp_mul<F>(inv, oc.d);
    const Fp<F> inv_b = fp_mul<F>(inv_ab, oa.d);
    const Fp<F> inv_a = fp_mul<F>(inv_ab, ob.d);
    Affine<C> t;
    bool tinf;
    apply_add<C>(oa, A1, i1, Gj, false, inv_a, t, tinf);
    A1 = t;
    i1 = tinf;
    apply_add<C>(ob, A2, i2, P, false, inv_b, t, tinf);
    A2 = t;
    i2 = tinf;
    apply_add<C>(oc, P, false, P, false, inv_c, t, tinf);
    P = t;
  }
  // ---- R = A1 + A2 ----
  AffOp<C> of = plan_add<C>(A1, i1, A2, i2);
  Fp<F> inv = wg_batch_inverse<F, WG, 4>(of.d, s_tot, s_inv);
  Affine<C> R;
  bool rinf;
  apply_add<C>(of, A1, i1, A2, i2, inv, R, rinf);

  // ---- R.x mod n == r: R.x is below p < 2n, so R.x = r or R.x = r + n ----
  if (live) {
    bool good = ok && !rinf;
    if (good) {
      uint32_t xw[8];
      fp_to_words<F>(fp_from_mont<F>(R.x), xw);
      uint32_t rn[8];
      uint64_t cy = 0;
#pragma unroll
      for (int k = 0; k < 8; k++) {
        uint64_t v = uint64_t(rw[k]) + n32.w[k] + cy;
        rn[k] = uint32_t(v);
        cy = v >> 32;
      }
      good = words_eq8<F>(xw, rw) || (cy == 0 && words_eq8<F>(xw, rn));
    }
    valid[i] = good ? 1 : 0;
  }
}

}  // namespace eccmi
