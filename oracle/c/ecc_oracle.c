/*
 * Plain C oracle for the elliptic-curve operations of the MSM / ECDSA path.
 *
 * TEST INFRASTRUCTURE ONLY: linked by the tests and by the benchmark's CPU
 * baseline, never by the product library.  It shares no code with it.
 *
 * What it computes (the plain definitions, no Pippenger, no batching):
 *   - F_p arithmetic on 64-bit limbs: schoolbook products (unsigned __int128)
 *     reduced by Barrett's method (Handbook of Applied Cryptography, Alg 14.42)
 *     with mu = floor(2^(128 L) / p) found by bit-serial long division;
 *     inversion by Fermat's little theorem, x^(p-2) (Section 2.2 names it as
 *     one of the two standard inversion methods).
 *   - the short-Weierstrass group law (Section 2.1, Eqn 1) in Jacobian
 *     coordinates x = X/Z^2, y = Y/Z^3 with every exceptional case
 *     (O operands, P = Q, P = -Q), normalised to affine at the end;
 *   - scalar multiplication by double-and-add, least significant bit first
 *     (Algorithm 1);
 *   - MSM as the literal sum of the scalar multiples, split over threads;
 *   - ECDSA verification: 1 <= r,s < n, Q on the curve, w = s^-1 mod n,
 *     u1 = e w, u2 = r w, R = u1 G + u2 Q, valid iff R != O and R.x mod n = r.
 *
 * Boundary conventions: coordinates are canonical (non-Montgomery) affine,
 * L little-endian u64 limbs each (x then y); (0,0) encodes the point at
 * infinity (never on these curves since b != 0); scalars are 4 u64 limbs.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
#define MAXL 6

typedef struct {
  int L;               /* limbs */
  uint64_t m[MAXL];    /* modulus */
  uint64_t mu[MAXL + 1];
} modulus_t;

typedef struct {
  int id;
  int L;
  modulus_t p;         /* field prime */
  modulus_t n;         /* group order */
  uint64_t a[MAXL];    /* curve a (canonical) */
  uint64_t b[MAXL];
  uint64_t gx[MAXL], gy[MAXL];
} curve_t;

/* ---------------- multi-precision helpers (k limbs) ---------------------- */

static int mp_cmp(const uint64_t *x, const uint64_t *y, int k) {
  for (int i = k - 1; i >= 0; i--) {
    if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
  }
  return 0;
}

static uint64_t mp_add(uint64_t *r, const uint64_t *x, const uint64_t *y, int k) {
  uint64_t c = 0;
  for (int i = 0; i < k; i++) {
    u128 s = (u128)x[i] + y[i] + c;
    r[i] = (uint64_t)s;
    c = (uint64_t)(s >> 64);
  }
  return c;
}

static uint64_t mp_sub(uint64_t *r, const uint64_t *x, const uint64_t *y, int k) {
  uint64_t br = 0;
  for (int i = 0; i < k; i++) {
    u128 d = (u128)x[i] - y[i] - br;
    r[i] = (uint64_t)d;
    br = (uint64_t)(d >> 64) & 1;
  }
  return br;
}

static int mp_is_zero(const uint64_t *x, int k) {
  for (int i = 0; i < k; i++)
    if (x[i]) return 0;
  return 1;
}

/* full product r[kx+ky] = x * y (schoolbook) */
static void mp_mul(uint64_t *r, const uint64_t *x, int kx, const uint64_t *y, int ky) {
  for (int i = 0; i < kx + ky; i++) r[i] = 0;
  for (int i = 0; i < kx; i++) {
    uint64_t c = 0;
    for (int j = 0; j < ky; j++) {
      u128 t = (u128)x[i] * y[j] + r[i + j] + c;
      r[i + j] = (uint64_t)t;
      c = (uint64_t)(t >> 64);
    }
    r[i + ky] = c;
  }
}

/* mu = floor(2^(128 L) / m) by bit-serial long division (rem < 2m fits L+1 limbs) */
static void modulus_init(modulus_t *M, const uint64_t *m, int L) {
  M->L = L;
  memcpy(M->m, m, sizeof(uint64_t) * L);
  uint64_t rem[MAXL + 1] = {0}, mm[MAXL + 1] = {0};
  memcpy(mm, m, sizeof(uint64_t) * L);
  for (int i = 0; i <= MAXL; i++) M->mu[i] = 0;
  int top = 128 * L; /* dividend = 2^top */
  for (int bit = top; bit >= 0; bit--) {
    /* rem = 2 rem + (bit == top) */
    uint64_t carry = (bit == top) ? 1 : 0;
    for (int i = 0; i <= L; i++) {
      uint64_t nc = rem[i] >> 63;
      rem[i] = (rem[i] << 1) | carry;
      carry = nc;
    }
    if (mp_cmp(rem, mm, L + 1) >= 0) {
      mp_sub(rem, rem, mm, L + 1);
      if (bit / 64 <= L) M->mu[bit / 64] |= (uint64_t)1 << (bit % 64);
    }
  }
}

/* r = x mod m for x < m^2 (2L limbs): Barrett reduction, HAC Alg 14.42 */
static void mod_reduce(const modulus_t *M, uint64_t *r, const uint64_t *x) {
  int k = M->L;
  uint64_t q2[2 * MAXL + 2], t[2 * MAXL + 2];
  const uint64_t *q1 = x + (k - 1);             /* floor(x / b^(k-1)), k+1 limbs */
  mp_mul(q2, q1, k + 1, M->mu, k + 1);          /* q2 = q1 * mu */
  const uint64_t *q3 = q2 + (k + 1);            /* floor(q2 / b^(k+1)), k+1 limbs */
  mp_mul(t, q3, k + 1, M->m, k);                /* q3 * m, keep low k+1 limbs */
  uint64_t r1[MAXL + 1], r2[MAXL + 1], mm[MAXL + 1];
  memcpy(r1, x, sizeof(uint64_t) * (k + 1));
  memcpy(r2, t, sizeof(uint64_t) * (k + 1));
  mp_sub(r1, r1, r2, k + 1);                    /* mod b^(k+1) */
  memcpy(mm, M->m, sizeof(uint64_t) * k);
  mm[k] = 0;
  while (mp_cmp(r1, mm, k + 1) >= 0) mp_sub(r1, r1, mm, k + 1);
  memcpy(r, r1, sizeof(uint64_t) * k);
}

static void mod_mul(const modulus_t *M, uint64_t *r, const uint64_t *x, const uint64_t *y) {
  uint64_t t[2 * MAXL];
  mp_mul(t, x, M->L, y, M->L);
  mod_reduce(M, r, t);
}

static void mod_add(const modulus_t *M, uint64_t *r, const uint64_t *x, const uint64_t *y) {
  uint64_t t[MAXL];
  int k = M->L;
  uint64_t c = mp_add(t, x, y, k);
  if (c || mp_cmp(t, M->m, k) >= 0) mp_sub(t, t, M->m, k);
  memcpy(r, t, sizeof(uint64_t) * k);
}

static void mod_sub(const modulus_t *M, uint64_t *r, const uint64_t *x, const uint64_t *y) {
  uint64_t t[MAXL];
  int k = M->L;
  if (mp_sub(t, x, y, k)) mp_add(t, t, M->m, k);
  memcpy(r, t, sizeof(uint64_t) * k);
}

/* r = x^e mod m, square-and-multiply from the top bit of e (ke limbs) */
static void mod_pow(const modulus_t *M, uint64_t *r, const uint64_t *x, const uint64_t *e, int ke) {
  int k = M->L;
  uint64_t acc[MAXL] = {0};
  acc[0] = 1;
  for (int i = ke * 64 - 1; i >= 0; i--) {
    mod_mul(M, acc, acc, acc);
    if ((e[i / 64] >> (i % 64)) & 1) mod_mul(M, acc, acc, x);
  }
  memcpy(r, acc, sizeof(uint64_t) * k);
}

/* Fermat: x^(m-2) */
static void mod_inv(const modulus_t *M, uint64_t *r, const uint64_t *x) {
  uint64_t e[MAXL], two[MAXL] = {0};
  two[0] = 2;
  mp_sub(e, M->m, two, M->L);
  mod_pow(M, r, x, e, M->L);
}

/* ---------------- curves ----------------------------------------------- */

static int hexval(char c) {
  if (c >= '0' && c <= '9') return c - '0';
  if (c >= 'a' && c <= 'f') return c - 'a' + 10;
  if (c >= 'A' && c <= 'F') return c - 'A' + 10;
  return -1;
}

static void from_hex(uint64_t *r, int L, const char *s) {
  for (int i = 0; i < L; i++) r[i] = 0;
  int n = (int)strlen(s);
  for (int i = 0; i < n; i++) {
    int v = hexval(s[n - 1 - i]);
    r[i / 16] |= (uint64_t)v << (4 * (i % 16));
  }
}

static curve_t CURVES[5];
static int curves_ready = 0;
static pthread_mutex_t curves_lock = PTHREAD_MUTEX_INITIALIZER;

static void setup_curve(curve_t *c, int id, int L, const char *p, const char *n, const char *a, const char *b,
                        const char *gx, const char *gy) {
  uint64_t t[MAXL];
  c->id = id;
  c->L = L;
  from_hex(t, L, p);
  modulus_init(&c->p, t, L);
  from_hex(t, 4, n);
  modulus_init(&c->n, t, 4);
  from_hex(c->a, L, a);
  from_hex(c->b, L, b);
  from_hex(c->gx, L, gx);
  from_hex(c->gy, L, gy);
}

static void init_curves(void) {
  pthread_mutex_lock(&curves_lock);
  if (!curves_ready) {
    setup_curve(&CURVES[1], 1, 4, "30644e72e131a029b85045b68181585d97816a916871ca8d3c208c16d87cfd47",
                "30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001", "0", "3", "1", "2");
    setup_curve(&CURVES[2], 2, 6,
                "1a0111ea397fe69a4b1ba7b6434bacd764774b84f38512bf6730d2a0f6b0f6241eabfffeb153ffffb9feffffffffaaab",
                "73eda753299d7d483339d80809a1d80553bda402fffe5bfeffffffff00000001", "0", "4",
                "17f1d3a73197d7942695638c4fa9ac0fc3688c4f9774b905a14e3a3f171bac586c55e83ff97a1aeffb3af00adb22c6bb",
                "08b3f481e3aaa0f1a09e30ed741d8ae4fcf5e095d5d00af600db18cb2c04b3edd03cc744a2888ae40caa232946c5e7e1");
    setup_curve(&CURVES[3], 3, 4, "ffffffff00000001000000000000000000000000ffffffffffffffffffffffff",
                "ffffffff00000000ffffffffffffffffbce6faada7179e84f3b9cac2fc632551",
                "ffffffff00000001000000000000000000000000fffffffffffffffffffffffc",
                "5ac635d8aa3a93e7b3ebbd55769886bc651d06b0cc53b0f63bce3c3e27d2604b",
                "6b17d1f2e12c4247f8bce6e563a440f277037d812deb33a0f4a13945d898c296",
                "4fe342e2fe1a7f9b8ee7eb4a7c0f9e162bce33576b315ececbb6406837bf51f5");
    /* SM2 (GB/T 32918.5) */
    setup_curve(&CURVES[4], 4, 4, "fffffffeffffffffffffffffffffffffffffffff00000000ffffffffffffffff",
                "fffffffeffffffffffffffffffffffff7203df6b21c6052b53bbf40939d54123",
                "fffffffeffffffffffffffffffffffffffffffff00000000fffffffffffffffc",
                "28e9fa9e9d9f5e344d5a9e4bcf6509a7f39789f515ab8f92ddbcbd414d940e93",
                "32c4ae2c1f1981195f9904466a39c9948fe30bbff2660be1715a4589334c74c7",
                "bc3736a2f4f6779c59bdcee36b692153d0a9877cc62a474002df32e52139f0a0");
    curves_ready = 1;
  }
  pthread_mutex_unlock(&curves_lock);
}

static const curve_t *get_curve(int id) {
  init_curves();
  if (id < 1 || id > 4) return NULL;
  return &CURVES[id];
}

/* ---------------- Jacobian points ------------------------------------- */

typedef struct {
  uint64_t X[MAXL], Y[MAXL], Z[MAXL]; /* Z = 0 encodes O */
} jac_t;

static void jac_set_inf(const curve_t *c, jac_t *P) {
  memset(P, 0, sizeof(*P));
  P->X[0] = 1;
  P->Y[0] = 1;
  (void)c;
}

static int jac_is_inf(const curve_t *c, const jac_t *P) { return mp_is_zero(P->Z, c->L); }

static void jac_from_affine(const curve_t *c, jac_t *P, const uint64_t *x, const uint64_t *y) {
  int L = c->L;
  if (mp_is_zero(x, L) && mp_is_zero(y, L)) {
    jac_set_inf(c, P);
    return;
  }
  memcpy(P->X, x, 8 * L);
  memcpy(P->Y, y, 8 * L);
  memset(P->Z, 0, sizeof(P->Z));
  P->Z[0] = 1;
}

/* doubling: M = 3X^2 + a Z^4, S = 4 X Y^2, X' = M^2 - 2S, Y' = M(S - X') - 8 Y^4, Z' = 2 Y Z */
static void jac_dbl(const curve_t *c, jac_t *R, const jac_t *P) {
  const modulus_t *F = &c->p;
  if (jac_is_inf(c, P) || mp_is_zero(P->Y, c->L)) {
    jac_set_inf(c, R);
    return;
  }
  uint64_t XX[MAXL], YY[MAXL], YYYY[MAXL], ZZ[MAXL], S[MAXL], M[MAXL], T[MAXL], X3[MAXL], Y3[MAXL], Z3[MAXL];
  mod_mul(F, XX, P->X, P->X);
  mod_mul(F, YY, P->Y, P->Y);
  mod_mul(F, YYYY, YY, YY);
  mod_mul(F, ZZ, P->Z, P->Z);
  mod_mul(F, S, P->X, YY);
  mod_add(F, S, S, S);
  mod_add(F, S, S, S); /* 4 X Y^2 */
  mod_add(F, M, XX, XX);
  mod_add(F, M, M, XX); /* 3 X^2 */
  if (!mp_is_zero(c->a, c->L)) {
    mod_mul(F, T, ZZ, ZZ);
    mod_mul(F, T, T, c->a);
    mod_add(F, M, M, T);
  }
  mod_mul(F, X3, M, M);
  mod_sub(F, X3, X3, S);
  mod_sub(F, X3, X3, S);
  mod_sub(F, T, S, X3);
  mod_mul(F, Y3, M, T);
  mod_add(F, T, YYYY, YYYY);
  mod_add(F, T, T, T);
  mod_add(F, T, T, T); /* 8 Y^4 */
  mod_sub(F, Y3, Y3, T);
  mod_mul(F, Z3, P->Y, P->Z);
  mod_add(F, Z3, Z3, Z3);
  memcpy(R->X, X3, sizeof(X3));
  memcpy(R->Y, Y3, sizeof(Y3));
  memcpy(R->Z, Z3, sizeof(Z3));
}

/* general addition with the full case analysis */
static void jac_add(const curve_t *c, jac_t *R, const jac_t *P, const jac_t *Q) {
  const modulus_t *F = &c->p;
  int L = c->L;
  if (jac_is_inf(c, P)) {
    *R = *Q;
    return;
  }
  if (jac_is_inf(c, Q)) {
    *R = *P;
    return;
  }
  uint64_t Z1Z1[MAXL], Z2Z2[MAXL], U1[MAXL], U2[MAXL], S1[MAXL], S2[MAXL], H[MAXL], Rr[MAXL], HH[MAXL],
      HHH[MAXL], V[MAXL], T[MAXL], X3[MAXL], Y3[MAXL], Z3[MAXL];
  mod_mul(F, Z1Z1, P->Z, P->Z);
  mod_mul(F, Z2Z2, Q->Z, Q->Z);
  mod_mul(F, U1, P->X, Z2Z2);
  mod_mul(F, U2, Q->X, Z1Z1);
  mod_mul(F, S1, P->Y, Q->Z);
  mod_mul(F, S1, S1, Z2Z2);
  mod_mul(F, S2, Q->Y, P->Z);
  mod_mul(F, S2, S2, Z1Z1);
  if (mp_cmp(U1, U2, L) == 0) {
    if (mp_cmp(S1, S2, L) == 0) {
      jac_dbl(c, R, P);
    } else {
      jac_set_inf(c, R);
    }
    return;
  }
  mod_sub(F, H, U2, U1);
  mod_sub(F, Rr, S2, S1);
  mod_mul(F, HH, H, H);
  mod_mul(F, HHH, HH, H);
  mod_mul(F, V, U1, HH);
  mod_mul(F, X3, Rr, Rr);
  mod_sub(F, X3, X3, HHH);
  mod_sub(F, X3, X3, V);
  mod_sub(F, X3, X3, V);
  mod_sub(F, T, V, X3);
  mod_mul(F, Y3, Rr, T);
  mod_mul(F, T, S1, HHH);
  mod_sub(F, Y3, Y3, T);
  mod_mul(F, Z3, P->Z, Q->Z);
  mod_mul(F, Z3, Z3, H);
  memcpy(R->X, X3, sizeof(X3));
  memcpy(R->Y, Y3, sizeof(Y3));
  memcpy(R->Z, Z3, sizeof(Z3));
}

static void jac_to_affine(const curve_t *c, const jac_t *P, uint64_t *x, uint64_t *y, uint8_t *inf) {
  int L = c->L;
  const modulus_t *F = &c->p;
  if (jac_is_inf(c, P)) {
    memset(x, 0, 8 * L);
    memset(y, 0, 8 * L);
    if (inf) *inf = 1;
    return;
  }
  uint64_t zi[MAXL], zi2[MAXL], zi3[MAXL];
  mod_inv(F, zi, P->Z);
  mod_mul(F, zi2, zi, zi);
  mod_mul(F, zi3, zi2, zi);
  mod_mul(F, x, P->X, zi2);
  mod_mul(F, y, P->Y, zi3);
  if (inf) *inf = 0;
}

/* Algorithm 1: for i = 0 .. l-1: if s_i then Q = Q + P; P = P + P */
static void jac_scalar_mul(const curve_t *c, jac_t *Q, const jac_t *P0, const uint64_t *s, int words) {
  jac_t P = *P0, acc;
  jac_set_inf(c, &acc);
  int top = words * 64 - 1;
  while (top >= 0 && !((s[top / 64] >> (top % 64)) & 1)) top--;
  for (int i = 0; i <= top; i++) {
    if ((s[i / 64] >> (i % 64)) & 1) jac_add(c, &acc, &acc, &P);
    if (i < top) jac_dbl(c, &P, &P);
  }
  *Q = acc;
}

static int affine_on_curve(const curve_t *c, const uint64_t *x, const uint64_t *y) {
  const modulus_t *F = &c->p;
  int L = c->L;
  if (mp_cmp(x, F->m, L) >= 0 || mp_cmp(y, F->m, L) >= 0) return 0;
  uint64_t l[MAXL], r[MAXL], t[MAXL];
  mod_mul(F, l, y, y);
  mod_mul(F, r, x, x);
  mod_mul(F, r, r, x);
  mod_mul(F, t, c->a, x);
  mod_add(F, r, r, t);
  mod_add(F, r, r, c->b);
  return mp_cmp(l, r, L) == 0;
}

/* ---------------- threading -------------------------------------------- */

typedef struct {
  const curve_t *c;
  const uint64_t *bases, *scalars;
  size_t lo, hi;
  jac_t acc;
  uint64_t *out; /* fixed-base output */
  const jac_t *table;
  int mode; /* 0 msm, 1 fixed base */
} job_t;

static void *msm_worker(void *arg) {
  job_t *j = (job_t *)arg;
  const curve_t *c = j->c;
  int L = c->L;
  jac_set_inf(c, &j->acc);
  for (size_t i = j->lo; i < j->hi; i++) {
    jac_t P, T;
    jac_from_affine(c, &P, j->bases + i * 2 * L, j->bases + i * 2 * L + L);
    jac_scalar_mul(c, &T, &P, j->scalars + 4 * i, 4);
    jac_add(c, &j->acc, &j->acc, &T);
  }
  return NULL;
}

/* k_i G with a table of 2^j G (double-and-add where the doublings of G are
   precomputed, i.e. the fixed-point variant of Algorithm 1) */
static void *fixed_worker(void *arg) {
  job_t *j = (job_t *)arg;
  const curve_t *c = j->c;
  int L = c->L;
  for (size_t i = j->lo; i < j->hi; i++) {
    jac_t acc;
    jac_set_inf(c, &acc);
    const uint64_t *k = j->scalars + 4 * i;
    for (int b = 0; b < 256; b++)
      if ((k[b / 64] >> (b % 64)) & 1) jac_add(c, &acc, &acc, &j->table[b]);
    jac_to_affine(c, &acc, j->out + i * 2 * L, j->out + i * 2 * L + L, NULL);
  }
  return NULL;
}

static void run_jobs(job_t *jobs, int nt, void *(*fn)(void *)) {
  pthread_t th[256];
  for (int t = 1; t < nt; t++) pthread_create(&th[t], NULL, fn, &jobs[t]);
  fn(&jobs[0]);
  for (int t = 1; t < nt; t++) pthread_join(th[t], NULL);
}

/* ---------------- exported API ----------------------------------------- */

int orc_curve_limbs(int curve) {
  const curve_t *c = get_curve(curve);
  return c ? c->L : -1;
}

int orc_fp_mul(int curve, const uint64_t *a, const uint64_t *b, uint64_t *r, size_t n) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  int L = c->L;
  for (size_t i = 0; i < n; i++) mod_mul(&c->p, r + i * L, a + i * L, b + i * L);
  return 0;
}

int orc_fp_inv(int curve, const uint64_t *a, uint64_t *r, size_t n) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  int L = c->L;
  for (size_t i = 0; i < n; i++) mod_inv(&c->p, r + i * L, a + i * L);
  return 0;
}

int orc_on_curve(int curve, const uint64_t *pts, size_t n, uint8_t *ok) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  int L = c->L;
  for (size_t i = 0; i < n; i++) ok[i] = (uint8_t)affine_on_curve(c, pts + 2 * L * i, pts + 2 * L * i + L);
  return 0;
}

/* elementwise affine additions r_i = p_i + q_i */
int orc_add(int curve, const uint64_t *p, const uint64_t *q, size_t n, uint64_t *r, uint8_t *inf) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  int L = c->L;
  for (size_t i = 0; i < n; i++) {
    jac_t P, Q, R;
    jac_from_affine(c, &P, p + 2 * L * i, p + 2 * L * i + L);
    jac_from_affine(c, &Q, q + 2 * L * i, q + 2 * L * i + L);
    jac_add(c, &R, &P, &Q);
    jac_to_affine(c, &R, r + 2 * L * i, r + 2 * L * i + L, inf ? inf + i : NULL);
  }
  return 0;
}

int orc_scalar_mul(int curve, const uint64_t *k, const uint64_t *p, size_t n, uint64_t *r, uint8_t *inf) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  int L = c->L;
  for (size_t i = 0; i < n; i++) {
    jac_t P, R;
    jac_from_affine(c, &P, p + 2 * L * i, p + 2 * L * i + L);
    jac_scalar_mul(c, &R, &P, k + 4 * i, 4);
    jac_to_affine(c, &R, r + 2 * L * i, r + 2 * L * i + L, inf ? inf + i : NULL);
  }
  return 0;
}

int orc_msm(int curve, const uint64_t *bases, const uint64_t *scalars, size_t n, int nthreads, uint64_t *out,
            uint8_t *out_inf) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((size_t)nthreads > n && n > 0) nthreads = (int)n;
  job_t *jobs = (job_t *)calloc(nthreads, sizeof(job_t));
  for (int t = 0; t < nthreads; t++) {
    jobs[t].c = c;
    jobs[t].bases = bases;
    jobs[t].scalars = scalars;
    jobs[t].lo = n * t / nthreads;
    jobs[t].hi = n * (t + 1) / nthreads;
  }
  run_jobs(jobs, nthreads, msm_worker);
  jac_t acc;
  jac_set_inf(c, &acc);
  for (int t = 0; t < nthreads; t++) jac_add(c, &acc, &acc, &jobs[t].acc);
  jac_to_affine(c, &acc, out, out + c->L, out_inf);
  free(jobs);
  return 0;
}

/* segmented MSMs: result j = sum over [offsets[j], offsets[j+1]) */
int orc_msm_batch(int curve, const uint64_t *bases, const uint64_t *scalars, const uint64_t *offsets, size_t m,
                  int nthreads, uint64_t *out, uint8_t *out_inf) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  int L = c->L;
  for (size_t j = 0; j < m; j++) {
    size_t lo = offsets[j], hi = offsets[j + 1];
    int rc = orc_msm(curve, bases + lo * 2 * L, scalars + lo * 4, hi - lo, nthreads, out + j * 2 * L, out_inf + j);
    if (rc) return rc;
  }
  return 0;
}

int orc_fixed_base(int curve, const uint64_t *ks, size_t n, int nthreads, uint64_t *out) {
  const curve_t *c = get_curve(curve);
  if (!c) return -1;
  jac_t *table = (jac_t *)malloc(sizeof(jac_t) * 256);
  jac_from_affine(c, &table[0], c->gx, c->gy);
  for (int b = 1; b < 256; b++) jac_dbl(c, &table[b], &table[b - 1]);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((size_t)nthreads > n && n > 0) nthreads = (int)n;
  job_t *jobs = (job_t *)calloc(nthreads, sizeof(job_t));
  for (int t = 0; t < nthreads; t++) {
    jobs[t].c = c;
    jobs[t].scalars = ks;
    jobs[t].lo = n * t / nthreads;
    jobs[t].hi = n * (t + 1) / nthreads;
    jobs[t].out = out;
    jobs[t].table = table;
  }
  run_jobs(jobs, nthreads, fixed_worker);
  free(jobs);
  free(table);
  return 0;
}

/* ECDSA verification; hashes are 32 bytes big-endian, keys canonical affine,
   sigs (r[4], s[4]) little-endian u64 */
int orc_ecdsa_verify(int curve, const uint8_t *hashes, const uint64_t *pubkeys, const uint64_t *sigs, size_t m,
                     uint8_t *valid) {
  const curve_t *c = get_curve(curve);
  if (!c || c->L != 4) return -1;
  const modulus_t *N = &c->n;
  uint64_t one[4] = {1, 0, 0, 0};
  for (size_t i = 0; i < m; i++) {
    const uint64_t *r = sigs + 8 * i, *s = sigs + 8 * i + 4;
    const uint64_t *qx = pubkeys + 8 * i, *qy = pubkeys + 8 * i + 4;
    valid[i] = 0;
    if (mp_is_zero(r, 4) || mp_is_zero(s, 4) || mp_cmp(r, N->m, 4) >= 0 || mp_cmp(s, N->m, 4) >= 0) continue;
    if (mp_is_zero(qx, 4) && mp_is_zero(qy, 4)) continue;
    if (!affine_on_curve(c, qx, qy)) continue;
    uint64_t e[4];
    for (int w = 0; w < 4; w++) {
      uint64_t v = 0;
      for (int byte = 0; byte < 8; byte++) v = (v << 8) | hashes[32 * i + 8 * (3 - w) + byte];
      e[w] = v;
    }
    /* e < 2^256 may exceed n: reduce (at most one subtraction since n > 2^255) */
    if (mp_cmp(e, N->m, 4) >= 0) mp_sub(e, e, N->m, 4);
    uint64_t w_[4], u1[4], u2[4];
    mod_inv(N, w_, s);
    mod_mul(N, u1, e, w_);
    mod_mul(N, u2, r, w_);
    jac_t G, Q, A, B, R;
    jac_from_affine(c, &G, c->gx, c->gy);
    jac_from_affine(c, &Q, qx, qy);
    jac_scalar_mul(c, &A, &G, u1, 4);
    jac_scalar_mul(c, &B, &Q, u2, 4);
    jac_add(c, &R, &A, &B);
    uint64_t x[4], y[4];
    uint8_t inf;
    jac_to_affine(c, &R, x, y, &inf);
    if (inf) continue;
    /* x mod n: x < p < 2n */
    if (mp_cmp(x, N->m, 4) >= 0) mp_sub(x, x, N->m, 4);
    valid[i] = (uint8_t)(mp_cmp(x, r, 4) == 0);
    (void)one;
  }
  return 0;
}
