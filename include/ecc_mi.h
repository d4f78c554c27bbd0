/*
 * eccmi: batched elliptic-curve multi-scalar multiplication and ECDSA
 * verification on AMD MI355X (gfx950).  C ABI.
 *
 * The arithmetic follows "gECC: A GPU-based high-throughput framework for
 * Elliptic Curve Cryptography" (arXiv 2501.03245): affine point addition
 * (Section 2.1, Eqns 2-3) batched with Montgomery's trick (Sections 2.2 and
 * 3.1), Gather-Apply-Scatter batch inversion (Section 3.2), x-only compress
 * and recomputation in the decompress step (Section 3.3), Montgomery
 * multiplication (Algorithm 2).  The multi-scalar multiplication drives these
 * from a Pippenger bucket method.
 *
 * Conventions shared by every call:
 *   - Pointers are DEVICE pointers (e.g. torch.Tensor.data_ptr() of a CUDA
 *     tensor) unless ECC_HOST_PTRS is set in opts->flags; the caller owns every
 *     buffer; the library keeps no pointer after the call returns.
 *   - A point is affine: x then y, each as L little-endian u64 limbs (L = 4 for
 *     BN254 and secp256r1, 6 for BLS12-381), canonical in [0, p) unless
 *     ECC_IN_MONTGOMERY says x R mod p, y R mod p with R = 2^(64 L).
 *     x = y = 0 encodes the point at infinity (not on any of the curves since
 *     b != 0).
 *   - A scalar is 4 little-endian u64 limbs, value < 2^bitlen(r) (254 bits for
 *     BN254, 255 for BLS12-381), not reduced: the result is the literal sum.
 *   - Results are canonical affine; the point at infinity is x = y = 0 with the
 *     matching out_inf byte set to 1.
 *   - Calls are synchronous: they return after the results are written,
 *     unless ECC_ASYNC is set (ecc_msm, ecc_msm_batch, ecc_verify_batch):
 *     then the call only enqueues its work on the stream and returns.  Inputs
 *     must stay valid and unmodified, and outputs are not to be read, until
 *     that stream has completed the work (stream or event synchronisation, or
 *     ecc_ctx_sync).  Input errors found on the device (ECC_ERR_RANGE,
 *     ECC_ERR_NOT_ON_CURVE) are then reported by ecc_ctx_sync instead; the
 *     outputs of a call with such an error are left untouched either way.
 *   - A non-OK status leaves the outputs untouched and ecc_last_error(ctx)
 *     describes the failure.
 *   - A context is used by one host thread at a time.
 */
#ifndef ECC_MI_H
#define ECC_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { ECC_BN254_G1 = 1, ECC_BLS12_381_G1 = 2, ECC_SECP256R1 = 3, ECC_SM2 = 4 } ecc_curve;

typedef enum {
  ECC_PENDING = 1,           /* ecc_server_wait without blocking: not finished yet */
  ECC_OK = 0,
  ECC_ERR_ARG = -1,          /* bad pointer, size, curve or option */
  ECC_ERR_RANGE = -2,        /* a coordinate >= p or a scalar >= 2^bitlen(r) */
  ECC_ERR_NOT_ON_CURVE = -3, /* with ECC_CHECK_ON_CURVE: a base is off the curve */
  ECC_ERR_NOMEM = -4,        /* device memory or the context's HBM budget exhausted */
  ECC_ERR_DEVICE = -5,       /* a HIP call failed */
  ECC_ERR_UNSUPPORTED = -6   /* curve/call combination not provided */
} ecc_status;

enum {
  ECC_IN_MONTGOMERY = 1u << 0,  /* input coordinates are already x R mod p */
  ECC_CHECK_ON_CURVE = 1u << 1, /* reject bases that are not on the curve */
  ECC_HOST_PTRS = 1u << 2,      /* all pointers of this call are host memory */
  ECC_USE_GRAPH = 1u << 3,      /* MSM calls: run the launch sequence as one captured
                                   hipGraph, kept by the context and replayed by later
                                   calls with the same sizes, flags, pointers and stream
                                   (ignored together with ECC_HOST_PTRS) */
  ECC_NO_ENDOMORPHISM = 1u << 4, /* MSM calls: no endomorphism split of the scalars.  Without
                                   it an MSM on BN254 or BLS12-381 (single or batched) may
                                   run over (P_i, [lambda] P_i) with half-length scalars,
                                   which is exact for points of the order-r subgroup only:
                                   set this flag for BLS12-381 bases that may lie outside G1
                                   (BN254 G1 has cofactor 1, so every curve point is in it) */
  ECC_VERIFY_BATCHED = 1u << 5,  /* ecc_verify_batch: the batched-affine form (one GAS
                                    inversion per scalar bit and workgroup, Section 3.4) */
  ECC_VERIFY_PER_LANE = 1u << 6, /* ecc_verify_batch: the per-lane XYZZ form (two inversions
                                    per launch); also the form used when neither flag is set */
  ECC_ASYNC = 1u << 7,           /* ecc_msm, ecc_msm_batch, ecc_verify_batch: enqueue on the
                                    stream and return without waiting (device pointers
                                    only; see the conventions above).  Asynchronous calls
                                    on one context share its device scratch, so they must
                                    run on one stream (or be ordered by the caller) */
  ECC_BASES_PER_MSM = 1u << 8,   /* ecc_msm_batch: `bases` is a HOST array of m DEVICE
                                    pointers, MSM j's bases starting at bases[j] (for
                                    example ranges of a resident set, read in place with
                                    no copy); not with ECC_HOST_PTRS */
  ECC_PMUL_BATCHED = 1u << 9     /* ecc_pmul_batch: the paper's batch UPMUL (Section 3.4,
                                    Algorithm 3): affine addition and doubling per scalar
                                    bit sharing one Montgomery-trick chain per lane, one
                                    GAS inversion per bit and workgroup, several requests
                                    per lane; the default is the per-lane XYZZ form */
};

typedef struct ecc_ctx ecc_ctx;

typedef struct {
  uint32_t flags;   /* ECC_* flags above */
  int32_t window_c; /* Pippenger window width in bits; 0 = library choice */
  void *stream;     /* hipStream_t to run on; NULL = the context's own stream, a
                       blocking stream (ordered with the legacy default stream) */
} ecc_opts;

/* Create a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * device scratch the context may hold (0 = no cap).  Returns ECC_OK and *out,
 * or an error (then *out is NULL). */
ecc_status ecc_ctx_create(int hip_device, size_t hbm_budget_bytes, ecc_ctx **out);

/* Release a context and all its device memory.  NULL is ignored. */
void ecc_ctx_destroy(ecc_ctx *ctx);

/* Message for the last non-OK status returned on this context ("" if none).
 * The string is owned by the context and valid until its next call. */
const char *ecc_last_error(const ecc_ctx *ctx);

/* Device scratch currently held by the context, in bytes. */
size_t ecc_ctx_scratch_bytes(const ecc_ctx *ctx);

/* Per-phase timing of ecc_msm calls, accumulated while profiling is on.
 * Times come from HIP events recorded on the stream the kernels run on. */
typedef struct {
  uint64_t msm_calls;      /* ecc_msm calls measured */
  uint64_t points;         /* sum of n over those calls */
  uint64_t round_launches; /* bucket-accumulation round kernels launched */
  uint64_t round_adds;     /* batch-affine additions done by those kernels */
  double prepare_ms;       /* ingest, windowing, bucket grouping, schedule */
  double round_ms;         /* bucket-accumulation rounds (sum of kernel times) */
  double reduce_ms;        /* bucket reduction */
  double combine_ms;       /* window combination and output */
  double total_ms;         /* whole calls, first kernel to last */
  double finish_ms;        /* per-lane finishing pass after the rounds (sum) */
} ecc_stats;

/* Turn per-phase timing on (1) or off (0); turning it on clears the stats. */
ecc_status ecc_ctx_set_profiling(ecc_ctx *ctx, int enable);

/* Design variant of the bucket-round kernel for later MSM calls on this
 * context, for ablations of the choices of Sections 3.2-3.4; every
 * variant gives the same results.  0 = the library's form (the default).
 * Bits 1-8 and 64 select a round kernel (BLS12-381 only): 1 stores each denominator
 * in the compress step instead of recomputing it (Section 3.3 recomputes); 2
 * stores the prefix products per lane, contiguous, instead of limb-major
 * planes that coalesce across a wave; 4 splits the decompress step from the
 * additions (a second kernel reloads the points: no DCWPA fusion); 8 inverts
 * every lane's chain product on its own lane instead of one GAS inversion
 * per workgroup (Section 3.2); 64 stores the prefix products of even steps
 * only and recomputes the odd ones (find-then-recompute, Section 3.4).  Bits
 * 16 and 32 choose where the rounds stop.
 * By default a single MSM stops them once they hold fewer additions than
 * twice the grid's lanes and no bucket has more than 16 partial sums, and
 * adds each bucket's remaining partial sums on its own lane in XYZZ
 * coordinates, while a batch runs the rounds to the end; 16 takes the
 * finishing pass for batches too, 32 runs the rounds to the end for every
 * call (the paper's form).  Built round kernels: 1, 2, 3, 4, 7, 8, 64, each
 * combinable with 16 or 32 (not both).  BN254 MSM calls on a context whose
 * variant has any of bits 1-8 or 64 return ECC_ERR_UNSUPPORTED.  Errors:
 * ECC_ERR_ARG (another value). */
ecc_status ecc_ctx_set_round_variant(ecc_ctx *ctx, int variant);

/* Copy the accumulated stats into *out. */
ecc_status ecc_ctx_get_stats(const ecc_ctx *ctx, ecc_stats *out);

/* Wait for every ECC_ASYNC call made on this context to finish, then report
 * the input errors those calls found on the device since the last
 * ecc_ctx_sync (ECC_ERR_RANGE or ECC_ERR_NOT_ON_CURVE, the first by this
 * order; ECC_OK if none) and clear them.  ECC_ERR_DEVICE if a HIP call
 * fails. */
ecc_status ecc_ctx_sync(ecc_ctx *ctx);

/* Multi-scalar multiplication R = sum_{i < n} scalars_i * bases_i
 * (the plain definition; computed by Pippenger buckets with batch-affine
 * additions).
 *   bases   : n points (2 L u64 each)        scalars : n x 4 u64
 *   out_xy  : 2 L u64                        out_inf : 1 byte
 * n = 0 gives the point at infinity.  Bases equal to (0, 0) contribute
 * nothing.  Subgroup membership of the bases is not checked: the result is
 * exact for points of the order-r subgroup (all of BN254, G1 of BLS12-381);
 * BLS12-381 bases outside G1 need ECC_NO_ENDOMORPHISM.
 * Errors: ECC_ERR_ARG (NULL pointer with n > 0, unknown curve, window_c
 * outside [2, 20]), ECC_ERR_RANGE, ECC_ERR_NOT_ON_CURVE, ECC_ERR_NOMEM,
 * ECC_ERR_DEVICE; ECC_ERR_UNSUPPORTED for ECC_SECP256R1. */
ecc_status ecc_msm(ecc_ctx *ctx, ecc_curve curve, const uint64_t *bases, const uint64_t *scalars, size_t n,
                   uint64_t *out_xy, uint8_t *out_inf, const ecc_opts *opts);

/* A batch of m independent MSMs in one launch sequence:
 *   R_j = sum over offsets[j] <= i < offsets[j+1] of scalars_i * bases_i.
 * The Pippenger buckets of all MSMs are accumulated together, so every round
 * of batch-affine additions (one Montgomery-trick chain per lane, one
 * Gather-Apply-Scatter inversion per workgroup, Sections 3.1-3.2) spans the
 * whole batch; reduction and window combination run per MSM.
 *   bases, scalars : offsets[m] points and scalars, concatenated, laid out as
 *                    for ecc_msm (device pointers unless ECC_HOST_PTRS)
 *   offsets        : m + 1 u64 in HOST memory, offsets[0] = 0, non-decreasing
 *                    (the launch geometry is planned on the host)
 *   out_xy         : m points (2 L u64 each)   out_inf : m bytes
 * Each MSM gets its own window width (opts->window_c, if nonzero, for all).
 * An empty MSM gives the point at infinity.  With ECC_USE_GRAPH the whole
 * sequence is captured once and replayed on identical later calls.
 * Errors: as ecc_msm, and ECC_ERR_ARG for bad offsets or more than 2^30
 * points in total; a non-OK status leaves every output untouched. */
ecc_status ecc_msm_batch(ecc_ctx *ctx, ecc_curve curve, const uint64_t *bases, const uint64_t *scalars,
                         const uint64_t *offsets, size_t m, uint64_t *out_xy, uint8_t *out_inf,
                         const ecc_opts *opts);

/* Device scratch, in bytes, that ecc_msm_batch with these offsets and options
 * would hold (the same launch geometry, added up instead of allocated; for
 * admission under an HBM budget).  offsets as for ecc_msm_batch (host
 * memory); with m = 1 it is the figure of ecc_msm on offsets[1] points.
 * Errors: ECC_ERR_ARG, ECC_ERR_UNSUPPORTED (a curve without MSM). */
ecc_status ecc_msm_batch_scratch_bytes(ecc_ctx *ctx, ecc_curve curve, const uint64_t *offsets, size_t m,
                                       const ecc_opts *opts, size_t *bytes);

/* Batched ECDSA signature verification on secp256r1 or SM2 (ECC_SECP256R1,
 * ECC_SM2: the curve of the paper's evaluation, Section 5).
 * Request i: valid_i = 1 iff 1 <= r_i, s_i <= n - 1, Q_i is a point of the
 * curve other than O, and with e = the hash read as a big-endian integer,
 * w = s^-1, u1 = e w, u2 = r w (mod n), the point R = u1 G + u2 Q is not O
 * and R.x mod n = r.  Verification is one fixed-point and one unknown-point
 * multiplication (Section 5.2), in one of two forms:
 *  - batched affine (ECC_VERIFY_BATCHED): both multiplications run as affine
 *    operations with one Montgomery-trick chain per request and one
 *    Gather-Apply-Scatter inversion per workgroup and scalar bit (Sections
 *    3.2-3.4, Algorithm 3); a launch takes 257 inversion latencies however
 *    few requests it holds;
 *  - per lane (ECC_VERIFY_PER_LANE): each request's double-scalar sum in XYZZ
 *    coordinates on its own lane (4-bit windows of u2 over a per-request table
 *    of d Q, a comb table of d 2^(8 j) G for u1), with two batched inversions
 *    per launch.  This is the default: it measured faster at every batch
 *    size, in latency and in throughput.
 * The inverses of s mod n are batched per workgroup in both.
 *   hashes  : m x 32 bytes (big-endian digests)
 *   pubkeys : m points Q (x[4], y[4] u64, canonical affine)
 *   sigs    : m x (r[4], s[4]) u64 little-endian
 *   valid   : m bytes, 1 valid / 0 invalid
 * A malformed request (r or s out of range, Q off the curve or O) yields
 * valid = 0, not an error; so does every request of a call on a curve that
 * carries no ECDSA keys here (ECC_BN254_G1, ECC_BLS12_381_G1).  Errors:
 * ECC_ERR_ARG (NULL pointer with m > 0, an unknown curve id, flags other than
 * ECC_HOST_PTRS, ECC_VERIFY_BATCHED and ECC_VERIFY_PER_LANE, or both of the
 * last two), ECC_ERR_DEVICE, ECC_ERR_NOMEM. */
ecc_status ecc_verify_batch(ecc_ctx *ctx, ecc_curve curve, const uint8_t *hashes, const uint64_t *pubkeys,
                            const uint64_t *sigs, size_t m, uint8_t *valid, const ecc_opts *opts);

/* ecc_verify_batch without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Computes exactly what ecc_verify_batch computes in
 * its per-lane form, on the HIP stream `stream` (NULL = the null stream), and
 * returns after the verdicts are written.  No context: hashes, pubkeys, sigs
 * and valid are DEVICE pointers with the layouts of ecc_verify_batch, owned
 * by the caller.  The device memory the work needs (the generator's comb
 * tables and one table of d Q per request) is a fixed array inside the
 * library, about 28 MB on every GPU the call runs on, held until the process
 * ends; the first call on a device builds the comb tables there.  Every call
 * on one GPU uses that same array: calls that overlap on one GPU (from
 * several threads or streams) race, so the caller orders them.  At most
 * ecc_verify_batch_noalloc_max() requests (8192) per call.  Errors:
 * ECC_ERR_ARG (NULL pointer with m > 0, m above the maximum, an unknown
 * curve id), ECC_ERR_DEVICE (a HIP call failed); BN254 and BLS12-381 give
 * valid = 0 for every request, as in ecc_verify_batch. */
ecc_status ecc_verify_batch_noalloc(ecc_curve curve, const uint8_t *hashes, const uint64_t *pubkeys,
                                    const uint64_t *sigs, size_t m, uint8_t *valid, void *stream);
/* The largest m that ecc_verify_batch_noalloc accepts. */
size_t ecc_verify_batch_noalloc_max(void);

/* Batched ECDSA signature generation on secp256r1 or SM2: one fixed-point
 * multiplication and one inversion mod n per request (Section 5.2).
 * Request i: with 1 <= d_i, k_i <= n - 1, R = k_i G, r = R.x mod n,
 * e = the hash read as a big-endian integer, s = k_i^-1 (e + r d_i) mod n.
 * k_i G is summed from a comb table of d 2^(8 j) G (made once per context)
 * in XYZZ coordinates, one request per lane; R.x's denominator and k_i are
 * inverted by one Gather-Apply-Scatter batch inversion each per workgroup.
 *   hashes   : m x 32 bytes (big-endian digests)
 *   privkeys : m x 4 u64 little-endian private keys d_i
 *   nonces   : m x 4 u64 little-endian nonces k_i (secret, never reused)
 *   sigs     : m x (r[4], s[4]) u64 little-endian, written
 * A request whose d_i or k_i is out of range, or whose r or s is zero,
 * gets r = s = 0 (draw another nonce), not an error.  Errors: ECC_ERR_ARG
 * (NULL pointer with m > 0, flags other than ECC_HOST_PTRS, m > 2^30),
 * ECC_ERR_UNSUPPORTED (another curve), ECC_ERR_DEVICE, ECC_ERR_NOMEM. */
ecc_status ecc_sign_batch(ecc_ctx *ctx, ecc_curve curve, const uint8_t *hashes, const uint64_t *privkeys,
                          const uint64_t *nonces, size_t m, uint64_t *sigs, const ecc_opts *opts);

/* Batched unknown-point multiplication: out_i = k_i P_i (Section 2.1's scalar
 * multiplication of a point known only at run time, the paper's UPMUL of
 * Section 3.4 and Table 5), on any of the four curves.  Two forms:
 *  - per lane (default): one request per lane, a table of d P_i (d = 1..15)
 *    normalised with one Montgomery-trick chain and one Gather-Apply-Scatter
 *    inversion per workgroup, 4-bit windows of k_i in XYZZ coordinates, and
 *    one more batched inversion for the affine result;
 *  - batched affine (ECC_PMUL_BATCHED): Algorithm 3, 256 steps over the bits
 *    of k_i from the least significant end, each an affine addition and an
 *    affine doubling per request whose denominators share one chain per lane
 *    (several requests per lane; only the product before both is stored and
 *    the other recomputed), inverted once per step and workgroup; the state
 *    of every request stays in device memory between steps.
 *   points  : n points, as for ecc_msm (canonical affine, (0, 0) = O; with
 *             ECC_IN_MONTGOMERY in Montgomery form)
 *   scalars : n x 4 u64, any 256-bit integers (not reduced)
 *   out_xy  : n points, canonical affine (Montgomery form with
 *             ECC_IN_MONTGOMERY), O written as (0, 0)
 * Every point is range- and curve-checked first.  Errors: ECC_ERR_RANGE (a
 * coordinate >= p), ECC_ERR_NOT_ON_CURVE, ECC_ERR_ARG (NULL pointer with
 * n > 0, flags other than ECC_IN_MONTGOMERY, ECC_HOST_PTRS and
 * ECC_PMUL_BATCHED, n > 2^30), ECC_ERR_DEVICE, ECC_ERR_NOMEM; a non-OK status
 * leaves out_xy untouched. */
ecc_status ecc_pmul_batch(ecc_ctx *ctx, ecc_curve curve, const uint64_t *points, const uint64_t *scalars, size_t n,
                          uint64_t *out_xy, const ecc_opts *opts);

/* k_i G for the curve's standard generator G (fixed-point multiplication,
 * the paper's FPMUL with precomputed multiples of G, Section 2.1): one mixed
 * addition per byte of k_i, of d 2^(8 j) G from a comb table that the
 * context makes once per curve with the double-and-add of Algorithm 1, then
 * one batched inversion for the affine results.  ks: n x 4 u64 scalars (any
 * 256-bit value); out: n points, canonical affine ((0,0) when k_i G is the
 * point at infinity).  Also used to produce seeded bases P_i = k_i G. */
ecc_status ecc_fixed_base_mul(ecc_ctx *ctx, ecc_curve curve, const uint64_t *ks, size_t n, uint64_t *out_xy,
                              const ecc_opts *opts);

/* ---- window tuning ----------------------------------------------------------
 * The window width c of a Pippenger MSM trades W = ceil((bits + 1) / c)
 * passes over the points against 2^(c-1) buckets per window to reduce; the
 * best value depends on n, the curve and the device.  Without tuning the
 * library takes c from a cost model.  ecc_tune measures, for every n = 2^k
 * with log2n_min <= k <= log2n_max, MSMs over seeded synthetic inputs made on
 * the device (bases k_i G, scalars of the curve's bit length) at the model's
 * c and its neighbours, then the target number of additions per lane in a
 * bucket round and the round kernel's occupancy target at the best c, taking
 * the median of `reps` timed calls; the
 * winners are used by later MSM calls of this context whose size falls in
 * the same power-of-two class (a nonzero opts->window_c still wins).
 * Errors: ECC_ERR_ARG (range outside [1, 26], reps outside [1, 101]),
 * ECC_ERR_UNSUPPORTED (secp256r1), and those of ecc_msm. */
ecc_status ecc_tune(ecc_ctx *ctx, ecc_curve curve, int log2n_min, int log2n_max, int reps);

/* The window width and additions-per-lane target an MSM of n points would
 * use on this context now. */
ecc_status ecc_tuned_params(ecc_ctx *ctx, ecc_curve curve, size_t n, int *window_c, int *adds_per_lane);

/* Write the context's tuned entries to a text file (one line per entry:
 * device key, curve, log2 n, window, additions per lane), or read such a
 * file and adopt the entries whose device key (architecture and CU count)
 * matches this context's device; *loaded (may be NULL) receives their count. */
ecc_status ecc_tune_save(ecc_ctx *ctx, const char *path);
ecc_status ecc_tune_load(ecc_ctx *ctx, const char *path, int *loaded);

/* ---- elementwise entry points for parity tests of the building blocks ---- */

/* out_i = a_i b_i mod p (canonical in and out, L u64 each); goes through the
 * Montgomery form and back (Algorithm 2).  When a and b are the same pointer
 * the dedicated squaring routine computes a_i^2. */
ecc_status ecc_test_fp_mul(ecc_ctx *ctx, ecc_curve curve, const uint64_t *a, const uint64_t *b, uint64_t *out,
                           size_t n);

/* The lane-parallel field arithmetic of the window combination (one element
 * per 16-lane row, four per wave): op 0: out_i = a_i b_i, op 1: a_i - b_i,
 * op 2: 3 a_i (a_i + b_i) - 2 b_i, op 3: 3 a_i b_i - a_i^2,
 * op 4: 3 b_i^2 + a_i b_i - a_i^2, op 5: a_i^2 - a_i b_i - 2 b_i^2,
 * op 6: (2 (a_i b_i - a_i^2))^2, op 7: a_i b_i - a_i^2, all mod p (canonical
 * in and out, L u64 each; the products are Algorithm 2 with the limb columns
 * spread over lanes; ops 3-5 take the differences of the point formulas on
 * unreduced product outputs, ops 6-7 a Y coordinate that the point formulas
 * may leave unreduced).  ECC_ERR_ARG for an op outside [0, 7]. */
ecc_status ecc_test_lane_field(ecc_ctx *ctx, ecc_curve curve, int op, const uint64_t *a, const uint64_t *b,
                               uint64_t *out, size_t n);

/* out_i = a_i^-1 mod p (0 maps to 0), computed by one workgroup-level
 * Gather-Apply-Scatter batch inversion per 256 inputs (Section 3.2). */
ecc_status ecc_test_fp_inv(ecc_ctx *ctx, ecc_curve curve, const uint64_t *a, uint64_t *out, size_t n);

/* out_i = p_i + q_i (affine, every case of the group law), computed by the
 * batch-affine addition kernel of the bucket accumulation. */
ecc_status ecc_test_batch_add(ecc_ctx *ctx, ecc_curve curve, const uint64_t *p, const uint64_t *q, uint64_t *out,
                              size_t n);

/* Bucket grouping of the Pippenger windows with signed digits:
 * counts[b] entries for bucket b = w 2^(c-1) + |d| - 1, offsets (B + 1
 * entries, exclusive prefix sums) and sorted (entry = index | sign << 31,
 * order inside a bucket unspecified).  B = W 2^(c-1), W = ceil((bits + 1)/c).
 * method: 0 = as ecc_msm would, 1 = device-wide atomic counting sort,
 * 2 = two-level counting sort: coarse bins per chunk of points, then fine
 * buckets per coarse bin in LDS (window_c <= 16, 0 < n <= 2^27).
 * Capacities: counts and offsets hold B + 1 u32, sorted holds n W u32. */
ecc_status ecc_test_bucket_sort(ecc_ctx *ctx, ecc_curve curve, const uint64_t *scalars, size_t n, int window_c,
                                int method, uint32_t *counts, uint32_t *offsets, uint32_t *sorted);

/* ---- measurement ----------------------------------------------------------------
 * Issue-rate probe (not a step of the path): every lane of
 * 256 x waves_per_simd workgroups of 256 lanes runs `chains` interleaved
 * dependency chains of 16 x iters instructions of one class: op 0 the
 * 32x32+64 -> 64 integer multiply-add of the field product (v_mad_u64_u32),
 * op 1 the fp64 fused multiply-add (v_fma_f64), op 2 the 32-bit low product
 * (v_mul_lo_u32).  One chain exposes the latency, several the issue rate
 * (Table 2 of the paper measures its GPU's integer instructions this way).
 * Outputs: *ms the device time of one launch (HIP events, after a warm-up
 * launch), *lane_ops the lane-operations it issued, *shader_mhz the shader
 * clock over the timed loop (cycle counter against the constant-rate wall
 * counter).  ECC_ERR_ARG for op outside [0, 2], chains not in {1, 2, 4, 8},
 * waves_per_simd outside [1, 8], iters outside [1, 2^20] or a null pointer. */
ecc_status ecc_probe_issue_rate(ecc_ctx *ctx, int op, int chains, int waves_per_simd, uint32_t iters, double *ms,
                                double *lane_ops, double *shader_mhz);

/* ---- request server (continuous batching on one GPU) -------------------------
 * Requests are queued as they arrive; `slots` worker threads, each with its
 * own context and stream, repeatedly take the kind of work whose oldest
 * request waits longest and admit as many queued requests of that kind as fit
 * max_batch_points (MSM) or max_batch_verify and, for MSMs, whose batched
 * call's device scratch (as ecc_msm_batch_scratch_bytes plans it) fits the
 * slot's share of hbm_budget_bytes; the admitted requests run as one batched
 * call (ecc_msm_batch over the MSMs of one curve, ecc_verify_batch over the
 * verifications).  A batch that still runs out of device memory is split in
 * halves and retried.  Requests that arrive while batches run join the next
 * batch of the next free slot, so batches of different slots overlap on the
 * GPU.  Each result is the same as the request's result alone.  Request data
 * is copied at submission (host memory); bases are registered once, stay in
 * device memory and are read there in place (ECC_BASES_PER_MSM).  Latency is
 * measured from submission to the end of the request's batch. */
typedef struct ecc_server ecc_server;

typedef struct {
  int slots;                 /* concurrent batches, 1..16 */
  size_t hbm_budget_bytes;   /* device scratch for all slots together (0 = no cap) */
  size_t max_batch_points;   /* MSM points admitted into one batch (and the largest MSM accepted) */
  size_t max_batch_verify;   /* verifications admitted into one batch */
  int use_graph;             /* run MSM batches as captured graphs (reused when shapes repeat) */
} ecc_server_cfg;

typedef struct {
  uint64_t done_msm, done_verify; /* requests finished */
  uint64_t batches;               /* batched calls made */
  uint64_t msm_points;            /* points over the finished MSM requests */
  double p50_msm_ms, p99_msm_ms;  /* latency percentiles of finished requests */
  double p50_verify_ms, p99_verify_ms;
  double span_ms;                 /* first submission to last completion */
  uint64_t budget_cuts;           /* MSM batches admission cut short to fit the HBM share */
  uint64_t nomem_splits;          /* batched calls that ran out of device memory and were halved */
  uint64_t max_queue;             /* longest queue seen at a submission */
} ecc_server_stats;

ecc_status ecc_server_create(int hip_device, const ecc_server_cfg *cfg, ecc_server **out);

/* Test-only executor, so that the server's admission and batching can be
 * tested without a GPU: msm_batch_bytes replaces the library's scratch plan
 * of an MSM batch (its m request sizes), and run_batch replaces the batched
 * call (kind 1: MSMs of sizes[j] points; kind 0: verifications), writing one
 * flag per request (MSM: 1 for a result at infinity; verification: valid)
 * and returning the batch's status.  Both are called from the worker
 * threads.  A server made this way holds no device memory: registered bases
 * are only counted, and MSM results are all-zero coordinates. */
typedef struct {
  void *user;
  size_t (*msm_batch_bytes)(void *user, const uint64_t *sizes, size_t m);
  ecc_status (*run_batch)(void *user, int kind, const uint64_t *sizes, size_t m, uint8_t *flags);
} ecc_server_exec;
ecc_status ecc_server_create_with_exec(const ecc_server_cfg *cfg, const ecc_server_exec *exec, ecc_server **out);
/* Finishes the queued requests, then stops the workers and frees everything. */
void ecc_server_destroy(ecc_server *s);
const char *ecc_server_last_error(const ecc_server *s);
/* Upload n bases (host memory, canonical affine as for ecc_msm) of an MSM
 * curve; *bases_id names them in later MSM requests. */
ecc_status ecc_server_add_bases(ecc_server *s, ecc_curve curve, const uint64_t *bases, size_t n, uint32_t *bases_id);
/* MSM over bases [first, first + n) of a registered set with n scalars (host
 * memory, 4 u64 each, copied now); *ticket identifies the request. */
ecc_status ecc_server_submit_msm(ecc_server *s, uint32_t bases_id, size_t first, size_t n, const uint64_t *scalars,
                                 uint64_t *ticket);
/* One secp256r1 verification (32-byte hash, Q as 8 u64, (r, s) as 8 u64). */
ecc_status ecc_server_submit_verify(ecc_server *s, const uint8_t *hash, const uint64_t *pubkey, const uint64_t *sig,
                                    uint64_t *ticket);
/* m secp256r1 verifications at once (hashes m x 32 bytes, pubkeys and sigs
 * m x 8 u64, host memory), queued in order under one lock: for load
 * generators that offer requests faster than one call each allows.
 * tickets[j] names request j. */
ecc_status ecc_server_submit_verify_many(ecc_server *s, const uint8_t *hashes, const uint64_t *pubkeys,
                                         const uint64_t *sigs, size_t m, uint64_t *tickets);
/* Blocks until the m tickets are finished, then takes their results (once):
 * flags[j] (valid, or infinity for an MSM), latency_ms[j] and status[j] (the
 * request's batch status); MSM coordinates are not returned here.  Any of
 * the three output arrays may be NULL.  ECC_ERR_ARG if a ticket is unknown
 * or already taken (the others are still taken). */
ecc_status ecc_server_wait_many(ecc_server *s, const uint64_t *tickets, size_t m, uint8_t *flags,
                                double *latency_ms, int32_t *status);
/* Result of a ticket (once): MSM -> out_xy (2 L u64) and out_flag = infinity;
 * verification -> out_flag = valid.  block = 0 returns ECC_PENDING while the
 * request is not finished.  A failed batch returns its error status.  A ticket
 * is waited for by one thread; a ticket already taken (or unknown) gives
 * ECC_ERR_ARG. */
ecc_status ecc_server_wait(ecc_server *s, uint64_t ticket, int block, uint64_t *out_xy, uint8_t *out_flag,
                           double *latency_ms);
ecc_status ecc_server_get_stats(ecc_server *s, ecc_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* ECC_MI_H */
