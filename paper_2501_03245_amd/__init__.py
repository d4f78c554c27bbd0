"""Python binding of the eccmi C ABI (include/ecc_mi.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libecc_mi.so.  Buffers are torch tensors on the GPU (device
pointers; the dtype is irrelevant, sizes are checked in bytes) or numpy arrays
(host pointers, passed with ECC_HOST_PTRS).  The first call raises when the
library has not been built; there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libecc_mi.so")

ECC_BN254_G1 = 1
ECC_BLS12_381_G1 = 2
ECC_SECP256R1 = 3
ECC_SM2 = 4
CURVES = {"bn254": ECC_BN254_G1, "bls12_381": ECC_BLS12_381_G1, "secp256r1": ECC_SECP256R1, "sm2": ECC_SM2}
LIMBS = {ECC_BN254_G1: 4, ECC_BLS12_381_G1: 6, ECC_SECP256R1: 4, ECC_SM2: 4}
SCALAR_BITS = {ECC_BN254_G1: 254, ECC_BLS12_381_G1: 255, ECC_SECP256R1: 256, ECC_SM2: 256}

ECC_OK = 0
STATUS = {1: "ECC_PENDING", 0: "ECC_OK", -1: "ECC_ERR_ARG", -2: "ECC_ERR_RANGE", -3: "ECC_ERR_NOT_ON_CURVE", -4: "ECC_ERR_NOMEM",
          -5: "ECC_ERR_DEVICE", -6: "ECC_ERR_UNSUPPORTED"}

ECC_IN_MONTGOMERY = 1 << 0
ECC_CHECK_ON_CURVE = 1 << 1
ECC_HOST_PTRS = 1 << 2
ECC_USE_GRAPH = 1 << 3
ECC_NO_ENDOMORPHISM = 1 << 4
ECC_VERIFY_BATCHED = 1 << 5
ECC_VERIFY_PER_LANE = 1 << 6
ECC_ASYNC = 1 << 7
ECC_BASES_PER_MSM = 1 << 8
ECC_PMUL_BATCHED = 1 << 9
ECC_PENDING = 1

# design variants of the bucket-round kernel (ecc_ctx_set_round_variant)
RV_STORE_DENOM = 1
RV_AOS_CHAIN = 2
RV_SPLIT_APPLY = 4
RV_LANE_INV = 8
RV_HALF_PREFIX = 64
RV_FINISH = 16
RV_ROUNDS_ONLY = 32

EXPORTED = ["ecc_ctx_create", "ecc_ctx_destroy", "ecc_last_error", "ecc_ctx_scratch_bytes",
            "ecc_ctx_set_profiling", "ecc_ctx_get_stats", "ecc_ctx_sync", "ecc_msm", "ecc_msm_batch", "ecc_msm_batch_scratch_bytes",
            "ecc_verify_batch",
            "ecc_sign_batch", "ecc_pmul_batch",
            "ecc_tune", "ecc_tuned_params", "ecc_tune_save", "ecc_tune_load",
            "ecc_server_create", "ecc_server_destroy", "ecc_server_last_error", "ecc_server_add_bases",
            "ecc_server_submit_msm", "ecc_server_submit_verify", "ecc_server_wait", "ecc_server_get_stats",
            "ecc_fixed_base_mul", "ecc_test_fp_mul", "ecc_test_lane_field", "ecc_test_fp_inv", "ecc_test_batch_add",
            "ecc_test_bucket_sort", "ecc_probe_issue_rate", "ecc_verify_batch_noalloc",
            "ecc_verify_batch_noalloc_max", "ecc_ctx_set_round_variant",
            "ecc_server_create_with_exec", "ecc_server_submit_verify_many", "ecc_server_wait_many"]


class EccError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class ecc_opts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("window_c", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class ecc_server_cfg(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_batch_points", ctypes.c_size_t), ("max_batch_verify", ctypes.c_size_t),
                ("use_graph", ctypes.c_int)]


class ecc_server_stats(ctypes.Structure):
    _fields_ = [("done_msm", ctypes.c_uint64), ("done_verify", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("msm_points", ctypes.c_uint64), ("p50_msm_ms", ctypes.c_double), ("p99_msm_ms", ctypes.c_double),
                ("p50_verify_ms", ctypes.c_double), ("p99_verify_ms", ctypes.c_double), ("span_ms", ctypes.c_double),
                ("budget_cuts", ctypes.c_uint64), ("nomem_splits", ctypes.c_uint64), ("max_queue", ctypes.c_uint64)]


# test-only executor of the request server (ecc_server_create_with_exec)
_MSM_BYTES_FN = ctypes.CFUNCTYPE(ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t)
_RUN_BATCH_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64),
                                 ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint8))


class ecc_server_exec(ctypes.Structure):
    _fields_ = [("user", ctypes.c_void_p), ("msm_batch_bytes", _MSM_BYTES_FN), ("run_batch", _RUN_BATCH_FN)]


class ecc_stats(ctypes.Structure):
    _fields_ = [("msm_calls", ctypes.c_uint64), ("points", ctypes.c_uint64), ("round_launches", ctypes.c_uint64),
                ("round_adds", ctypes.c_uint64), ("prepare_ms", ctypes.c_double), ("round_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("combine_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("finish_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2501_03245_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, ci = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    P = ctypes.POINTER
    lib.ecc_ctx_create.argtypes = [ci, sz, P(vp)]
    lib.ecc_ctx_create.restype = ci
    lib.ecc_ctx_destroy.argtypes = [vp]
    lib.ecc_ctx_destroy.restype = None
    lib.ecc_last_error.argtypes = [vp]
    lib.ecc_last_error.restype = ctypes.c_char_p
    lib.ecc_ctx_scratch_bytes.argtypes = [vp]
    lib.ecc_ctx_scratch_bytes.restype = sz
    lib.ecc_ctx_set_profiling.argtypes = [vp, ci]
    lib.ecc_ctx_set_profiling.restype = ci
    lib.ecc_ctx_get_stats.argtypes = [vp, P(ecc_stats)]
    lib.ecc_ctx_get_stats.restype = ci
    lib.ecc_ctx_sync.argtypes = [vp]
    lib.ecc_ctx_sync.restype = ci
    lib.ecc_msm.argtypes = [vp, ci, vp, vp, sz, vp, vp, P(ecc_opts)]
    lib.ecc_msm_batch.argtypes = [vp, ci, vp, vp, vp, sz, vp, vp, P(ecc_opts)]
    lib.ecc_msm_batch_scratch_bytes.argtypes = [vp, ci, vp, sz, P(ecc_opts), P(sz)]
    lib.ecc_msm_batch_scratch_bytes.restype = ci
    lib.ecc_verify_batch.argtypes = [vp, ci, vp, vp, vp, sz, vp, P(ecc_opts)]
    lib.ecc_sign_batch.argtypes = [vp, ci, vp, vp, vp, sz, vp, P(ecc_opts)]
    lib.ecc_pmul_batch.argtypes = [vp, ci, vp, vp, sz, vp, P(ecc_opts)]
    lib.ecc_server_create.argtypes = [ci, P(ecc_server_cfg), P(vp)]
    lib.ecc_server_destroy.argtypes = [vp]
    lib.ecc_server_destroy.restype = None
    lib.ecc_server_last_error.argtypes = [vp]
    lib.ecc_server_last_error.restype = ctypes.c_char_p
    lib.ecc_server_add_bases.argtypes = [vp, ci, vp, sz, P(ctypes.c_uint32)]
    lib.ecc_server_submit_msm.argtypes = [vp, ctypes.c_uint32, sz, sz, vp, P(ctypes.c_uint64)]
    lib.ecc_server_submit_verify.argtypes = [vp, vp, vp, vp, P(ctypes.c_uint64)]
    lib.ecc_server_wait.argtypes = [vp, ctypes.c_uint64, ci, vp, vp, P(ctypes.c_double)]
    lib.ecc_server_get_stats.argtypes = [vp, P(ecc_server_stats)]
    for f in ("ecc_server_create", "ecc_server_add_bases", "ecc_server_submit_msm", "ecc_server_submit_verify",
              "ecc_server_wait", "ecc_server_get_stats"):
        getattr(lib, f).restype = ci
    lib.ecc_tune.argtypes = [vp, ci, ci, ci, ci]
    lib.ecc_tuned_params.argtypes = [vp, ci, sz, P(ci), P(ci)]
    lib.ecc_tune_save.argtypes = [vp, ctypes.c_char_p]
    lib.ecc_tune_load.argtypes = [vp, ctypes.c_char_p, P(ci)]
    lib.ecc_fixed_base_mul.argtypes = [vp, ci, vp, sz, vp, P(ecc_opts)]
    lib.ecc_test_fp_mul.argtypes = [vp, ci, vp, vp, vp, sz]
    lib.ecc_test_lane_field.argtypes = [vp, ci, ci, vp, vp, vp, sz]
    lib.ecc_test_fp_inv.argtypes = [vp, ci, vp, vp, sz]
    lib.ecc_test_batch_add.argtypes = [vp, ci, vp, vp, vp, sz]
    lib.ecc_test_bucket_sort.argtypes = [vp, ci, vp, sz, ci, ci, vp, vp, vp]
    lib.ecc_probe_issue_rate.argtypes = [vp, ci, ci, ci, ctypes.c_uint32, P(ctypes.c_double), P(ctypes.c_double),
                                         P(ctypes.c_double)]
    lib.ecc_server_create_with_exec.argtypes = [P(ecc_server_cfg), P(ecc_server_exec), P(vp)]
    lib.ecc_server_create_with_exec.restype = ci
    lib.ecc_server_submit_verify_many.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.ecc_server_submit_verify_many.restype = ci
    lib.ecc_server_wait_many.argtypes = [vp, vp, sz, vp, vp, vp]
    lib.ecc_server_wait_many.restype = ci
    lib.ecc_ctx_set_round_variant.argtypes = [vp, ci]
    lib.ecc_ctx_set_round_variant.restype = ci
    lib.ecc_verify_batch_noalloc.argtypes = [ci, vp, vp, vp, sz, vp, vp]
    lib.ecc_verify_batch_noalloc.restype = ci
    lib.ecc_verify_batch_noalloc_max.argtypes = []
    lib.ecc_verify_batch_noalloc_max.restype = sz
    for f in ("ecc_msm", "ecc_msm_batch", "ecc_verify_batch", "ecc_sign_batch", "ecc_pmul_batch",
            "ecc_tune", "ecc_tuned_params", "ecc_tune_save", "ecc_tune_load",
            "ecc_server_create", "ecc_server_destroy", "ecc_server_last_error", "ecc_server_add_bases",
            "ecc_server_submit_msm", "ecc_server_submit_verify", "ecc_server_wait", "ecc_server_get_stats", "ecc_fixed_base_mul", "ecc_test_fp_mul", "ecc_test_lane_field", "ecc_test_fp_inv", "ecc_test_batch_add",
              "ecc_test_bucket_sort", "ecc_probe_issue_rate"):
        getattr(lib, f).restype = ci
    return lib


class _LazyLib:
    """Loads libecc_mi.so on first use and raises if it is missing."""

    _handle = None

    def __getattr__(self, name):
        if _LazyLib._handle is None:
            _LazyLib._handle = _load()
        return getattr(_LazyLib._handle, name)


_lib = _LazyLib()


def library():
    """The loaded ctypes library (raises ImportError when it was not built)."""
    if _LazyLib._handle is None:
        _LazyLib._handle = _load()
    return _LazyLib._handle


def _ptr(buf, nbytes: int | None = None):
    """(address, is_host) of a torch tensor or numpy array, checking its size."""
    if buf is None:
        return None, None
    if isinstance(buf, np.ndarray):
        if not buf.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        if nbytes is not None and buf.nbytes < nbytes:
            raise ValueError(f"array holds {buf.nbytes} bytes, needs {nbytes}")
        return buf.ctypes.data, True
    # torch tensor
    if not buf.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if nbytes is not None and buf.numel() * buf.element_size() < nbytes:
        raise ValueError(f"tensor holds {buf.numel() * buf.element_size()} bytes, needs {nbytes}")
    return buf.data_ptr(), not buf.is_cuda


class Context:
    """An ecc_ctx on one HIP device (device scratch, stream, last error)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        st = _lib.ecc_ctx_create(device, hbm_budget_bytes, ctypes.byref(h))
        if st != ECC_OK:
            raise EccError(st, f"ecc_ctx_create(device={device})")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _lib.ecc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return _lib.ecc_last_error(self._h).decode()

    def scratch_bytes(self) -> int:
        return int(_lib.ecc_ctx_scratch_bytes(self._h))

    def set_profiling(self, enable: bool) -> None:
        self._check(_lib.ecc_ctx_set_profiling(self._h, 1 if enable else 0))

    def stats(self) -> dict:
        st = ecc_stats()
        self._check(_lib.ecc_ctx_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def set_round_variant(self, variant: int) -> None:
        """Design variant of the bucket-round kernel (ablations; 0 = library form)."""
        self._check(_lib.ecc_ctx_set_round_variant(self._h, variant))

    def sync(self) -> None:
        """Wait for this context's ECC_ASYNC calls; raise the input error they found, if any."""
        self._check(_lib.ecc_ctx_sync(self._h))

    def _check(self, st: int):
        if st != ECC_OK:
            raise EccError(st, self.last_error())


def _opts(flags: int, window_c: int, stream) -> ecc_opts:
    """Call options.  Without an explicit stream, a call on device buffers runs
    on torch's current stream, so that it is ordered after the torch work that
    wrote its inputs and before later work on its outputs (torch's legacy
    default stream is handle 0, which the library maps to its own stream; that
    stream is a blocking one and so is ordered with the legacy default stream
    too).  Calls on host buffers stage their own copies."""
    s = None
    if stream is not None:
        s = stream if isinstance(stream, int) else stream.cuda_stream
    elif not (flags & ECC_HOST_PTRS):
        import torch
        if torch.cuda.is_available():
            s = torch.cuda.current_stream().cuda_stream or None
    return ecc_opts(flags, window_c, s)


def _host_flag(*flags):
    hosts = {f for f in flags if f is not None}
    if len(hosts) > 1:
        raise ValueError("mix of host and device buffers")
    return ECC_HOST_PTRS if hosts == {True} else 0


def ecc_msm(ctx: Context, curve: int, bases, scalars, n: int, out_xy, out_inf, flags: int = 0, window_c: int = 0,
            stream=None) -> None:
    """R = sum_i scalars_i * bases_i; writes out_xy (2L u64) and out_inf (1 byte)."""
    L = LIMBS[curve]
    pb, hb = _ptr(bases, n * 2 * L * 8) if n else (0, None)
    ps, hs = _ptr(scalars, n * 32) if n else (0, None)
    po, ho = _ptr(out_xy, 2 * L * 8)
    pi, hi = _ptr(out_inf, 1)
    f = flags | _host_flag(hb, hs, ho, hi)
    o = _opts(f, window_c, stream)
    ctx._check(_lib.ecc_msm(ctx.handle, curve, pb, ps, n, po, pi, ctypes.byref(o)))


def ecc_msm_batch(ctx: Context, curve: int, bases, scalars, offsets, out_xy, out_inf, flags: int = 0,
                  window_c: int = 0, stream=None) -> None:
    """R_j = sum over offsets[j] <= i < offsets[j+1] of scalars_i * bases_i for the
    m = len(offsets) - 1 MSMs; offsets is a host sequence of u64."""
    import numpy as np
    L = LIMBS[curve]
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    m = int(offs.shape[0]) - 1
    if m < 0:
        raise ValueError("offsets needs at least one entry")
    total = int(offs[-1]) if m >= 0 else 0
    if isinstance(bases, (list, tuple)):
        # one device buffer (or device address) per MSM, read in place
        if len(bases) != m:
            raise ValueError(f"{len(bases)} base buffers for {m} MSMs")
        addrs = []
        for j, b in enumerate(bases):
            nb = int(offs[j + 1] - offs[j]) * 2 * L * 8
            if isinstance(b, int):
                addrs.append(b)
                continue
            a, is_host = _ptr(b, nb) if nb else (b.data_ptr(), not b.is_cuda)
            if is_host:
                raise ValueError("per-MSM bases must be device buffers")
            addrs.append(a)
        table = (ctypes.c_void_p * max(1, m))(*addrs)
        ps, hs = _ptr(scalars, total * 32) if total else (0, None)
        po, ho = _ptr(out_xy, max(1, m) * 2 * L * 8)
        pi, hi = _ptr(out_inf, max(1, m))
        f = flags | ECC_BASES_PER_MSM | _host_flag(False, hs, ho, hi)
        o = _opts(f, window_c, stream)
        ctx._check(_lib.ecc_msm_batch(ctx.handle, curve, ctypes.cast(table, ctypes.c_void_p), ps,
                                      offs.ctypes.data, m, po, pi, ctypes.byref(o)))
        return
    pb, hb = _ptr(bases, total * 2 * L * 8) if total else (0, None)
    ps, hs = _ptr(scalars, total * 32) if total else (0, None)
    po, ho = _ptr(out_xy, max(1, m) * 2 * L * 8)
    pi, hi = _ptr(out_inf, max(1, m))
    f = flags | _host_flag(hb, hs, ho, hi)
    o = _opts(f, window_c, stream)
    ctx._check(_lib.ecc_msm_batch(ctx.handle, curve, pb, ps, offs.ctypes.data, m, po, pi, ctypes.byref(o)))


def ecc_msm_batch_scratch_bytes(ctx: Context, curve: int, offsets, flags: int = 0, window_c: int = 0) -> int:
    """Device scratch bytes an ecc_msm_batch call with these offsets would hold."""
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    out = ctypes.c_size_t(0)
    o = ecc_opts(flags, window_c, None)
    ctx._check(_lib.ecc_msm_batch_scratch_bytes(ctx.handle, curve, offs.ctypes.data, int(offs.shape[0]) - 1,
                                                ctypes.byref(o), ctypes.byref(out)))
    return int(out.value)


def ecc_verify_batch(ctx: Context, curve: int, hashes, pubkeys, sigs, m: int, valid, flags: int = 0,
                     stream=None) -> None:
    """valid_i = 1 iff signature (r_i, s_i) on hash_i verifies under Q_i (secp256r1 or SM2)."""
    ph, hh = _ptr(hashes, m * 32)
    pq, hq = _ptr(pubkeys, m * 64)
    ps, hs = _ptr(sigs, m * 64)
    pv, hv = _ptr(valid, m)
    f = flags | _host_flag(hh, hq, hs, hv)
    o = _opts(f, 0, stream)
    ctx._check(_lib.ecc_verify_batch(ctx.handle, curve, ph, pq, ps, m, pv, ctypes.byref(o)))


def ecc_verify_batch_noalloc(curve: int, hashes, pubkeys, sigs, m: int, valid, stream=None) -> None:
    """ecc_verify_batch's per-lane verification with no allocation: device
    buffers only, the library's fixed device array as scratch, on `stream`
    (default: torch's current stream)."""
    ph, hh = _ptr(hashes, m * 32)
    pq, hq = _ptr(pubkeys, m * 64)
    ps, hs = _ptr(sigs, m * 64)
    pv, hv = _ptr(valid, m)
    if m and _host_flag(hh, hq, hs, hv):
        raise ValueError("ecc_verify_batch_noalloc takes device buffers only")
    if stream is not None:
        s = stream if isinstance(stream, int) else stream.cuda_stream
    else:
        import torch
        s = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    st = _lib.ecc_verify_batch_noalloc(curve, ph, pq, ps, m, pv, s or None)
    if st != ECC_OK:
        raise EccError(st, f"ecc_verify_batch_noalloc(curve={curve}, m={m})")


def ecc_verify_batch_noalloc_max() -> int:
    """Largest request count ecc_verify_batch_noalloc accepts."""
    return int(_lib.ecc_verify_batch_noalloc_max())


def ecc_sign_batch(ctx: Context, curve: int, hashes, privkeys, nonces, m: int, sigs, flags: int = 0,
                   stream=None) -> None:
    """sigs_i = (r_i, s_i), the ECDSA signature of hash_i under d_i with nonce k_i
    (secp256r1 or SM2); all zero for out-of-range d_i, k_i or a zero r or s."""
    ph, hh = _ptr(hashes, m * 32)
    pd, hd = _ptr(privkeys, m * 32)
    pk, hk = _ptr(nonces, m * 32)
    ps, hs = _ptr(sigs, m * 64)
    f = flags | _host_flag(hh, hd, hk, hs)
    o = _opts(f, 0, stream)
    ctx._check(_lib.ecc_sign_batch(ctx.handle, curve, ph, pd, pk, m, ps, ctypes.byref(o)))


def ecc_pmul_batch(ctx: Context, curve: int, points, scalars, n: int, out_xy, flags: int = 0,
                   stream=None) -> None:
    """out_i = k_i P_i for run-time points P_i (canonical affine, (0, 0) = O)."""
    L = LIMBS[curve]
    pp, hp = _ptr(points, n * 2 * L * 8)
    pk, hk = _ptr(scalars, n * 32)
    po, ho = _ptr(out_xy, n * 2 * L * 8)
    f = flags | _host_flag(hp, hk, ho)
    o = _opts(f, 0, stream)
    ctx._check(_lib.ecc_pmul_batch(ctx.handle, curve, pp, pk, n, po, ctypes.byref(o)))


def ecc_tune(ctx: Context, curve: int, log2n_min: int, log2n_max: int, reps: int = 3) -> None:
    """Measure and adopt the window width and round shape for sizes 2^log2n_min .. 2^log2n_max."""
    ctx._check(_lib.ecc_tune(ctx.handle, curve, log2n_min, log2n_max, reps))


def ecc_tuned_params(ctx: Context, curve: int, n: int) -> tuple[int, int]:
    """(window_c, adds_per_lane) an MSM of n points would use now."""
    c, k = ctypes.c_int(0), ctypes.c_int(0)
    ctx._check(_lib.ecc_tuned_params(ctx.handle, curve, n, ctypes.byref(c), ctypes.byref(k)))
    return c.value, k.value


def ecc_tune_save(ctx: Context, path: str) -> None:
    ctx._check(_lib.ecc_tune_save(ctx.handle, os.fsencode(path)))


def ecc_tune_load(ctx: Context, path: str) -> int:
    """Adopt the entries of a tuning file that match this device; returns their count."""
    k = ctypes.c_int(0)
    ctx._check(_lib.ecc_tune_load(ctx.handle, os.fsencode(path), ctypes.byref(k)))
    return k.value


def ecc_fixed_base_mul(ctx: Context, curve: int, ks, n: int, out_xy, flags: int = 0, stream=None) -> None:
    """out_i = k_i G (canonical affine, or Montgomery with ECC_IN_MONTGOMERY)."""
    L = LIMBS[curve]
    pk, hk = _ptr(ks, n * 32)
    po, ho = _ptr(out_xy, n * 2 * L * 8)
    f = flags | _host_flag(hk, ho)
    o = _opts(f, 0, stream)
    ctx._check(_lib.ecc_fixed_base_mul(ctx.handle, curve, pk, n, po, ctypes.byref(o)))


def ecc_test_fp_mul(ctx: Context, curve: int, a, b, out, n: int) -> None:
    L = LIMBS[curve]
    ctx._check(_lib.ecc_test_fp_mul(ctx.handle, curve, _ptr(a, n * L * 8)[0], _ptr(b, n * L * 8)[0],
                                    _ptr(out, n * L * 8)[0], n))


def ecc_test_lane_field(ctx: Context, curve: int, op: int, a, b, out, n: int) -> None:
    """op 0: a b, op 1: a - b, op 2: 3a (a + b) - 2b (mod p), by the lane-parallel field."""
    L = LIMBS[curve]
    ctx._check(_lib.ecc_test_lane_field(ctx.handle, curve, op, _ptr(a, n * L * 8)[0], _ptr(b, n * L * 8)[0],
                                        _ptr(out, n * L * 8)[0], n))


def ecc_test_fp_inv(ctx: Context, curve: int, a, out, n: int) -> None:
    L = LIMBS[curve]
    ctx._check(_lib.ecc_test_fp_inv(ctx.handle, curve, _ptr(a, n * L * 8)[0], _ptr(out, n * L * 8)[0], n))


def ecc_test_batch_add(ctx: Context, curve: int, p, q, out, n: int) -> None:
    L = LIMBS[curve]
    nb = n * 2 * L * 8
    ctx._check(_lib.ecc_test_batch_add(ctx.handle, curve, _ptr(p, nb)[0], _ptr(q, nb)[0], _ptr(out, nb)[0], n))


PROBE_OPS = {"v_mad_u64_u32": 0, "v_fma_f64": 1, "v_mul_lo_u32": 2}


def ecc_probe_issue_rate(ctx: Context, op: str, chains: int, waves_per_simd: int, iters: int = 4096) -> dict:
    """Issue-rate probe of one instruction class: elapsed device time, lane
    operations, and the shader clock measured in the kernel."""
    ms, ops, mhz = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    ctx._check(library().ecc_probe_issue_rate(ctx.handle, PROBE_OPS[op], chains, waves_per_simd, iters,
                                              ctypes.byref(ms), ctypes.byref(ops), ctypes.byref(mhz)))
    return {"ms": ms.value, "lane_ops": ops.value, "shader_mhz": mhz.value}


def bucket_geometry(curve: int, window_c: int):
    """(windows W, buckets per window D, total buckets B) of the signed-digit split."""
    bits = SCALAR_BITS[curve]
    W = (bits + 1 + window_c - 1) // window_c
    D = 1 << (window_c - 1)
    return W, D, W * D


def ecc_test_bucket_sort(ctx: Context, curve: int, scalars, n: int, window_c: int, counts, offsets, sorted_,
                         method: int = 0) -> None:
    W, D, B = bucket_geometry(curve, window_c)
    ctx._check(_lib.ecc_test_bucket_sort(ctx.handle, curve, _ptr(scalars, n * 32)[0], n, window_c, method,
                                         _ptr(counts, (B + 1) * 4)[0], _ptr(offsets, (B + 1) * 4)[0],
                                         _ptr(sorted_, max(1, n * W) * 4)[0]))


class Server:
    """Continuous-batching request server (ecc_server_* of the C ABI).
    Requests are host arrays; results come back through wait()."""

    def __init__(self, device: int = 0, slots: int = 2, hbm_budget_bytes: int = 0,
                 max_batch_points: int = 1 << 22, max_batch_verify: int = 1 << 16, use_graph: bool = False,
                 test_exec=None):
        """test_exec: (msm_batch_bytes(sizes) -> int, run_batch(kind, sizes) -> (status, flags)),
        Python callables that replace the device (ecc_server_create_with_exec; tests only)."""
        cfg = ecc_server_cfg(slots, hbm_budget_bytes, max_batch_points, max_batch_verify, 1 if use_graph else 0)
        h = ctypes.c_void_p()
        self.handle = None
        self._limbs = {}
        if test_exec is None:
            st = _lib.ecc_server_create(device, ctypes.byref(cfg), ctypes.byref(h))
        else:
            plan, run = test_exec

            def _bytes(user, sizes, m):
                return int(plan([sizes[j] for j in range(m)]))

            def _run(user, kind, sizes, m, flags):
                st_, fl = run(kind, [sizes[j] for j in range(m)])
                for j in range(m):
                    flags[j] = int(fl[j]) if fl is not None else 0
                return int(st_)

            # the callbacks must outlive the server
            self._exec = ecc_server_exec(None, _MSM_BYTES_FN(_bytes), _RUN_BATCH_FN(_run))
            st = _lib.ecc_server_create_with_exec(ctypes.byref(cfg), ctypes.byref(self._exec), ctypes.byref(h))
        if st != ECC_OK:
            raise EccError(st, "ecc_server_create failed")
        self.handle = h

    def _check(self, st: int):
        if st != ECC_OK:
            raise EccError(st, _lib.ecc_server_last_error(self.handle).decode())

    def add_bases(self, curve: int, bases) -> int:
        """Upload bases (host u64 array, n x 2L) once; returns their id."""
        import numpy as np
        b = np.ascontiguousarray(bases, dtype=np.uint64)
        n = b.size // (2 * LIMBS[curve])
        bid = ctypes.c_uint32(0)
        self._check(_lib.ecc_server_add_bases(self.handle, curve, b.ctypes.data, n, ctypes.byref(bid)))
        self._limbs[bid.value] = LIMBS[curve]
        return bid.value

    def submit_msm(self, bases_id: int, first: int, scalars) -> int:
        import numpy as np
        s = np.ascontiguousarray(scalars, dtype=np.uint64)
        t = ctypes.c_uint64(0)
        self._check(_lib.ecc_server_submit_msm(self.handle, bases_id, first, s.size // 4, s.ctypes.data,
                                               ctypes.byref(t)))
        return (t.value, self._limbs[bases_id])

    def submit_verify(self, hash32, pubkey, sig) -> int:
        import numpy as np
        h = np.ascontiguousarray(hash32, dtype=np.uint8)
        q = np.ascontiguousarray(pubkey, dtype=np.uint64)
        g = np.ascontiguousarray(sig, dtype=np.uint64)
        t = ctypes.c_uint64(0)
        self._check(_lib.ecc_server_submit_verify(self.handle, h.ctypes.data, q.ctypes.data, g.ctypes.data,
                                                  ctypes.byref(t)))
        return (t.value, 0)

    def submit_verify_many(self, hashes, pubkeys, sigs) -> list:
        """m verifications queued at once (rows of hashes u8[m,32], pubkeys and sigs u64[m,8])."""
        import numpy as np
        h = np.ascontiguousarray(hashes, dtype=np.uint8)
        q = np.ascontiguousarray(pubkeys, dtype=np.uint64)
        g = np.ascontiguousarray(sigs, dtype=np.uint64)
        m = h.shape[0]
        t = np.zeros(max(1, m), dtype=np.uint64)
        self._check(_lib.ecc_server_submit_verify_many(self.handle, h.ctypes.data, q.ctypes.data, g.ctypes.data, m,
                                                       t.ctypes.data))
        return [(int(x), 0) for x in t[:m]]

    def wait_many(self, tickets):
        """Block for every ticket; (flags u8[m], latency_ms f64[m], status i32[m])."""
        import numpy as np
        ids = np.ascontiguousarray([t for t, _ in tickets], dtype=np.uint64)
        m = ids.size
        fl = np.zeros(max(1, m), dtype=np.uint8)
        lat = np.zeros(max(1, m), dtype=np.float64)
        stt = np.zeros(max(1, m), dtype=np.int32)
        self._check(_lib.ecc_server_wait_many(self.handle, ids.ctypes.data, m, fl.ctypes.data, lat.ctypes.data,
                                              stt.ctypes.data))
        return fl[:m], lat[:m], stt[:m]

    def wait(self, ticket, block: bool = True):
        """(xy u64 array or None, flag, latency_ms); flag = infinity (MSM) or valid (verify).
        Returns None when block is False and the request is not finished."""
        import numpy as np
        tid, L = ticket
        xy = np.zeros(max(1, 2 * L), dtype=np.uint64)
        flag = ctypes.c_uint8(0)
        lat = ctypes.c_double(0)
        st = _lib.ecc_server_wait(self.handle, tid, 1 if block else 0, xy.ctypes.data, ctypes.byref(flag),
                                  ctypes.byref(lat))
        if st == ECC_PENDING:
            return None
        self._check(st)
        return (xy if L else None), flag.value, lat.value

    def wait_status(self, ticket):
        """(status, flag): the request's status instead of an exception (blocks)."""
        tid, L = ticket
        import numpy as np
        xy = np.zeros(max(1, 2 * L), dtype=np.uint64)
        flag = ctypes.c_uint8(0)
        lat = ctypes.c_double(0)
        st = _lib.ecc_server_wait(self.handle, tid, 1, xy.ctypes.data, ctypes.byref(flag), ctypes.byref(lat))
        return st, flag.value

    def stats(self) -> dict:
        st = ecc_server_stats()
        self._check(_lib.ecc_server_get_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if self.handle:
            _lib.ecc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
