"""ctypes binding of libfrntt.so (C ABI declared in include/frntt.h).

Argument marshalling only: every step of every transform runs in the HIP
library. Device buffers are passed as integer addresses (for example
``tensor.data_ptr()`` of a torch CUDA/HIP tensor) and streams as integer
``hipStream_t`` handles (``torch.cuda.current_stream().cuda_stream``; 0 is
the null stream). If the library has not been built, loading raises: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libfrntt.so")

FWD, INV, COSET, COSET_INV = 0, 1, 2, 3
ALGO_AUTO, ALGO_BUTTERFLY, ALGO_FOURSTEP_MFMA = 0, 1, 2
VALIDATE = 1
SPLIT_TWIDDLES = 2

OK, EINVAL, ERANGE, EALIGN, ENOMEM, EHIP, EBUSY, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7

# Every exported entry point: name -> (restype, argtypes)
_vp = ctypes.c_void_p
_i = ctypes.c_int
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t


class Job(ctypes.Structure):
    _fields_ = [("data", _vp), ("log_n", _i), ("kind", _i)]


SIGNATURES = {
    "frntt_ctx_create": (_i, [ctypes.POINTER(_vp), _i, _i, ctypes.c_uint]),
    "frntt_ctx_destroy": (_i, [_vp]),
    "ntt_fwd": (_i, [_vp, _vp, _i, _i, _vp]),
    "ntt_inv": (_i, [_vp, _vp, _i, _i, _vp]),
    "ntt_coset": (_i, [_vp, _vp, _i, _i, _vp]),
    "ntt_coset_inv": (_i, [_vp, _vp, _i, _i, _vp]),
    "ntt_transform": (_i, [_vp, _vp, _i, _i, _i, _vp]),
    "ntt_transform_algo": (_i, [_vp, _vp, _i, _i, _i, _i, _vp]),
    "ntt_transform_noalloc": (_i, [_vp, _vp, _i, _i, _i, _vp]),
    "frntt_set_algo": (_i, [_vp, _i]),
    "frntt_get_algo": (_i, [_vp]),
    "frntt_set_plan": (_i, [_vp, _i, _i, ctypes.POINTER(_i), _i]),
    "frntt_get_plan": (_i, [_vp, _i, _i, ctypes.POINTER(_i), _i]),
    "frntt_get_plan_levels": (_i, [_vp, _i, _i, _i, ctypes.POINTER(_i), _i]),
    "ntt_batch": (_i, [_vp, ctypes.POINTER(Job), _i, _vp]),
    "ntt_batch_graph": (_i, [_vp, ctypes.POINTER(Job), _i, _vp]),
    "frntt_tune": (_i, [_vp, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i),
                        ctypes.POINTER(ctypes.c_float), _vp]),
    "frntt_tune_save": (_i, [_vp, ctypes.c_char_p]),
    "frntt_tune_load": (_i, [_vp, ctypes.c_char_p]),
    "frntt_generate": (_i, [_vp, _vp, _u64, _u64, _u64, _u64, _vp]),
    "frntt_check_inputs": (_i, [_vp]),
    "frntt_scratch_bytes": (_sz, [_i, _i]),
    "frntt_prepare": (_i, [_vp, _i, _i]),
    "frntt_table_bytes": (_sz, [_vp]),
    "frntt_last_hip_error": (_i, [_vp]),
    "frntt_strerror": (ctypes.c_char_p, [_i]),
    "frntt_server_create": (_i, [ctypes.POINTER(_vp), _vp, _sz, _i]),
    "frntt_server_submit": (_i, [_vp, _i, _i, _u64, ctypes.POINTER(_u64)]),
    "frntt_server_poll": (_i, [_vp, _u64, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double)]),
    "frntt_server_result": (_i, [_vp, _u64, _vp]),
    "frntt_server_release": (_i, [_vp, _u64]),
    "frntt_server_drain": (_i, [_vp, ctypes.c_double]),
    "frntt_server_set_release_on_done": (_i, [_vp, _i]),
    "frntt_server_stats": (_i, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                ctypes.POINTER(_u64)]),
    "frntt_server_peak_inflight": (_i, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "frntt_server_destroy": (_i, [_vp]),
    "frntt_rns_moduli": (_i, [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
    "frntt_rns_encode": (_i, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_rns_mul": (_i, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_rns_decode": (_i, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_mont_mul": (_i, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_rns_field_create": (_i, [ctypes.POINTER(_vp), _vp, ctypes.POINTER(ctypes.c_uint32), _i]),
    "frntt_rns_field_destroy": (_i, [_vp]),
    "frntt_rns_field_shape": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i),
                                   ctypes.POINTER(_i)]),
    "frntt_rns_field_encode": (_i, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_rns_field_mul": (_i, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_rns_field_decode": (_i, [_vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_rns_field_mont_mul": (_i, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "frntt_msm": (_i, [_vp, _vp, _vp, ctypes.c_int64, _i, _vp, _vp]),
    "frntt_msm_presort": (_i, [_vp, _vp, _vp, ctypes.c_int64, _i, _vp, _vp]),
    "frntt_msm_batch": (_i, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int64), _i,
                             _i, ctypes.POINTER(_vp), _vp]),
    "frntt_msm_window": (_i, [ctypes.c_int64]),
    "frntt_ec_mul": (_i, [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp]),
    "frntt_msm_workspace_bytes": (_sz, [ctypes.c_int64, _i]),
}

RNS_Q_WORDS = 20
RNS_P_WORDS = 12

# The wider moduli of the RNS lazy product: the largest primes below 2^377 and
# 2^753 (the paper evaluates 256/377/753-bit fields without naming curves).
FIELD_377 = (1 << 377) - 259
FIELD_753 = (1 << 753) - 1101

_lib = None


def rns_moduli():
    """(q_0..q_16, p_0..p_8) of the RNS lazy product (host only)."""
    q = (ctypes.c_uint32 * 17)()
    p = (ctypes.c_uint32 * 9)()
    _check(lib().frntt_rns_moduli(q, p), "frntt_rns_moduli")
    return list(q), list(p)


def msm_window(n: int) -> int:
    """Window width frntt_msm picks for n points (host only)."""
    return lib().frntt_msm_window(n)


def msm_workspace_bytes(n: int, window: int = 0) -> int:
    return lib().frntt_msm_workspace_bytes(n, window)


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libfrntt.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise FileNotFoundError(
                f"{_LIB_PATH} is not built; run `python -m paper_2604_17808_amd.build` "
                "(or __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class FrnttError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = lib().frntt_strerror(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")
        self.status = status


def _check(rc: int, what: str):
    if rc != OK:
        raise FrnttError(rc, what)
    return rc


class Context:
    """A frntt context on one HIP device (owns twiddle tables and scratch)."""

    def __init__(self, device: int = 0, max_log_n: int = 28, flags: int = 0):
        h = _vp()
        _check(lib().frntt_ctx_create(ctypes.byref(h), device, max_log_n, flags), "frntt_ctx_create")
        self._h = h
        self.device = device
        self.max_log_n = max_log_n

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().frntt_ctx_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- transforms on raw device addresses
    def transform(self, ptr: int, log_n: int, batch: int = 1, kind: int = FWD, stream: int = 0,
                  algo: int | None = None) -> int:
        if algo is None:
            rc = lib().ntt_transform(self._h, ptr, log_n, batch, kind, stream)
        else:
            rc = lib().ntt_transform_algo(self._h, ptr, log_n, batch, kind, algo, stream)
        return rc

    def transform_checked(self, ptr, log_n, batch=1, kind=FWD, stream=0, algo=None):
        return _check(self.transform(ptr, log_n, batch, kind, stream, algo), "ntt_transform")

    def fwd(self, ptr, log_n, batch=1, stream=0):
        return _check(lib().ntt_fwd(self._h, ptr, log_n, batch, stream), "ntt_fwd")

    def inv(self, ptr, log_n, batch=1, stream=0):
        return _check(lib().ntt_inv(self._h, ptr, log_n, batch, stream), "ntt_inv")

    def coset(self, ptr, log_n, batch=1, stream=0):
        return _check(lib().ntt_coset(self._h, ptr, log_n, batch, stream), "ntt_coset")

    def coset_inv(self, ptr, log_n, batch=1, stream=0):
        return _check(lib().ntt_coset_inv(self._h, ptr, log_n, batch, stream), "ntt_coset_inv")

    def set_algo(self, algo: int):
        return _check(lib().frntt_set_algo(self._h, algo), "frntt_set_algo")

    def get_algo(self) -> int:
        return lib().frntt_get_algo(self._h)

    def set_plan(self, algo: int, log_n: int, pass_logs):
        arr = (_i * max(1, len(pass_logs)))(*pass_logs)
        return _check(lib().frntt_set_plan(self._h, algo, log_n, arr, len(pass_logs)), "frntt_set_plan")

    def get_plan_levels(self, algo: int, log_n: int, pass_index: int):
        arr = (_i * 3)()
        n = lib().frntt_get_plan_levels(self._h, algo, log_n, pass_index, arr, 3)
        if n < 0:
            _check(n, "frntt_get_plan_levels")
        return list(arr[:n])

    def get_plan(self, algo: int, log_n: int):
        arr = (_i * 4)()
        n = lib().frntt_get_plan(self._h, algo, log_n, arr, 4)
        if n < 0:
            raise FrnttError(n, "frntt_get_plan")
        return list(arr[:n])

    def batch(self, jobs, stream: int = 0, graph: bool = False):
        """jobs: iterable of (device address, log_n, kind)."""
        jobs = list(jobs)
        arr = (Job * max(1, len(jobs)))(*[Job(p, l, k) for p, l, k in jobs])
        fn = lib().ntt_batch_graph if graph else lib().ntt_batch
        return _check(fn(self._h, arr, len(jobs), stream), "ntt_batch")

    def tune(self, log_n: int, batch: int = 1, stream: int = 0):
        a, p = _i(), _i()
        ms = ctypes.c_float()
        _check(lib().frntt_tune(self._h, log_n, batch, ctypes.byref(a), ctypes.byref(p),
                                ctypes.byref(ms), stream), "frntt_tune")
        return a.value, p.value, ms.value

    def tune_save(self, path: str):
        return _check(lib().frntt_tune_save(self._h, path.encode()), "frntt_tune_save")

    def tune_load(self, path: str):
        return _check(lib().frntt_tune_load(self._h, path.encode()), "frntt_tune_load")

    def generate(self, ptr: int, seed: int, stream_id: int, start: int, count: int, stream: int = 0):
        return _check(lib().frntt_generate(self._h, ptr, seed, stream_id, start, count, stream),
                      "frntt_generate")

    def prepare(self, log_n: int, kind: int = FWD):
        return _check(lib().frntt_prepare(self._h, log_n, kind), "frntt_prepare")

    def table_bytes(self) -> int:
        return lib().frntt_table_bytes(self._h)

    # RNS lazy modular product (pointers to device memory, n elements)
    def rns_encode(self, a: int, xq: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_encode(self._h, a, xq, n, stream), "frntt_rns_encode")

    def rns_mul(self, xa: int, xb: int, xp: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_mul(self._h, xa, xb, xp, n, stream), "frntt_rns_mul")

    def rns_decode(self, xp: int, out: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_decode(self._h, xp, out, n, stream), "frntt_rns_decode")

    def mont_mul(self, a: int, b: int, out: int, n: int, stream: int = 0):
        return _check(lib().frntt_mont_mul(self._h, a, b, out, n, stream), "frntt_mont_mul")

    # multi-scalar multiplication on the twisted Edwards curve over Fr:
    # scalars n x 8 words, points n x 16 words (x, y), out 16 words (x, y)
    def msm(self, scalars: int, points: int, n: int, out: int, window: int = 0, stream: int = 0):
        return _check(lib().frntt_msm(self._h, scalars, points, n, window, out, stream), "frntt_msm")

    def msm_batch(self, scalars, points, ns, outs, window: int = 0, stream: int = 0):
        """Independent MSMs (lists of device pointers and sizes) in one call."""
        k = len(ns)
        if not (len(scalars) == len(points) == len(outs) == k):
            raise ValueError("msm_batch: lists of different lengths")
        arr = lambda v: (_vp * max(k, 1))(*v)
        return _check(lib().frntt_msm_batch(self._h, arr(scalars), arr(points), (ctypes.c_int64 * max(k, 1))(*ns),
                                            k, window, arr(outs), stream), "frntt_msm_batch")

    def msm_presort(self, scalars: int, points: int, n: int, out: int, window: int = 0, stream: int = 0):
        """The Presort-PPG baseline of the same MSM (bit-identical)."""
        return _check(lib().frntt_msm_presort(self._h, scalars, points, n, window, out, stream),
                      "frntt_msm_presort")

    def ec_mul(self, scalars: int, points: int, n: int, out: int, stream: int = 0):
        return _check(lib().frntt_ec_mul(self._h, scalars, points, n, out, stream), "frntt_ec_mul")

    def check_inputs(self) -> int:
        return lib().frntt_check_inputs(self._h)

    def last_hip_error(self) -> int:
        return lib().frntt_last_hip_error(self._h)


class RnsField:
    """RNS lazy modular product over the prime field of `modulus` (at most 254,
    377 or 753 bits: 8, 12 or 24 words); see frntt_rns_field_* in
    include/frntt.h. Pointers are device addresses of n elements."""

    def __init__(self, ctx: "Context", modulus: int):
        bits = modulus.bit_length()
        self.words = 8 if bits <= 254 else 12 if bits <= 377 else 24
        self.modulus = modulus
        m = (ctypes.c_uint32 * self.words)(*[(modulus >> (32 * w)) & 0xFFFFFFFF for w in range(self.words)])
        h = _vp()
        _check(lib().frntt_rns_field_create(ctypes.byref(h), ctx.handle, m, self.words), "frntt_rns_field_create")
        self._h = h
        q, p, qw, pw = _i(), _i(), _i(), _i()
        _check(lib().frntt_rns_field_shape(self._h, ctypes.byref(q), ctypes.byref(p), ctypes.byref(qw),
                                           ctypes.byref(pw)), "frntt_rns_field_shape")
        self.n_q, self.n_p, self.q_words, self.p_words = q.value, p.value, qw.value, pw.value

    def encode(self, a: int, xq: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_field_encode(self._h, a, xq, n, stream), "frntt_rns_field_encode")

    def mul(self, xa: int, xb: int, xp: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_field_mul(self._h, xa, xb, xp, n, stream), "frntt_rns_field_mul")

    def decode(self, xp: int, out: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_field_decode(self._h, xp, out, n, stream), "frntt_rns_field_decode")

    def mont_mul(self, a: int, b: int, out: int, n: int, stream: int = 0):
        return _check(lib().frntt_rns_field_mont_mul(self._h, a, b, out, n, stream), "frntt_rns_field_mont_mul")

    def close(self):
        if getattr(self, "_h", None):
            lib().frntt_rns_field_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server (see frntt_server_* in include/frntt.h)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, slots: int = 4):
        h = _vp()
        _check(lib().frntt_server_create(ctypes.byref(h), ctx.handle, hbm_budget_bytes, slots),
               "frntt_server_create")
        self._h = h
        self.ctx = ctx

    def submit(self, kind: int, log_n: int, data_seed: int) -> int:
        t = _u64()
        _check(lib().frntt_server_submit(self._h, kind, log_n, data_seed, ctypes.byref(t)),
               "frntt_server_submit")
        return t.value

    def poll(self, ticket: int):
        done = _i()
        lat = ctypes.c_double()
        _check(lib().frntt_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(lat)),
               "frntt_server_poll")
        return bool(done.value), lat.value

    def result(self, ticket: int, host_ptr: int):
        return _check(lib().frntt_server_result(self._h, ticket, host_ptr), "frntt_server_result")

    def release(self, ticket: int):
        return _check(lib().frntt_server_release(self._h, ticket), "frntt_server_release")

    def drain(self, timeout_s: float = 600.0):
        return _check(lib().frntt_server_drain(self._h, timeout_s), "frntt_server_drain")

    def set_release_on_done(self, on: bool = True):
        return _check(lib().frntt_server_set_release_on_done(self._h, 1 if on else 0),
                      "frntt_server_set_release_on_done")

    def stats(self):
        c, b, p = _u64(), _u64(), _u64()
        _check(lib().frntt_server_stats(self._h, ctypes.byref(c), ctypes.byref(b), ctypes.byref(p)),
               "frntt_server_stats")
        pb, pr = _u64(), _u64()
        _check(lib().frntt_server_peak_inflight(self._h, ctypes.byref(pb), ctypes.byref(pr)),
               "frntt_server_peak_inflight")
        return {"completed": c.value, "batches": b.value, "peak_bytes": p.value,
                "peak_inflight_batches": pb.value, "peak_inflight_requests": pr.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().frntt_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
