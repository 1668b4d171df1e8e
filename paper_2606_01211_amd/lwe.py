"""ctypes binding of liblwe_hip.so (the C ABI in include/lwe.h).

Argument marshalling only: every step of KeyGen / Encaps / Decaps runs in the HIP library.
Buffers may be torch tensors (CUDA/HIP device or CPU, uint8, contiguous), numpy arrays or
bytes.  Device tensors are passed by pointer together with the current torch stream, so the
calls queue asynchronously on that stream; host buffers make the call synchronous.

Raises ``LweLibraryMissing`` if the compiled library is absent: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblwe_hip.so")

LWE_OK, LWE_EINVAL, LWE_ENOMEM, LWE_EDEVICE, LWE_EUNSUPPORTED = 0, -1, -2, -3, -4

# every symbol include/lwe.h declares
EXPORTS = [
    "lwe_ctx_create", "lwe_ctx_destroy", "lwe_ctx_device_bytes", "lwe_ctx_set_budget", "lwe_ctx_trim",
    "lwe_ctx_call_bytes", "lwe_ctx_stream",
    "lwe_ctx_set_side_stream", "lwe_ctx_set_hash_lanes", "lwe_strerror",
    "lwe_param_id", "lwe_param_id_paper", "lwe_param_register", "lwe_param_get", "lwe_pk_bytes", "lwe_sk_bytes",
    "lwe_ct_bytes", "lwe_mu_bytes", "lwe_cdf_table",
    "lwe_keygen", "lwe_encaps", "lwe_decaps",
    "lwe_keygen_rand", "lwe_encaps_rand",
    "lwe_keygen_batch", "lwe_encaps_batch", "lwe_decaps_batch",
    "lwe_test_expand_A", "lwe_test_keystream", "lwe_test_sample", "lwe_test_sample_batch",
    "lwe_test_product", "lwe_test_encrypt",
    "lwe_test_decrypt", "lwe_test_sha3", "lwe_set_tuning", "lwe_get_tuning",
    "lwe_prof_enable", "lwe_prof_reset", "lwe_prof_read", "lwe_decaps_batch_noalloc",
]

KERNELS = ["sample", "prod_strip", "prod_strip_cmp", "prod_stream", "finalize", "decrypt", "fo_coins", "expand_keys",
           "hash_records", "final_ss", "fill", "keystream", "sample_stream", "expand_A", "drbg_chain", "pb_sample",
           "pb_rows", "pb_decrypt"]


class LweLibraryMissing(ImportError):
    pass


class LweError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, strerror(status), status))
        self.status = status


class ParamInfo(C.Structure):
    _fields_ = [
        ("n", C.c_uint32), ("logq", C.c_uint32), ("B", C.c_uint32), ("K", C.c_uint32),
        ("sigma", C.c_double), ("pk_bytes", C.c_size_t), ("sk_bytes", C.c_size_t),
        ("ct_bytes", C.c_size_t), ("mu_bytes", C.c_size_t),
        ("paper", C.c_uint32), ("q", C.c_uint32), ("nbar", C.c_uint32), ("mbar", C.c_uint32),
        ("coef_bytes", C.c_uint32), ("eta", C.c_uint32), ("k", C.c_uint32),
    ]


class Tuning(C.Structure):
    _fields_ = [
        ("col_groups", C.c_uint32), ("row_groups", C.c_uint32), ("m_chunks", C.c_uint32),
        ("host_hash_max", C.c_uint32), ("a_source", C.c_uint32),
    ]


_lib = None


def lib() -> C.CDLL:
    """Loads liblwe_hip.so (build it with ``python -m paper_2606_01211_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname as the
    # system one).  Loading torch first makes the library bind to that copy; the other
    # order would map two runtimes and the second would find no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise LweLibraryMissing(
            "liblwe_hip.so not found at %s; build it with python -m paper_2606_01211_amd.build"
            % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, sz, i32, u32, u64 = C.c_void_p, C.c_size_t, C.c_int, C.c_uint32, C.c_uint64
    sigs = {
        "lwe_ctx_create": (i32, [C.POINTER(vp), i32, sz]),
        "lwe_ctx_destroy": (None, [vp]),
        "lwe_ctx_device_bytes": (sz, [vp]),
        "lwe_ctx_set_budget": (i32, [vp, sz]),
        "lwe_ctx_trim": (i32, [vp]),
        "lwe_ctx_call_bytes": (sz, [vp, i32, i32, sz]),
        "lwe_ctx_stream": (vp, [vp]),
        "lwe_ctx_set_side_stream": (i32, [vp, i32]),
        "lwe_ctx_set_hash_lanes": (i32, [vp, i32]),
        "lwe_strerror": (C.c_char_p, [i32]),
        "lwe_param_id": (i32, [u32]),
        "lwe_param_id_paper": (i32, [u32]),
        "lwe_param_register": (i32, [u32, u32, u32, u32, C.c_double]),
        "lwe_param_get": (i32, [i32, C.POINTER(ParamInfo)]),
        "lwe_pk_bytes": (sz, [i32]),
        "lwe_sk_bytes": (sz, [i32]),
        "lwe_ct_bytes": (sz, [i32]),
        "lwe_mu_bytes": (sz, [i32]),
        "lwe_cdf_table": (i32, [i32, vp, sz]),
        "lwe_keygen": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "lwe_encaps": (i32, [vp, i32, vp, vp, vp, vp, vp]),
        "lwe_decaps": (i32, [vp, i32, vp, vp, vp, vp]),
        "lwe_keygen_rand": (i32, [vp, i32, sz, vp, vp, vp]),
        "lwe_encaps_rand": (i32, [vp, i32, sz, vp, vp, vp, vp]),
        "lwe_keygen_batch": (i32, [vp, i32, sz, vp, vp, vp, vp, vp, vp]),
        "lwe_encaps_batch": (i32, [vp, i32, sz, vp, vp, vp, vp, vp]),
        "lwe_decaps_batch": (i32, [vp, i32, sz, vp, vp, vp, vp]),
        "lwe_test_expand_A": (i32, [vp, i32, vp, u32, u32, vp, vp]),
        "lwe_test_keystream": (i32, [vp, vp, u32, u64, sz, vp, vp]),
        "lwe_test_sample": (i32, [vp, i32, vp, u32, u64, sz, vp, vp]),
        "lwe_test_sample_batch": (i32, [vp, i32, sz, i32, i32, vp, vp, vp, vp, vp, vp]),
        "lwe_test_product": (i32, [vp, i32, sz, vp, vp, vp, vp, vp, vp, vp, vp]),
        "lwe_test_encrypt": (i32, [vp, i32, sz, vp, vp, vp, vp, vp]),
        "lwe_test_decrypt": (i32, [vp, i32, sz, vp, vp, vp, vp]),
        "lwe_test_sha3": (i32, [vp, sz, sz, vp, vp, vp]),
        "lwe_set_tuning": (i32, [vp, i32, C.POINTER(Tuning)]),
        "lwe_get_tuning": (i32, [vp, i32, C.POINTER(Tuning)]),
        "lwe_prof_enable": (i32, [vp, i32]),
        "lwe_prof_reset": (i32, [vp]),
        "lwe_prof_read": (i32, [vp, C.c_char_p, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]),
        "lwe_decaps_batch_noalloc": (i32, [i32, sz, vp, vp, vp, vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().lwe_strerror(status).decode()


def _check(status: int, what: str) -> None:
    if status != LWE_OK:
        raise LweError(status, what)


# ---- parameter registry ------------------------------------------------------------------
@dataclass(frozen=True)
class Params:
    pid: int
    n: int
    logq: int
    B: int
    K: int
    sigma: float
    pk_bytes: int
    sk_bytes: int
    ct_bytes: int
    mu_bytes: int
    paper: int = 0       # 1 for the paper's own sets (Table 1)
    q: int = 0
    nbar: int = 8
    mbar: int = 8
    coef_bytes: int = 2
    eta: int = 0
    k: int = 0


def param_id(n: int) -> int:
    pid = lib().lwe_param_id(n)
    if pid < 0:
        raise KeyError("no parameter set for n=%d" % n)
    return pid


def param_id_paper(n: int) -> int:
    """Id of the paper's own set for n (Table 1: one encryption per message bit, prime q)."""
    pid = lib().lwe_param_id_paper(n)
    if pid < 0:
        raise KeyError("no Table 1 parameter set for n=%d" % n)
    return pid


def register_params(n: int, logq: int, B: int, K: int, sigma: float) -> int:
    pid = lib().lwe_param_register(n, logq, B, K, sigma)
    _check(pid if pid < 0 else 0, "lwe_param_register")
    return pid


_PARAMS: dict = {}


def params(pid: int) -> Params:
    # the registry is fixed once the library is loaded, so each set is asked for once: every
    # call below starts here, and a foreign call would give up the interpreter lock each time
    pp = _PARAMS.get(pid)
    if pp is not None:
        return pp
    info = ParamInfo()
    _check(lib().lwe_param_get(pid, C.byref(info)), "lwe_param_get")
    pp = _PARAMS[pid] = Params(pid, info.n, info.logq, info.B, info.K, info.sigma, info.pk_bytes,
                               info.sk_bytes, info.ct_bytes, info.mu_bytes, info.paper, info.q, info.nbar,
                               info.mbar, info.coef_bytes, info.eta, info.k)
    return pp


def cdf_table(pid: int) -> np.ndarray:
    p = params(pid)
    T = np.zeros(p.K + 1, np.uint16)
    _check(lib().lwe_cdf_table(pid, T.ctypes.data, T.size), "lwe_cdf_table")
    return T


# ---- buffers -----------------------------------------------------------------------------
def _torch():
    import torch  # imported lazily: only device memory and streams come from torch

    return torch


class _Arg:
    """Pointer view of a caller buffer; keeps temporaries alive for the call."""

    def __init__(self, x, nbytes: Optional[int] = None, writable: bool = False):
        self.keep = None
        self.device = False
        if x is None:
            self.ptr = None
            return
        mod = type(x).__module__
        if mod.startswith("torch"):
            if not x.is_contiguous():
                raise ValueError("tensor arguments must be contiguous")
            self.device = x.is_cuda
            self.ptr = x.data_ptr()
            size = x.numel() * x.element_size()
        elif isinstance(x, np.ndarray):
            if not x.flags["C_CONTIGUOUS"]:
                raise ValueError("array arguments must be C-contiguous")
            if writable and not x.flags["WRITEABLE"]:
                raise ValueError("output array is read-only")
            self.ptr = x.ctypes.data
            self.keep = x
            size = x.nbytes
        elif isinstance(x, (bytes, bytearray, memoryview)):
            if writable:
                raise ValueError("outputs must be tensors or numpy arrays")
            b = bytes(x)
            buf = (C.c_uint8 * max(1, len(b))).from_buffer_copy(b or b"\0")
            self.keep = buf
            self.ptr = C.addressof(buf)
            size = len(b)
        else:
            raise TypeError("unsupported buffer type %r" % type(x))
        if nbytes is not None and size < nbytes:
            raise ValueError("buffer holds %d bytes, %d needed" % (size, nbytes))


def _stream_ptr(args, stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    if any(a.device for a in args):
        torch = _torch()
        return torch.cuda.current_stream().cuda_stream
    return None


# bytes of the static device array behind decaps_batch_noalloc (LWE_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 32 << 20


def decaps_batch_noalloc(pid, count, sk, ct, ss, stream=None):
    """lwe_decaps_batch_noalloc: decapsulation on the current device that allocates no device
    memory (its working memory is the library's static per-device array).  sk, ct and ss must
    be device tensors; the work is queued on `stream` (default: torch's current stream)."""
    p = params(pid)
    a = [_Arg(sk, p.sk_bytes), _Arg(ct, p.ct_bytes * count), _Arg(ss, 32 * count, True)]
    if not all(x.device for x in a):
        raise ValueError("decaps_batch_noalloc takes device tensors only")
    st = _stream_ptr(a, stream)
    _check(lib().lwe_decaps_batch_noalloc(pid, count, *[x.ptr for x in a], st), "lwe_decaps_batch_noalloc")


class Context:
    """One lwe_ctx on one device (not thread-safe; use one per thread)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, tuning: bool = True):
        """tuning: apply the autotuner's table (tuning.json next to this file) if present."""
        self._lib = lib()
        h = C.c_void_p()
        _check(self._lib.lwe_ctx_create(C.byref(h), device, hbm_budget_bytes), "lwe_ctx_create")
        self._h = h
        self.device = device
        if tuning:
            from . import tune

            tune.apply_table(self, tune.load_table())

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.lwe_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def device_bytes(self) -> int:
        return self._lib.lwe_ctx_device_bytes(self._h)

    def set_budget(self, nbytes: int) -> None:
        """Bound on device_bytes for later calls (0 = none); held memory is not released."""
        _check(self._lib.lwe_ctx_set_budget(self._h, int(nbytes)), "lwe_ctx_set_budget")

    def trim(self) -> None:
        """Release the context's working buffers (ordered after its queued work)."""
        _check(self._lib.lwe_ctx_trim(self._h), "lwe_ctx_trim")

    def call_bytes(self, pid: int, op: int, count: int) -> int:
        """Device bytes one call of op (0 KeyGen, 1 Encaps, 2 Decaps) on count instances holds
        at most, starting from a trimmed context."""
        b = self._lib.lwe_ctx_call_bytes(self._h, pid, int(op), int(count))
        if b == 0:
            raise LweError(LWE_EINVAL, "lwe_ctx_call_bytes")
        return b

    @property
    def stream_handle(self) -> int:
        """The context's own HIP stream (an integer handle, e.g. for torch.cuda.ExternalStream)."""
        return self._lib.lwe_ctx_stream(self._h) or 0

    def set_side_stream(self, enable: bool) -> None:
        """Whether decaps_batch hashes the received ciphertexts on the context's second stream,
        overlapping the re-encryption (True, the default), or on the call's own stream, so
        that the context uses one stream only (False)."""
        _check(self._lib.lwe_ctx_set_side_stream(self._h, 1 if enable else 0), "lwe_ctx_set_side_stream")

    def set_hash_lanes(self, lanes: int) -> None:
        """Lanes per record of the batched SHA3 hashing: 2 (default, shorter latency) or 1 (less
        work per record, for many contexts at once)."""
        _check(self._lib.lwe_ctx_set_hash_lanes(self._h, int(lanes)), "lwe_ctx_set_hash_lanes")

    # ---- tuning ----
    def set_tuning(self, pid: int, col_groups=0, row_groups=0, m_chunks=0, host_hash_max=0, a_source=0):
        """a_source 0 regenerates A inside the product (fused), 1 expands it once per call
        into device memory first (unfused)."""
        t = Tuning(col_groups, row_groups, m_chunks, host_hash_max, a_source)
        _check(self._lib.lwe_set_tuning(self._h, pid, C.byref(t)), "lwe_set_tuning")

    def get_tuning(self, pid: int) -> dict:
        t = Tuning()
        _check(self._lib.lwe_get_tuning(self._h, pid, C.byref(t)), "lwe_get_tuning")
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    # ---- kernel timing ----
    def prof_enable(self, on: bool = True) -> None:
        _check(self._lib.lwe_prof_enable(self._h, 1 if on else 0), "lwe_prof_enable")

    def prof_reset(self) -> None:
        _check(self._lib.lwe_prof_reset(self._h), "lwe_prof_reset")

    def prof_read(self) -> dict:
        """{kernel: (launches, total device ms)} for kernels launched since the last reset."""
        out = {}
        for k in KERNELS:
            n, ms = C.c_uint64(), C.c_double()
            _check(self._lib.lwe_prof_read(self._h, k.encode(), C.byref(n), C.byref(ms)), "lwe_prof_read")
            if n.value:
                out[k] = (n.value, ms.value)
        return out

    # ---- KEM (outputs are caller-provided buffers) ----
    def keygen_batch(self, pid, count, seedA, seedSK, z, pk, sk, stream=None):
        p = params(pid)
        a = [_Arg(seedA, 16 * count), _Arg(seedSK, 16 * count), _Arg(z, 32 * count),
             _Arg(pk, p.pk_bytes * count, True), _Arg(sk, p.sk_bytes * count, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_keygen_batch(self._h, pid, count, *[x.ptr for x in a], st),
               "lwe_keygen_batch")

    def encaps_batch(self, pid, count, pk, mu, ct, ss, stream=None):
        p = params(pid)
        a = [_Arg(pk, p.pk_bytes), _Arg(mu, p.mu_bytes * count),
             _Arg(ct, p.ct_bytes * count, True), _Arg(ss, 32 * count, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_encaps_batch(self._h, pid, count, *[x.ptr for x in a], st),
               "lwe_encaps_batch")

    def decaps_batch(self, pid, count, sk, ct, ss, stream=None):
        p = params(pid)
        a = [_Arg(sk, p.sk_bytes), _Arg(ct, p.ct_bytes * count), _Arg(ss, 32 * count, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_decaps_batch(self._h, pid, count, *[x.ptr for x in a], st),
               "lwe_decaps_batch")

    def keygen_rand(self, pid, count, pk, sk, stream=None):
        """KeyGen with seeds drawn from the operating system's random source."""
        p = params(pid)
        a = [_Arg(pk, p.pk_bytes * count, True), _Arg(sk, p.sk_bytes * count, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_keygen_rand(self._h, pid, count, a[0].ptr, a[1].ptr, st), "lwe_keygen_rand")

    def encaps_rand(self, pid, count, pk, ct, ss, stream=None):
        """Encaps of messages drawn from the operating system's random source."""
        p = params(pid)
        a = [_Arg(pk, p.pk_bytes), _Arg(ct, p.ct_bytes * count, True), _Arg(ss, 32 * count, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_encaps_rand(self._h, pid, count, *[x.ptr for x in a], st), "lwe_encaps_rand")

    def keygen(self, pid, seedA, seedSK, z, pk, sk, stream=None):
        p = params(pid)
        a = [_Arg(seedA, 16), _Arg(seedSK, 16), _Arg(z, 32), _Arg(pk, p.pk_bytes, True),
             _Arg(sk, p.sk_bytes, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_keygen(self._h, pid, *[x.ptr for x in a], st), "lwe_keygen")

    def encaps(self, pid, pk, mu, ct, ss, stream=None):
        p = params(pid)
        a = [_Arg(pk, p.pk_bytes), _Arg(mu, p.mu_bytes), _Arg(ct, p.ct_bytes, True),
             _Arg(ss, 32, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_encaps(self._h, pid, *[x.ptr for x in a], st), "lwe_encaps")

    def decaps(self, pid, sk, ct, ss, stream=None):
        p = params(pid)
        a = [_Arg(sk, p.sk_bytes), _Arg(ct, p.ct_bytes), _Arg(ss, 32, True)]
        st = _stream_ptr(a, stream)
        _check(self._lib.lwe_decaps(self._h, pid, *[x.ptr for x in a], st), "lwe_decaps")

    # ---- test hooks ----
    def test_expand_A(self, pid, seedA, col0, ncols, out, stream=None):
        p = params(pid)
        a = [_Arg(seedA, 16), _Arg(out, 2 * ncols * p.n, True)]
        _check(self._lib.lwe_test_expand_A(self._h, pid, a[0].ptr, col0, ncols, a[1].ptr,
                                           _stream_ptr(a, stream)), "lwe_test_expand_A")

    def test_keystream(self, key, domain, block0, nblocks, out, stream=None):
        a = [_Arg(key, 16), _Arg(out, 16 * nblocks, True)]
        _check(self._lib.lwe_test_keystream(self._h, a[0].ptr, domain, block0, nblocks, a[1].ptr,
                                            _stream_ptr(a, stream)), "lwe_test_keystream")

    def test_sample(self, pid, key, domain, word0, count, out, stream=None):
        a = [_Arg(key, 16), _Arg(out, 2 * count, True)]
        _check(self._lib.lwe_test_sample(self._h, pid, a[0].ptr, domain, word0, count, a[1].ptr,
                                         _stream_ptr(a, stream)), "lwe_test_sample")

    def test_sample_batch(self, pid, count, mode, layout, keys, X, E, E2=None, X16=None, stream=None):
        """The batched sampler kernel (mode 0 KeyGen, 1 Encrypt) into the operand layout
        (0 row-major, 1 MFMA fragment order); see lwe_test_sample_batch."""
        p = params(pid)
        ldx = (p.n + 63) // 64 * 64
        rows = (count * 8 + 15) // 16 * 16 if layout else count * 8
        a = [_Arg(keys, 16 * count), _Arg(X, rows * ldx, True), _Arg(E, 8 * count * p.n, True),
             _Arg(E2, 64 * count, True), _Arg(X16, 16 * p.n * count, True)]
        _check(self._lib.lwe_test_sample_batch(self._h, pid, count, mode, layout, *[x.ptr for x in a],
                                               _stream_ptr(a, stream)), "lwe_test_sample_batch")

    def test_product(self, pid, count, seedA, Bt, S, E, E2, mu, ct, stream=None):
        """The encryption product with injected S', E', E'' (see lwe_test_product)."""
        p = params(pid)
        a = [_Arg(seedA, 16), _Arg(Bt, 16 * p.n), _Arg(S, 8 * count * p.n), _Arg(E, 8 * count * p.n),
             _Arg(E2, 64 * count), _Arg(mu, p.mu_bytes * count), _Arg(ct, p.ct_bytes * count, True)]
        _check(self._lib.lwe_test_product(self._h, pid, count, *[x.ptr for x in a], _stream_ptr(a, stream)),
               "lwe_test_product")

    def test_encrypt(self, pid, count, pk, coins, mu, ct, stream=None):
        p = params(pid)
        a = [_Arg(pk, p.pk_bytes), _Arg(coins, 16 * count), _Arg(mu, p.mu_bytes * count),
             _Arg(ct, p.ct_bytes * count, True)]
        _check(self._lib.lwe_test_encrypt(self._h, pid, count, *[x.ptr for x in a],
                                          _stream_ptr(a, stream)), "lwe_test_encrypt")

    def test_decrypt(self, pid, count, sk, ct, mu, stream=None):
        p = params(pid)
        a = [_Arg(sk, p.sk_bytes), _Arg(ct, p.ct_bytes * count), _Arg(mu, p.mu_bytes * count, True)]
        _check(self._lib.lwe_test_decrypt(self._h, pid, count, *[x.ptr for x in a],
                                          _stream_ptr(a, stream)), "lwe_test_decrypt")

    def test_sha3(self, count, length, data, out, stream=None):
        a = [_Arg(data, count * length), _Arg(out, 32 * count, True)]
        _check(self._lib.lwe_test_sha3(self._h, count, length, a[0].ptr, a[1].ptr,
                                       _stream_ptr(a, stream)), "lwe_test_sha3")
