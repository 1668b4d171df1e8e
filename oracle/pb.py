"""Oracle of the paper's own parameterisation -- TEST INFRASTRUCTURE ONLY.

ctypes front end of ``lwe_oracle_pb.c``: one encryption per message bit (256 rows u_r and
values v_r per ciphertext), prime q and the noise distributions of the paper's Table 1
(binomial eta for s, discrete Gaussian sigma for e, r, e1, centred uniform k for e2), all
noise from the AES-256 CTR_DRBG.  See ``lwe_oracle.h`` for the definitions.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _buf, _ptr, lib as _lib

BITS = 256
BINOMIAL, GAUSSIAN, UNIFORM = 0, 1, 2
TABLE1_N = (512, 1024, 2048, 4096, 8192, 16384, 32768)


class _PbParams(C.Structure):
    _fields_ = [("n", C.c_int), ("q", C.c_int), ("sigma", C.c_double), ("K", C.c_int), ("k", C.c_int),
                ("eta", C.c_int)]


@dataclass(frozen=True)
class PbParams:
    n: int
    q: int
    sigma: float
    K: int
    k: int
    eta: int

    @property
    def coef_bytes(self) -> int:
        return 4 if self.q > 65536 else 2

    @property
    def pk_bytes(self) -> int:
        return 16 + self.n * self.coef_bytes

    @property
    def sk_bytes(self) -> int:
        return 2 * self.n + self.pk_bytes + 64

    @property
    def ct_bytes(self) -> int:
        return BITS * (self.n + 1) * self.coef_bytes

    mu_bytes = 32

    def _c(self) -> _PbParams:
        return _PbParams(self.n, self.q, self.sigma, self.K, self.k, self.eta)


_done = False


def lib():
    global _done
    L = _lib()
    if not _done:
        P = C.POINTER(_PbParams)
        vp = C.c_void_p
        sigs = {
            "orc_pb_params_for": (C.c_int, [C.c_int, P]),
            "orc_pb_support": (C.c_int, [C.c_double]),
            "orc_pb_binomial": (C.c_int, [C.c_uint16, C.c_int]),
            "orc_pb_uniform": (C.c_int, [C.c_uint16, C.c_int]),
            "orc_pb_noise": (None, [P, vp, C.c_uint32, C.c_int, C.c_size_t, vp]),
            "orc_pb_expand_A_cols": (None, [P, vp, C.c_int, C.c_int, vp]),
            "orc_pb_pke_keygen": (None, [P, vp, vp, vp, vp]),
            "orc_pb_pke_encrypt": (None, [P, vp, vp, vp, vp, vp, vp]),
            "orc_pb_decode": (C.c_int, [C.c_int, C.c_uint32]),
            "orc_pb_pke_decrypt": (None, [P, vp, vp, vp, vp]),
            "orc_pb_noise_max": (C.c_long, [P, vp, vp]),
            "orc_pb_t_entry": (C.c_uint32, [P, vp, vp, C.c_long]),
            "orc_pb_u_entry": (C.c_uint32, [P, vp, vp, C.c_int, C.c_long]),
            "orc_pb_kem_keygen": (None, [P, vp, vp, vp, vp, vp]),
            "orc_pb_kem_encaps": (None, [P, vp, vp, vp, vp]),
            "orc_pb_kem_decaps": (C.c_int, [P, vp, vp, vp]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _done = True
    return L


def params_for(n: int) -> PbParams:
    p = _PbParams()
    if lib().orc_pb_params_for(n, C.byref(p)) != 0:
        raise KeyError("no Table 1 parameter set for n=%d" % n)
    return PbParams(p.n, p.q, p.sigma, p.K, p.k, p.eta)


def custom(n: int, q: int, sigma: float, k: int, eta: int = 3) -> PbParams:
    """A parameter set outside Table 1 (small n for brute-force checks)."""
    return PbParams(n, q, sigma, lib().orc_pb_support(sigma), k, eta)


def support(sigma: float) -> int:
    return lib().orc_pb_support(sigma)


def binomial(w: int, eta: int) -> int:
    return lib().orc_pb_binomial(w, eta)


def uniform(w: int, k: int) -> int:
    return lib().orc_pb_uniform(w, k)


def noise(p: PbParams, key: bytes, domain: int, dist: int, count: int) -> np.ndarray:
    out = np.zeros(max(1, count), np.int16)
    lib().orc_pb_noise(C.byref(p._c()), _buf(key), domain, dist, count, _ptr(out))
    return out[:count]


def expand_A_cols(p: PbParams, seedA: bytes, col0: int, ncols: int) -> np.ndarray:
    out = np.zeros((ncols, p.n), np.uint32)
    lib().orc_pb_expand_A_cols(C.byref(p._c()), _buf(seedA), col0, ncols, _ptr(out))
    return out


def pke_keygen(p: PbParams, seedA: bytes, seedSK: bytes):
    s = np.zeros(p.n, np.int16)
    t = np.zeros(p.n, np.uint32)
    lib().orc_pb_pke_keygen(C.byref(p._c()), _buf(seedA), _buf(seedSK), _ptr(s), _ptr(t))
    return s, t


def pke_encrypt(p: PbParams, seedA: bytes, t: np.ndarray, coins: bytes, mu: bytes):
    t = np.ascontiguousarray(t, np.uint32)
    U = np.zeros((BITS, p.n), np.uint32)
    v = np.zeros(BITS, np.uint32)
    lib().orc_pb_pke_encrypt(C.byref(p._c()), _buf(seedA), _ptr(t), _buf(coins), _buf(mu), _ptr(U), _ptr(v))
    return U, v


def decode(q: int, x: int) -> int:
    return lib().orc_pb_decode(q, x)


def pke_decrypt(p: PbParams, s: np.ndarray, U: np.ndarray, v: np.ndarray) -> bytes:
    s = np.ascontiguousarray(s, np.int16)
    U = np.ascontiguousarray(U, np.uint32)
    v = np.ascontiguousarray(v, np.uint32)
    out = (C.c_uint8 * 32)()
    lib().orc_pb_pke_decrypt(C.byref(p._c()), _ptr(s), _ptr(U), _ptr(v), out)
    return bytes(out)


def noise_max(p: PbParams, seedSK: bytes, coins: bytes) -> int:
    return lib().orc_pb_noise_max(C.byref(p._c()), _buf(seedSK), _buf(coins))


def t_entry(p: PbParams, seedA: bytes, seedSK: bytes, i: int) -> int:
    return lib().orc_pb_t_entry(C.byref(p._c()), _buf(seedA), _buf(seedSK), i)


def u_entry(p: PbParams, seedA: bytes, coins: bytes, r: int, j: int) -> int:
    return lib().orc_pb_u_entry(C.byref(p._c()), _buf(seedA), _buf(coins), r, j)


def kem_keygen(p: PbParams, seedA: bytes, seedSK: bytes, z: bytes):
    pk = (C.c_uint8 * p.pk_bytes)()
    sk = (C.c_uint8 * p.sk_bytes)()
    lib().orc_pb_kem_keygen(C.byref(p._c()), _buf(seedA), _buf(seedSK), _buf(z), pk, sk)
    return bytes(pk), bytes(sk)


def kem_encaps(p: PbParams, pk: bytes, mu: bytes):
    ct = (C.c_uint8 * p.ct_bytes)()
    ss = (C.c_uint8 * 32)()
    lib().orc_pb_kem_encaps(C.byref(p._c()), _buf(pk), _buf(mu), ct, ss)
    return bytes(ct), bytes(ss)


def kem_decaps(p: PbParams, sk: bytes, ct: bytes):
    """Returns (shared secret, accepted)."""
    ss = (C.c_uint8 * 32)()
    ok = lib().orc_pb_kem_decaps(C.byref(p._c()), _buf(sk), _buf(ct), ss)
    return bytes(ss), bool(ok)
