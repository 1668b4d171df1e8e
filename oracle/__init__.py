"""Plain CPU oracle of the LWE KEM hot path -- TEST INFRASTRUCTURE ONLY.

ctypes front end of ``lwe_oracle.c`` (plain C, built with gcc).  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import this package.  It shares
no code with the GPU library and never imports it.

Every function follows the scheme of the paper (Sec. 2.1 eq. (1), Alg. 1-5) in the
matrix form nbar = mbar = 8, q = 2^logq; see ``lwe_oracle.h`` for the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lwe_oracle.c")
_SRC_PB = os.path.join(_HERE, "lwe_oracle_pb.c")
_LIB_PATH = os.path.join(_HERE, "liblwe_oracle.so")
NBAR = 8
MBAR = 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP threaded outer loops)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(_SRC_PB), os.path.getmtime(os.path.join(_HERE, "lwe_oracle.h"))
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, _SRC_PB, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [
        ("n", C.c_int),
        ("logq", C.c_int),
        ("B", C.c_int),
        ("K", C.c_int),
        ("sigma", C.c_double),
    ]


@dataclass(frozen=True)
class Params:
    n: int
    logq: int
    B: int
    K: int
    sigma: float

    @property
    def q(self) -> int:
        return 1 << self.logq

    @property
    def pk_bytes(self) -> int:
        return 16 + NBAR * self.n * 2

    @property
    def sk_bytes(self) -> int:
        return NBAR * self.n * 2 + self.pk_bytes + 64

    @property
    def ct_bytes(self) -> int:
        return MBAR * self.n * 2 + MBAR * NBAR * 2

    @property
    def mu_bytes(self) -> int:
        return MBAR * NBAR * self.B // 8

    def _c(self) -> _Params:
        return _Params(self.n, self.logq, self.B, self.K, self.sigma)


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        P = C.POINTER(_Params)
        u8p = C.c_void_p
        sigs = {
            "orc_params_for": (C.c_int, [C.c_int, P]),
            "orc_aes128_expand_key": (None, [u8p, u8p]),
            "orc_aes128_encrypt": (None, [u8p, u8p, u8p]),
            "orc_ctr_blocks": (None, [u8p, C.c_uint32, C.c_uint64, C.c_size_t, u8p]),
            "orc_ctr_words": (None, [u8p, C.c_uint32, C.c_uint64, C.c_size_t, u8p]),
            "orc_sha3_256": (None, [u8p, C.c_size_t, u8p]),
            "orc_cdf_table": (C.c_int, [C.c_int, C.c_double, u8p]),
            "orc_sample_word": (C.c_int, [C.c_uint16, u8p, C.c_int]),
            "orc_sample_stream": (None, [P, u8p, C.c_uint32, C.c_uint64, C.c_size_t, u8p]),
            "orc_expand_A_cols": (None, [P, u8p, C.c_int, C.c_int, u8p]),
            "orc_encode_coeff": (C.c_uint16, [P, u8p, C.c_int]),
            "orc_decode_value": (C.c_int, [P, C.c_uint16]),
            "orc_pke_keygen": (None, [P, u8p, u8p, u8p, u8p]),
            "orc_pke_encrypt": (None, [P, u8p, u8p, u8p, u8p, u8p, u8p]),
            "orc_pke_decrypt_M": (None, [P, u8p, u8p, u8p, u8p]),
            "orc_pke_decode": (None, [P, u8p, u8p]),
            "orc_A_entry": (C.c_uint16, [P, u8p, C.c_long, C.c_long]),
            "orc_Bt_entry": (C.c_uint16, [P, u8p, u8p, C.c_int, C.c_long]),
            "orc_Bp_entry": (C.c_uint16, [P, u8p, u8p, C.c_int, C.c_long]),
            "orc_noise_max": (C.c_long, [P, u8p, u8p]),
            "orc_pke_V": (None, [P, u8p, u8p, u8p, u8p]),
            "orc_kem_keygen": (None, [P, u8p, u8p, u8p, u8p, u8p]),
            "orc_kem_encaps": (None, [P, u8p, u8p, u8p, u8p]),
            "orc_kem_decaps": (C.c_int, [P, u8p, u8p, u8p]),
            "orc_fo_coins": (None, [P, u8p, u8p, u8p, u8p]),
            "orc_threads": (C.c_int, []),
            "orc_aes256_expand_key": (None, [u8p, u8p]),
            "orc_aes256_encrypt": (None, [u8p, u8p, u8p]),
            "orc_drbg_instantiate": (None, [u8p, u8p, u8p]),
            "orc_drbg_generate": (None, [u8p, u8p, C.c_size_t, u8p]),
            "orc_drbg_words": (None, [u8p, C.c_uint32, C.c_size_t, u8p]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _buf(b) -> C.Array:
    b = bytes(b)
    return (C.c_uint8 * max(1, len(b))).from_buffer_copy(b if b else b"\0")


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def params_for(n: int) -> Params:
    p = _Params()
    if lib().orc_params_for(n, C.byref(p)) != 0:
        raise KeyError("no parameter set for n=%d" % n)
    return Params(p.n, p.logq, p.B, p.K, p.sigma)


def threads() -> int:
    return lib().orc_threads()


# ---- AES / CTR / SHA3 -------------------------------------------------------------------
def aes128_encrypt(key: bytes, block: bytes) -> bytes:
    rk = (C.c_uint8 * 176)()
    lib().orc_aes128_expand_key(_buf(key), rk)
    out = (C.c_uint8 * 16)()
    lib().orc_aes128_encrypt(rk, _buf(block), out)
    return bytes(out)


def aes128_round_keys(key: bytes) -> bytes:
    rk = (C.c_uint8 * 176)()
    lib().orc_aes128_expand_key(_buf(key), rk)
    return bytes(rk)


def ctr_blocks(key: bytes, domain: int, block0: int, nblocks: int) -> bytes:
    out = np.zeros(16 * nblocks, np.uint8)
    lib().orc_ctr_blocks(_buf(key), domain, block0, nblocks, _ptr(out))
    return out.tobytes()


def ctr_words(key: bytes, domain: int, word0: int, nwords: int) -> np.ndarray:
    out = np.zeros(max(1, nwords), np.uint16)
    lib().orc_ctr_words(_buf(key), domain, word0, nwords, _ptr(out))
    return out[:nwords]


def sha3_256(data: bytes) -> bytes:
    out = (C.c_uint8 * 32)()
    lib().orc_sha3_256(_buf(data), len(data), out)
    return bytes(out)


# ---- sampler ----------------------------------------------------------------------------
def cdf_table(K: int, sigma: float) -> np.ndarray:
    T = np.zeros(K + 1, np.uint16)
    if lib().orc_cdf_table(K, sigma, _ptr(T)) != 0:
        raise ValueError("CDF table not strictly increasing for K=%d sigma=%g" % (K, sigma))
    return T


def sample_word(u: int, T: np.ndarray, K: int) -> int:
    T = np.ascontiguousarray(T, np.uint16)
    return lib().orc_sample_word(u, _ptr(T), K)


def sample_stream(p: Params, key: bytes, domain: int, word0: int, count: int) -> np.ndarray:
    out = np.zeros(max(1, count), np.int16)
    lib().orc_sample_stream(C.byref(p._c()), _buf(key), domain, word0, count, _ptr(out))
    return out[:count]


# ---- A and products ---------------------------------------------------------------------
def expand_A_cols(p: Params, seedA: bytes, col0: int, ncols: int) -> np.ndarray:
    """Returns [ncols, n]: row c is column col0+c of A."""
    out = np.zeros((ncols, p.n), np.uint16)
    lib().orc_expand_A_cols(C.byref(p._c()), _buf(seedA), col0, ncols, _ptr(out))
    return out


def encode_coeff(p: Params, mu: bytes, coeff: int) -> int:
    return lib().orc_encode_coeff(C.byref(p._c()), _buf(mu), coeff)


def decode_value(p: Params, x: int) -> int:
    return lib().orc_decode_value(C.byref(p._c()), x)


def pke_keygen(p: Params, seedA: bytes, seedSK: bytes):
    St = np.zeros((NBAR, p.n), np.int16)
    Bt = np.zeros((NBAR, p.n), np.uint16)
    lib().orc_pke_keygen(C.byref(p._c()), _buf(seedA), _buf(seedSK), _ptr(St), _ptr(Bt))
    return St, Bt


def pke_encrypt(p: Params, seedA: bytes, Bt: np.ndarray, coins: bytes, mu: bytes):
    Bt = np.ascontiguousarray(Bt, np.uint16)
    Bp = np.zeros((MBAR, p.n), np.uint16)
    V = np.zeros((MBAR, NBAR), np.uint16)
    lib().orc_pke_encrypt(
        C.byref(p._c()), _buf(seedA), _ptr(Bt), _buf(coins), _buf(mu), _ptr(Bp), _ptr(V)
    )
    return Bp, V


def pke_decrypt_M(p: Params, St: np.ndarray, Bp: np.ndarray, V: np.ndarray) -> np.ndarray:
    St = np.ascontiguousarray(St, np.int16)
    Bp = np.ascontiguousarray(Bp, np.uint16)
    V = np.ascontiguousarray(V, np.uint16)
    M = np.zeros((MBAR, NBAR), np.uint16)
    lib().orc_pke_decrypt_M(C.byref(p._c()), _ptr(St), _ptr(Bp), _ptr(V), _ptr(M))
    return M


def pke_decode(p: Params, M: np.ndarray) -> bytes:
    M = np.ascontiguousarray(M, np.uint16)
    out = (C.c_uint8 * p.mu_bytes)()
    lib().orc_pke_decode(C.byref(p._c()), _ptr(M), out)
    return bytes(out)


def A_entry(p: Params, seedA: bytes, i: int, j: int) -> int:
    return lib().orc_A_entry(C.byref(p._c()), _buf(seedA), i, j)


def Bt_entry(p: Params, seedA: bytes, seedSK: bytes, c: int, i: int) -> int:
    return lib().orc_Bt_entry(C.byref(p._c()), _buf(seedA), _buf(seedSK), c, i)


def Bp_entry(p: Params, seedA: bytes, coins: bytes, r: int, j: int) -> int:
    return lib().orc_Bp_entry(C.byref(p._c()), _buf(seedA), _buf(coins), r, j)


def pke_V(p: Params, Bt: np.ndarray, coins: bytes, mu: bytes) -> np.ndarray:
    Bt = np.ascontiguousarray(Bt, np.uint16)
    V = np.zeros((MBAR, NBAR), np.uint16)
    lib().orc_pke_V(C.byref(p._c()), _ptr(Bt), _buf(coins), _buf(mu), _ptr(V))
    return V


def noise_max(p: Params, seedSK: bytes, coins: bytes) -> int:
    return lib().orc_noise_max(C.byref(p._c()), _buf(seedSK), _buf(coins))


# ---- KEM --------------------------------------------------------------------------------
def kem_keygen(p: Params, seedA: bytes, seedSK: bytes, z: bytes):
    pk = (C.c_uint8 * p.pk_bytes)()
    sk = (C.c_uint8 * p.sk_bytes)()
    lib().orc_kem_keygen(C.byref(p._c()), _buf(seedA), _buf(seedSK), _buf(z), pk, sk)
    return bytes(pk), bytes(sk)


def kem_encaps(p: Params, pk: bytes, mu: bytes):
    ct = (C.c_uint8 * p.ct_bytes)()
    ss = (C.c_uint8 * 32)()
    lib().orc_kem_encaps(C.byref(p._c()), _buf(pk), _buf(mu), ct, ss)
    return bytes(ct), bytes(ss)


def kem_decaps(p: Params, sk: bytes, ct: bytes):
    """Returns (shared secret, accepted)."""
    ss = (C.c_uint8 * 32)()
    ok = lib().orc_kem_decaps(C.byref(p._c()), _buf(sk), _buf(ct), ss)
    return bytes(ss), bool(ok)


def fo_coins(p: Params, pkh: bytes, mu: bytes):
    coins = (C.c_uint8 * 16)()
    kp = (C.c_uint8 * 32)()
    lib().orc_fo_coins(C.byref(p._c()), _buf(pkh), _buf(mu), coins, kp)
    return bytes(coins), bytes(kp)


# ---- AES-256 and the CTR_DRBG noise source ----------------------------------------------
def aes256_encrypt(key: bytes, block: bytes) -> bytes:
    rk = (C.c_uint8 * 240)()
    lib().orc_aes256_expand_key(_buf(key), rk)
    out = (C.c_uint8 * 16)()
    lib().orc_aes256_encrypt(rk, _buf(block), out)
    return bytes(out)


def drbg_instantiate(entropy: bytes):
    """(Key, V) after Instantiate with a 48-byte entropy input (no personalization)."""
    key = (C.c_uint8 * 32)()
    V = (C.c_uint8 * 16)()
    lib().orc_drbg_instantiate(_buf(entropy), key, V)
    return bytes(key), bytes(V)


def drbg_generate(key: bytes, V: bytes, nbytes: int):
    """One Generate request: (output, new Key, new V)."""
    k = (C.c_uint8 * 32).from_buffer_copy(key)
    v = (C.c_uint8 * 16).from_buffer_copy(V)
    out = (C.c_uint8 * max(1, nbytes))()
    lib().orc_drbg_generate(k, v, nbytes, out)
    return bytes(out)[:nbytes], bytes(k), bytes(v)


def drbg_words(key16: bytes, domain: int, nwords: int) -> np.ndarray:
    out = np.zeros(max(1, nwords), np.uint16)
    lib().orc_drbg_words(_buf(key16), domain, nwords, _ptr(out))
    return out[:nwords]
