"""All-cores CPU implementation of the matrix-form KEM, the CPU side of the GPU-versus-CPU
comparison (the paper compares with a multithreaded OpenMP CPU version on all cores,
Sec. 4.1).  ctypes front end of ``lwe_cpu.cpp`` (g++, OpenMP, AES-NI, AVX2).

It is a comparator, not part of the GPU product path: the GPU library and its Python binding
never load it, and it shares no code with the oracle.  The benchmark times it; the tests
check it byte for byte against the oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lwe_cpu.cpp")
_HDR = os.path.join(_HERE, "lwe_cpu.h")
_LIB_PATH = os.path.join(_HERE, "liblwe_cpu.so")


def build(force: bool = False) -> str:
    """Compile with g++ for x86-64 hosts with AES-NI and AVX2 (portable across the build
    machine and the GPU hosts)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
            os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-mavx2", "-maes", "-mpclmul", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _P(C.Structure):
    _fields_ = [("n", C.c_int), ("logq", C.c_int), ("B", C.c_int), ("K", C.c_int), ("sigma", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        vp, sz, P = C.c_void_p, C.c_size_t, C.POINTER(_P)
        for name, res, args in (
            ("lwc_threads", C.c_int, []),
            ("lwc_keygen_batch", C.c_int, [P, sz, vp, vp, vp, vp, vp]),
            ("lwc_encaps_batch", C.c_int, [P, sz, vp, vp, vp, vp]),
            ("lwc_decaps_batch", C.c_int, [P, sz, vp, vp, vp]),
        ):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def threads() -> int:
    return lib().lwc_threads()


class Kem:
    """KEM of one matrix-form parameter set (n, logq, B, K, sigma)."""

    def __init__(self, n: int, logq: int, B: int, K: int, sigma: float):
        self.p = _P(n, logq, B, K, sigma)
        self.pk_bytes = 16 + 16 * n
        self.sk_bytes = 16 * n + self.pk_bytes + 64
        self.ct_bytes = 16 * n + 128
        self.mu_bytes = 8 * B

    @staticmethod
    def _c(a: np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data_as(C.c_void_p)

    def keygen_batch(self, seedA, seedSK, z):
        count = len(seedA)
        pk = np.zeros((count, self.pk_bytes), np.uint8)
        sk = np.zeros((count, self.sk_bytes), np.uint8)
        lib().lwc_keygen_batch(C.byref(self.p), count, *[self._c(np.ascontiguousarray(x, np.uint8)) for x in
                                                         (seedA, seedSK, z)], self._c(pk), self._c(sk))
        return pk, sk

    def encaps_batch(self, pk, mu):
        count = len(mu)
        ct = np.zeros((count, self.ct_bytes), np.uint8)
        ss = np.zeros((count, 32), np.uint8)
        lib().lwc_encaps_batch(C.byref(self.p), count, self._c(np.ascontiguousarray(pk, np.uint8)),
                               self._c(np.ascontiguousarray(mu, np.uint8)), self._c(ct), self._c(ss))
        return ct, ss

    def decaps_batch(self, sk, ct):
        count = len(ct)
        ss = np.zeros((count, 32), np.uint8)
        lib().lwc_decaps_batch(C.byref(self.p), count, self._c(np.ascontiguousarray(sk, np.uint8)),
                               self._c(np.ascontiguousarray(ct, np.uint8)), self._c(ss))
        return ss
