"""Pins of the oracle's AES-128 and CTR keystream (the seed expansion sample(rho) of Alg. 1
and the noise source of Sec. 3.3) against the published AES worked examples and against
OpenSSL run as an independent implementation."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import lwe_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "aes128_known_answers.txt")


def _golden(kind):
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == kind:
                rows.append([bytes.fromhex(x) for x in parts[1:]])
    return rows


def test_fips197_worked_examples(orc):
    rows = _golden("ecb")
    assert len(rows) == 2
    for key, pt, ct in rows:
        assert orc.aes128_encrypt(key, pt) == ct


def test_sp800_38a_ctr_vectors(orc):
    rows = _golden("ctr")
    assert len(rows) == 4
    for key, ctr, pt, ct in rows:
        ks = orc.aes128_encrypt(key, ctr)
        assert bytes(a ^ b for a, b in zip(ks, pt)) == ct


def test_key_schedule_last_round_key(orc):
    # FIPS-197 Appendix A.1: the expansion of 2b7e1516... ends with w[40..43] = d014f9a8 c9ee2589 e13f0cc8 b6630ca6
    rk = orc.aes128_round_keys(bytes.fromhex("2b7e151628aed2a6abf7158809cf4f3c"))
    assert rk[160:176].hex() == "d014f9a8c9ee2589e13f0cc8b6630ca6"


def _openssl_ctr(key: bytes, iv: bytes, nbytes: int) -> bytes:
    r = subprocess.run(
        ["openssl", "enc", "-aes-128-ctr", "-K", key.hex(), "-iv", iv.hex()],
        input=bytes(nbytes), capture_output=True, check=True)
    return r.stdout


needs_openssl = pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI absent")


@needs_openssl
@pytest.mark.parametrize("domain,block0,nblocks", [(0, 0, 64), (1, 0, 37), (2, 5, 40),
                                                    (3, 2**32 - 3, 8), (7, 2**40 + 11, 5)])
def test_ctr_keystream_matches_openssl(orc, domain, block0, nblocks):
    g = lwe_inputs.rng(0, 100 + domain)
    key = lwe_inputs.random_bytes(g, 1, 16)[0].tobytes()
    iv = domain.to_bytes(4, "big") + block0.to_bytes(12, "big")
    assert orc.ctr_blocks(key, domain, block0, nblocks) == _openssl_ctr(key, iv, 16 * nblocks)


@needs_openssl
def test_ctr_words_little_endian(orc):
    key = bytes(range(16))
    ks = _openssl_ctr(key, (2).to_bytes(4, "big") + bytes(12), 16 * 10)
    words = np.frombuffer(ks, dtype="<u2")
    got = orc.ctr_words(key, 2, 3, 70)
    assert np.array_equal(got, words[3:73])


@needs_openssl
@pytest.mark.parametrize("n", [640, 976])
def test_A_is_the_column_major_keystream(orc, n):
    """A[i][j] = word(j*n + i) mod q of the domain-0 keystream under seedA."""
    p = orc.params_for(n)
    g = lwe_inputs.rng(0, 7)
    seedA = lwe_inputs.random_bytes(g, 1, 16)[0].tobytes()
    cols = orc.expand_A_cols(p, seedA, 3, 4)  # columns 3..6
    ks = _openssl_ctr(seedA, bytes(16), 2 * n * 7)
    words = np.frombuffer(ks, dtype="<u2").astype(np.int64)
    for c in range(4):
        j = 3 + c
        expect = words[j * n:(j + 1) * n] % p.q
        assert np.array_equal(cols[c].astype(np.int64), expect)
    # single entries agree with the column expansion
    for i, j in [(0, 3), (n - 1, 6), (17, 4)]:
        assert orc.A_entry(p, seedA, i, j) == cols[j - 3][i]
