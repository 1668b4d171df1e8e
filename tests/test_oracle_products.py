"""Pins of the oracle's products (Alg. 1-3 in matrix form) by brute force on tiny n.

A is rebuilt from OpenSSL's CTR keystream (an independent AES) with the column-major
index rule, the secrets and errors from the oracle's sampler (pinned exhaustively in
test_oracle_sampler.py), and every product is recomputed with numpy's int64 matmul."""
import shutil
import subprocess

import numpy as np
import pytest

import lwe_inputs

needs_openssl = pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI absent")

TINY = [(16, 16, 2, 6, 1.4), (24, 15, 2, 6, 1.4), (40, 16, 4, 5, 1.2), (64, 12, 3, 4, 1.0)]


def _A_openssl(p, seedA):
    ks = subprocess.run(["openssl", "enc", "-aes-128-ctr", "-K", seedA.hex(), "-iv", (0).to_bytes(16, "big").hex()],
                        input=bytes(2 * p.n * p.n), capture_output=True, check=True).stdout
    w = np.frombuffer(ks, dtype="<u2").astype(np.int64)
    # A[i][j] = word(j*n + i)
    return (w.reshape(p.n, p.n).T) % p.q


def _sample(orc, p, key, domain, count):
    return orc.sample_stream(p, key, domain, 0, count).astype(np.int64)


@needs_openssl
@pytest.mark.parametrize("n,logq,B,K,sigma", TINY)
def test_keygen_encrypt_decrypt_bruteforce(orc, n, logq, B, K, sigma):
    p = orc.Params(n, logq, B, K, sigma)
    g = lwe_inputs.rng(0, 300 + n)
    seedA, seedSK, coins = (lwe_inputs.random_bytes(g, 1, 16)[0].tobytes() for _ in range(3))
    mu = lwe_inputs.random_bytes(g, 1, p.mu_bytes)[0].tobytes()
    q = p.q
    A = _A_openssl(p, seedA)
    # KeyGen: B^T = S^T A^T + E^T
    St, Bt = orc.pke_keygen(p, seedA, seedSK)
    St_ref = _sample(orc, p, seedSK, 1, 8 * n).reshape(8, n)
    Et_ref = _sample(orc, p, seedSK, 2, 8 * n).reshape(8, n)
    assert np.array_equal(St.astype(np.int64), St_ref)
    assert np.array_equal(Bt.astype(np.int64), (St_ref @ A.T + Et_ref) % q)
    # Encrypt: B' = S' A + E', V = S' B + E'' + enc(mu)
    Bp, V = orc.pke_encrypt(p, seedA, Bt, coins, mu)
    Sp = _sample(orc, p, coins, 1, 8 * n).reshape(8, n)
    Ep = _sample(orc, p, coins, 2, 8 * n).reshape(8, n)
    Epp = _sample(orc, p, coins, 3, 64).reshape(8, 8)
    assert np.array_equal(Bp.astype(np.int64), (Sp @ A + Ep) % q)
    enc = np.array([orc.encode_coeff(p, mu, c) for c in range(64)], np.int64).reshape(8, 8)
    assert np.array_equal(V.astype(np.int64), (Sp @ Bt.astype(np.int64).T + Epp + enc) % q)
    # Decrypt: M = V - B' S
    M = orc.pke_decrypt_M(p, St, Bp, V)
    assert np.array_equal(M.astype(np.int64), (V.astype(np.int64) - Bp.astype(np.int64) @ St_ref.T) % q)
    # the V columns equal the V-only routine
    assert np.array_equal(orc.pke_V(p, Bt, coins, mu), V)
    # single-entry routines agree with the full products
    for c, i in [(0, 0), (7, n - 1), (3, n // 2)]:
        assert orc.Bt_entry(p, seedA, seedSK, c, i) == Bt[c, i]
    for r, j in [(0, 0), (7, n - 1), (5, n // 3)]:
        assert orc.Bp_entry(p, seedA, coins, r, j) == Bp[r, j]


@pytest.mark.parametrize("n", [640, 976, 1344])
def test_linearity_and_noise_identity(orc, n):
    """M - enc(mu) = S'E - E'S + E'' (mod q): the decryption identity behind Alg. 3."""
    p = orc.params_for(n)
    g = lwe_inputs.rng(0, 400 + n)
    seedA, seedSK, coins = (lwe_inputs.random_bytes(g, 1, 16)[0].tobytes() for _ in range(3))
    mu = lwe_inputs.random_bytes(g, 1, p.mu_bytes)[0].tobytes()
    q = p.q
    St, Bt = orc.pke_keygen(p, seedA, seedSK)
    Bp, V = orc.pke_encrypt(p, seedA, Bt, coins, mu)
    M = orc.pke_decrypt_M(p, St, Bp, V).astype(np.int64)
    Et = _sample(orc, p, seedSK, 2, 8 * n).reshape(8, n)
    Sp = _sample(orc, p, coins, 1, 8 * n).reshape(8, n)
    Ep = _sample(orc, p, coins, 2, 8 * n).reshape(8, n)
    Epp = _sample(orc, p, coins, 3, 64).reshape(8, 8)
    enc = np.array([orc.encode_coeff(p, mu, c) for c in range(64)], np.int64).reshape(8, 8)
    N = Sp @ Et.T - Ep @ St.astype(np.int64).T + Epp
    assert np.array_equal((M - enc) % q, N % q)
    assert int(np.abs(N).max()) == orc.noise_max(p, seedSK, coins)
    assert orc.pke_decode(p, M.astype(np.uint16)) == mu
