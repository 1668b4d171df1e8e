"""Pins of the oracle's second part: the paper's own parameterisation (one encryption per
message bit, prime q of Table 1, binomial / Gaussian / uniform noise) and its noise source,
an AES-256 CTR_DRBG (Sec. 3.3).

What pins what:
* AES-256: the FIPS-197 C.3 and SP 800-38A F.5.5 values (tests/golden/aes256_known_answers.txt)
  and OpenSSL as an independent implementation (ECB blocks, CTR keystream with carries).
* CTR_DRBG: the composition (Instantiate / Generate / Update of SP 800-90A 10.2.1) has no
  published vector in this container -- parity unpinned beyond its AES-256 primitive; the
  tests check its structural properties only (request independence of the word stream,
  distinct domains, output blocks are AES-256 of consecutive counters).
* Samplers: exhaustive 2^16 histograms against closed forms (binomial counts 2^10 C(6, 3+x);
  the uniform map's counts; Gaussian = the CDF sampler pinned in test_oracle_sampler).
* A mod q, t = A s + e, u_r = A^T r_r + e1_r, v_r = t^T r_r + e2_r + bit round(q/2): numpy
  brute force over the OpenSSL-pinned AES-128 keystream at small n.
* Decode: exhaustive over [0, q) against Alg. 3's inequalities in exact rational arithmetic.
* KEM: decaps(encaps(pk)) = K over seeds at n = 512 and 1024, the noise below q/4, and
  implicit rejection of tampered ciphertexts giving exactly H(z || H(ct)).
"""
import hashlib
import os
import shutil
import subprocess
from fractions import Fraction
from math import comb

import numpy as np
import pytest

import lwe_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "aes256_known_answers.txt")
needs_openssl = pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI absent")
H = lambda b: hashlib.sha3_256(b).digest()  # noqa: E731


@pytest.fixture(scope="module")
def pb(orc):
    import oracle.pb as m

    return m


def _golden(kind):
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            parts = line.split()
            if parts[0] == kind:
                rows.append([bytes.fromhex(x) for x in parts[1:]])
    return rows


def test_aes256_published_vectors(orc):
    rows = _golden("ecb")
    assert len(rows) == 1
    for key, pt, ct in rows:
        assert orc.aes256_encrypt(key, pt) == ct
    rows = _golden("ctr")
    assert len(rows) == 2
    for key, ctr, pt, ct in rows:
        assert bytes(a ^ b for a, b in zip(orc.aes256_encrypt(key, ctr), pt)) == ct


@needs_openssl
def test_aes256_against_openssl(orc):
    g = lwe_inputs.rng(0, 300)
    keys = lwe_inputs.random_bytes(g, 6, 32)
    blocks = lwe_inputs.random_bytes(g, 6, 16)
    for key, blk in zip(keys, blocks):
        r = subprocess.run(["openssl", "enc", "-aes-256-ecb", "-nopad", "-K", key.tobytes().hex()],
                           input=blk.tobytes(), capture_output=True, check=True)
        assert orc.aes256_encrypt(key.tobytes(), blk.tobytes()) == r.stdout


@needs_openssl
def test_drbg_generate_is_aes256_ctr_from_v_plus_one(orc):
    """A Generate request's output is AES-256 of V+1, V+2, ... under the current key: the
    same bytes as OpenSSL's CTR keystream from IV = V + 1 (its counter also carries over the
    whole 128 bits), here across a carry out of the low 64 bits."""
    g = lwe_inputs.rng(0, 301)
    key = lwe_inputs.random_bytes(g, 1, 32)[0].tobytes()
    V = bytes.fromhex("0123456789abcdef" + "ffffffffffffffff")[:16]
    V = V[:8] + bytes.fromhex("fffffffffffffffd")
    out, _, _ = orc.drbg_generate(key, V, 160)
    iv = (int.from_bytes(V, "big") + 1) % (1 << 128)
    r = subprocess.run(["openssl", "enc", "-aes-256-ctr", "-K", key.hex(), "-iv", iv.to_bytes(16, "big").hex()],
                       input=bytes(160), capture_output=True, check=True)
    assert out == r.stdout


def test_drbg_stream_structure(orc):
    """The noise word stream does not depend on how much of it is read (every request is a
    full 2^16 bytes), crosses request boundaries, and differs between keys and domains."""
    key = bytes(range(16))
    long = orc.drbg_words(key, 1, 70000)
    assert np.array_equal(orc.drbg_words(key, 1, 33000), long[:33000])
    assert not np.array_equal(orc.drbg_words(key, 2, 1000), long[:1000])
    assert not np.array_equal(orc.drbg_words(bytes(16), 1, 1000), long[:1000])
    # the first 2^15 words are request 0: the bytes of one Generate after Instantiate
    ent = key + (1).to_bytes(4, "little") + bytes(28)
    k, v = orc.drbg_instantiate(ent)
    out, k2, v2 = orc.drbg_generate(k, v, 65536)
    assert np.array_equal(np.frombuffer(out, "<u2"), long[:32768])
    out2, _, _ = orc.drbg_generate(k2, v2, 65536)
    assert np.array_equal(np.frombuffer(out2, "<u2"), long[32768:65536])
    # the Update after a request re-keys: the next request is not the continuation of the first
    cont, _, _ = orc.drbg_generate(k, v, 2 * 65536)
    assert cont[65536:65600] != out2[:64]


def test_binomial_exhaustive(pb):
    """eta = 3: a - b with a, b the bit counts of the two 3-bit fields; over all 2^16 words
    value x occurs 2^10 C(6, 3 + x) times (the other 10 bits are ignored)."""
    vals = np.array([pb.binomial(w, 3) for w in range(1 << 16)])
    for x in range(-3, 4):
        assert int((vals == x).sum()) == (1 << 10) * comb(6, 3 + x)
    assert vals.min() == -3 and vals.max() == 3


@pytest.mark.parametrize("k", [1, 2, 3])
def test_uniform_exhaustive(pb, k):
    """floor(w (2k+1) / 2^16) - k: value x takes the words w with
    2^16 (x+k) <= w (2k+1) < 2^16 (x+k+1), i.e. counts that differ by at most one."""
    vals = np.array([pb.uniform(w, k) for w in range(1 << 16)])
    m = 2 * k + 1
    for x in range(-k, k + 1):
        lo = -(-(65536 * (x + k)) // m)
        hi = -(-(65536 * (x + k + 1)) // m)
        assert int((vals == x).sum()) == hi - lo
    assert vals.min() == -k and vals.max() == k


def test_table1_registry_and_support(pb, orc):
    """Table 1's (n, q, sigma, k, eta) rows; K is the largest support whose 15-bit table is
    strictly increasing (every support value keeps probability), so K + 1 is not."""
    rows = {512: (3329, 2.3, 3), 1024: (12289, 2.3, 3), 2048: (12289, 2.3, 3), 4096: (12289, 1.7, 3),
            8192: (65537, 1.2, 2), 16384: (65537, 1.2, 2), 32768: (65537, 1.0, 2)}
    for n, (q, sigma, k) in rows.items():
        p = pb.params_for(n)
        assert (p.q, p.sigma, p.k, p.eta) == (q, sigma, k, 3)
        T = orc.cdf_table(p.K, p.sigma)
        assert np.all(np.diff(T.astype(int)) > 0)
        with pytest.raises(ValueError):
            orc.cdf_table(p.K + 1, p.sigma)
    assert {pb.params_for(n).K for n in (512, 4096, 8192, 32768)} == {10, 7, 5, 4}


def _A_numpy(orc, p, seedA):
    """A[i][j] = (keystream word j n + i) mod q from the AES-128-CTR words (pinned to OpenSSL)."""
    w = orc.ctr_words(seedA, 0, 0, p.n * p.n).astype(np.int64)
    return (w.reshape(p.n, p.n).T % p.q)  # [i][j]


@pytest.mark.parametrize("q,sigma,k", [(3329, 2.3, 3), (12289, 1.7, 3), (65537, 1.0, 2)])
def test_products_brute_force(pb, orc, q, sigma, k):
    n = 64
    p = pb.custom(n, q, sigma, k)
    g = lwe_inputs.rng(0, 310 + q)
    seedA, seedSK, _ = lwe_inputs.keygen_seeds(g, 1)
    seedA, seedSK = seedA[0].tobytes(), seedSK[0].tobytes()
    A = _A_numpy(orc, p, seedA)
    assert np.array_equal(pb.expand_A_cols(p, seedA, 0, n).T.astype(np.int64), A)
    s, t = pb.pke_keygen(p, seedA, seedSK)
    s_ref = pb.noise(p, seedSK, 1, pb.BINOMIAL, n).astype(np.int64)
    e_ref = pb.noise(p, seedSK, 2, pb.GAUSSIAN, n).astype(np.int64)
    assert np.array_equal(s.astype(np.int64), s_ref)
    assert np.array_equal(t.astype(np.int64), (A @ s_ref + e_ref) % q)
    coins = lwe_inputs.coins(g, 1)[0].tobytes()
    mu = lwe_inputs.messages(g, 1, 32)[0].tobytes()
    U, v = pb.pke_encrypt(p, seedA, t, coins, mu)
    R = pb.noise(p, coins, 1, pb.GAUSSIAN, 256 * n).astype(np.int64).reshape(256, n)
    E1 = pb.noise(p, coins, 2, pb.GAUSSIAN, 256 * n).astype(np.int64).reshape(256, n)
    e2 = pb.noise(p, coins, 3, pb.UNIFORM, 256).astype(np.int64)
    bits = np.unpackbits(np.frombuffer(mu, np.uint8), bitorder="little").astype(np.int64)
    assert np.array_equal(U.astype(np.int64), (R @ A + E1) % q)
    assert np.array_equal(v.astype(np.int64), (R @ t.astype(np.int64) + e2 + bits * ((q + 1) // 2)) % q)
    # decryption recovers the message (noise far below q/4 at this n)
    assert pb.pke_decrypt(p, s, U, v) == mu
    # single entries
    for (r, j) in ((0, 0), (255, n - 1), (17, 33)):
        assert pb.u_entry(p, seedA, coins, r, j) == U[r, j]
    for i in (0, n - 1, 29):
        assert pb.t_entry(p, seedA, seedSK, i) == t[i]


@pytest.mark.parametrize("q", [3329, 12289, 65537])
def test_decode_exhaustive(pb, q):
    """Alg. 3: 0 when x <= q/4 or x >= 3q/4, else 1, over every x in [0, q)."""
    got = np.array([pb.decode(q, x) for x in range(q)])
    want = np.array([0 if (Fraction(x) <= Fraction(q, 4) or Fraction(x) >= Fraction(3 * q, 4)) else 1
                     for x in range(q)])
    assert np.array_equal(got, want)
    # an encoded bit with noise strictly inside (-q/4, q/4) decodes back
    half = (q + 1) // 2
    for noise in (-(q // 4) + 1, 0, q // 4 - 1):
        assert pb.decode(q, (half + noise) % q) == 1
        assert pb.decode(q, noise % q) == 0


@pytest.mark.parametrize("n,reps", [(512, 12), (1024, 3)])
def test_kem_invariant_and_rejection(pb, n, reps):
    p = pb.params_for(n)
    g = lwe_inputs.rng(0, 320 + n)
    for rep in range(reps):
        seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
        pk, sk = pb.kem_keygen(p, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())
        assert len(pk) == p.pk_bytes and len(sk) == p.sk_bytes
        assert sk[2 * n + p.pk_bytes:2 * n + p.pk_bytes + 32] == H(pk)
        mu = lwe_inputs.messages(g, 1, 32)[0].tobytes()
        ct, ss = pb.kem_encaps(p, pk, mu)
        assert len(ct) == p.ct_bytes
        ss2, ok = pb.kem_decaps(p, sk, ct)
        assert ok and ss2 == ss
        coins = H(b"\x01" + H(pk) + mu)[:16]
        assert pb.noise_max(p, seedSK[0].tobytes(), coins) * 4 < p.q
        if rep == 0:
            bad = bytearray(ct)
            bad[5] ^= 1
            ss3, ok3 = pb.kem_decaps(p, sk, bytes(bad))
            assert not ok3 and ss3 == H(z[0].tobytes() + H(bytes(bad)))
