"""KEM-level pins of the oracle (Alg. 4-5, Fujisaki-Okamoto with implicit rejection):
the invariant decaps(encaps(pk)) = ss over many seeds, the decoding margin, the FO hash
structure recomputed with hashlib, implicit rejection of tampered ciphertexts, and the
byte formats."""
import hashlib
import os

import numpy as np
import pytest

import lwe_inputs

H = lambda b: hashlib.sha3_256(b).digest()  # noqa: E731
SEEDS = {640: 200, 976: 80, 1344: 60}
if os.environ.get("LWE_SLOW") == "1":
    SEEDS = {640: 1000, 976: 1000, 1344: 1000, 4096: 100}


@pytest.mark.parametrize("n", sorted(SEEDS))
def test_kem_invariant_and_margin(orc, n):
    p = orc.params_for(n)
    g = lwe_inputs.rng(0, 500 + n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    pk, sk = orc.kem_keygen(p, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())
    pkh = H(pk)
    bound = p.q >> (p.B + 1)
    mus = lwe_inputs.messages(g, SEEDS[n], p.mu_bytes)
    for k in range(SEEDS[n]):
        mu = mus[k].tobytes()
        ct, ss = orc.kem_encaps(p, pk, mu)
        ss2, ok = orc.kem_decaps(p, sk, ct)
        assert ok and ss2 == ss
        coins, kp = orc.fo_coins(p, pkh, mu)
        assert orc.noise_max(p, seedSK[0].tobytes(), coins) < bound
        if k < 5:
            assert ss == H(kp + H(ct))


def test_fo_coins_structure(orc):
    p = orc.params_for(1344)
    pkh = bytes(range(32))
    mu = bytes(range(100, 132))
    coins, kp = orc.fo_coins(p, pkh, mu)
    assert coins == H(b"\x01" + pkh + mu)[:16]
    assert kp == H(pkh + mu)


@pytest.mark.parametrize("n", [640, 1344])
def test_implicit_rejection(orc, n):
    p = orc.params_for(n)
    g = lwe_inputs.rng(0, 600 + n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    zb = z[0].tobytes()
    pk, sk = orc.kem_keygen(p, seedA[0].tobytes(), seedSK[0].tobytes(), zb)
    mu = lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes()
    ct, ss = orc.kem_encaps(p, pk, mu)
    for pos in [0, 2 * 8 * n - 1, len(ct) - 1, len(ct) // 2]:
        bad = bytearray(ct)
        bad[pos] ^= 0x01
        bad = bytes(bad)
        ss_bad, ok = orc.kem_decaps(p, sk, bad)
        assert not ok
        assert ss_bad == H(zb + H(bad))
        assert ss_bad != ss


def test_byte_formats(orc):
    p = orc.params_for(640)
    n = p.n
    seedA, seedSK, z = bytes(range(16)), bytes(range(16, 32)), bytes(range(32, 64))
    pk, sk = orc.kem_keygen(p, seedA, seedSK, z)
    assert len(pk) == 10256 and len(sk) == 20560
    St, Bt = orc.pke_keygen(p, seedA, seedSK)
    assert pk[:16] == seedA
    assert np.array_equal(np.frombuffer(pk[16:], "<u2").reshape(8, n), Bt)
    assert np.array_equal(np.frombuffer(sk[:16 * n], "<i2").reshape(8, n), St)
    assert sk[16 * n:16 * n + len(pk)] == pk
    assert sk[16 * n + len(pk):16 * n + len(pk) + 32] == H(pk)
    assert sk[-32:] == z
    mu = bytes(range(200, 216))
    ct, _ = orc.kem_encaps(p, pk, mu)
    assert len(ct) == 10368
    coins, _ = orc.fo_coins(p, H(pk), mu)
    Bp, V = orc.pke_encrypt(p, seedA, Bt, coins, mu)
    assert np.array_equal(np.frombuffer(ct[:16 * n], "<u2").reshape(8, n), Bp)
    assert np.array_equal(np.frombuffer(ct[16 * n:], "<u2").reshape(8, 8), V)


@pytest.mark.parametrize("n", [640, 976, 1344, 16384])
def test_encode_decode_exhaustive(orc, n):
    """decode(enc(k) + e) = k for every k < 2^B and every |e| < q / 2^(B+1)."""
    p = orc.params_for(n)
    q, B = p.q, p.B
    bound = q >> (B + 1)
    step = max(1, bound // 512)
    for k in range(1 << B):
        base = k << (p.logq - B)
        for e in list(range(-bound + 1, bound, step)) + [-bound + 1, bound - 1]:
            assert orc.decode_value(p, (base + e) % q) == k
    # message bit placement: coefficient c carries bits c*B .. c*B+B-1, LSB first
    mu = bytearray(p.mu_bytes)
    mu[0] = 0b10110101
    vals = [orc.encode_coeff(p, bytes(mu), c) >> (p.logq - B) for c in range(8 // B + 1)]
    bits = [(mu[0] >> i) & 1 for i in range(8)]
    for c in range(8 // B):
        assert vals[c] == sum(bits[c * B + t] << t for t in range(B))


@pytest.mark.slow
@pytest.mark.parametrize("n", [8192, 16384])
def test_kem_invariant_large(orc, n):
    p = orc.params_for(n)
    g = lwe_inputs.rng(2, n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    pk, sk = orc.kem_keygen(p, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())
    mu = lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes()
    ct, ss = orc.kem_encaps(p, pk, mu)
    ss2, ok = orc.kem_decaps(p, sk, ct)
    assert ok and ss == ss2
