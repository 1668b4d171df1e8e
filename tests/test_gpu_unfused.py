"""GPU parity of the unfused variant (tuning a_source = 1): A is expanded once per call into
device memory and the product kernels read it back instead of regenerating it.  The outputs
must be byte-identical to the oracle's, exactly as for the fused path (integer arithmetic,
tolerance 0), on the streaming product (plain encryption, single key generation, Alg. 1 and
2), the strip product (batched encryption, and decapsulation's re-encryption in compare mode,
Alg. 5), and a key-generation batch (which stays fused: every instance has its own A)."""
import sys

import numpy as np
import pytest

import lwe_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(orc, n):
    import paper_2606_01211_amd as lib

    if n == 200:
        pid = lib.register_params(200, 16, 2, 6, 1.4)
        return lib.params(pid), orc.Params(200, 16, 2, 6, 1.4)
    return lib.params(lib.param_id(n)), orc.params_for(n)


@pytest.fixture(scope="module")
def uctx(orc):
    import paper_2606_01211_amd as lib

    c = lib.Context(0)
    for n in (200, 640, 976, 1344, 8192):
        lp, _ = _pair(orc, n)
        c.set_tuning(lp.pid, a_source=1)
    assert c.get_tuning(lib.param_id(1344))["a_source"] == 1
    yield c
    c.close()


def _keypair(orc, op, g):
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    return orc.kem_keygen(op, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())


def _expand_launches(c):
    prof = c.prof_read()
    return prof.get("expand_A", (0, 0.0))[0]


@pytest.mark.parametrize("n", [200, 640, 976, 1344])
@pytest.mark.parametrize("count", [1, 33, 300])
def test_unfused_encrypt(uctx, orc, n, count):
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(4, 100 + n + count)
    pk, _ = _keypair(orc, op, g)
    coins = lwe_inputs.coins(g, count)
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    say("unfused encrypt", n, count)
    uctx.prof_reset()
    uctx.prof_enable(True)
    uctx.test_encrypt(lp.pid, count, pk, coins, mus, ct)
    launches = _expand_launches(uctx)
    uctx.prof_enable(False)
    assert launches == 1  # the unfused variant really ran
    Bt = np.frombuffer(pk[16:], "<u2").reshape(8, n)
    for i in sorted(set([0, count - 1, count // 2])):
        Bp, V = orc.pke_encrypt(op, pk[:16], Bt, coins[i].tobytes(), mus[i].tobytes())
        assert ct[i].tobytes() == Bp.astype("<u2").tobytes() + V.astype("<u2").tobytes(), i


@pytest.mark.parametrize("n", [200, 1344])
@pytest.mark.parametrize("count", [1, 3])
def test_unfused_keygen(uctx, orc, n, count):
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(4, 200 + n + count)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, count)
    pk = np.zeros((count, op.pk_bytes), np.uint8)
    sk = np.zeros((count, op.sk_bytes), np.uint8)
    say("unfused keygen", n, count)
    uctx.prof_reset()
    uctx.prof_enable(True)
    uctx.keygen_batch(lp.pid, count, seedA, seedSK, z, pk, sk)
    launches = _expand_launches(uctx)
    uctx.prof_enable(False)
    assert launches == (1 if count == 1 else 0)
    for i in range(count):
        opk, osk = orc.kem_keygen(op, seedA[i].tobytes(), seedSK[i].tobytes(), z[i].tobytes())
        assert pk[i].tobytes() == opk, i
        assert sk[i].tobytes() == osk, i


@pytest.mark.parametrize("n", [640, 1344])
def test_unfused_encaps_decaps(uctx, orc, n):
    """Batched encaps against the oracle, then decaps (strip kernel in compare mode) of the
    oracle's ciphertexts, every other one tampered."""
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(4, 300 + n)
    pk, sk = _keypair(orc, op, g)
    count = 300
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("unfused encaps", n, count)
    uctx.encaps_batch(lp.pid, count, pk, mus, ct, ss)
    octs = []
    for i in (0, 150, 299):
        oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
        assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, i
        octs.append(oct_)
    nd = 64
    dec_in = np.zeros((nd, op.ct_bytes), np.uint8)
    for k in range(nd):
        c = bytearray(octs[k % 3])
        if k % 2:
            c[(k * 131) % op.ct_bytes] ^= 1 << (k % 8)
        dec_in[k] = np.frombuffer(bytes(c), np.uint8)
    ss2 = np.zeros((nd, 32), np.uint8)
    say("unfused decaps", n, nd)
    uctx.decaps_batch(lp.pid, nd, sk, dec_in, ss2)
    for k in range(nd):
        oss, ok = orc.kem_decaps(op, sk, dec_in[k].tobytes())
        assert ok == (k % 2 == 0), k
        assert ss2[k].tobytes() == oss, k
    ss3 = np.zeros((count, 32), np.uint8)
    uctx.decaps_batch(lp.pid, count, sk, ct, ss3)
    assert np.array_equal(ss3, ss)


def test_unfused_large_8192(uctx, orc):
    """One KEM at n = 8192 with A (128 MiB) expanded once per call."""
    lp, op = _pair(orc, 8192)
    g = lwe_inputs.rng(4, 8192)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    pk = np.zeros(op.pk_bytes, np.uint8)
    sk = np.zeros(op.sk_bytes, np.uint8)
    say("unfused large keygen 8192")
    uctx.keygen(lp.pid, seedA[0], seedSK[0], z[0], pk, sk)
    opk, osk = orc.kem_keygen(op, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())
    assert pk.tobytes() == opk and sk.tobytes() == osk
    mu = lwe_inputs.messages(g, 1, op.mu_bytes)[0]
    ct = np.zeros(op.ct_bytes, np.uint8)
    ss = np.zeros(32, np.uint8)
    say("unfused large encaps 8192")
    uctx.encaps(lp.pid, pk, mu, ct, ss)
    oct_, oss = orc.kem_encaps(op, opk, mu.tobytes())
    assert ct.tobytes() == oct_ and ss.tobytes() == oss
    ss2 = np.zeros(32, np.uint8)
    uctx.decaps(lp.pid, sk, ct, ss2)
    assert np.array_equal(ss2, ss)


def test_unfused_set_tuning_checks(uctx, orc):
    import paper_2606_01211_amd as lib

    lp, _ = _pair(orc, 640)
    with pytest.raises(lib.LweError) as e:
        uctx.set_tuning(lp.pid, a_source=2)
    assert e.value.status == lib.lwe.LWE_EINVAL
    uctx.set_tuning(lp.pid, a_source=1)
