"""GPU parity of the paper's own parameter sets (Table 1) through the C ABI: one encryption
per message bit (256 rows u_r and values v_r per ciphertext), prime q, s binomial (eta = 3),
e / r / e1 Gaussian through the CDF table, e2 uniform on [-k, k], all noise from the
AES-256 CTR_DRBG, decoding by Alg. 3's thresholds.

* n = 512 .. 4096 (q = 3329, 12289): KeyGen, Encaps and Decaps records byte-equal to the
  oracle's, for batches of one to three instances (768 rows of the product), and implicit
  rejection of tampered ciphertexts equal to the oracle's.
* n = 8192, 16384, 32768 (q = 65537, 4-byte coefficients, split contraction): sampled entries
  of t and u_r from the oracle's single-entry definitions, every v_r from the oracle's
  noise streams, the secret key's s and H(pk), the FO layer recomputed with hashlib, and the
  KEM invariant including rejection.
Integer outputs: tolerance 0.
"""
import hashlib
import sys

import numpy as np
import pytest

import lwe_inputs

pytestmark = pytest.mark.gpu
H = lambda b: hashlib.sha3_256(b).digest()  # noqa: E731


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pb(orc):
    import oracle.pb as m

    return m


def L():
    import paper_2606_01211_amd as mod

    return mod


def test_paper_registry(pb):
    lib = L()
    for n in pb.TABLE1_N:
        p = lib.params(lib.param_id_paper(n))
        o = pb.params_for(n)
        assert (p.paper, p.n, p.q, p.K, p.eta, p.k, p.nbar, p.mbar, p.B) == (1, n, o.q, o.K, 3, o.k, 1, 256, 1)
        assert (p.pk_bytes, p.sk_bytes, p.ct_bytes, p.mu_bytes, p.coef_bytes) == (
            o.pk_bytes, o.sk_bytes, o.ct_bytes, 32, o.coef_bytes)
        assert abs(p.sigma - o.sigma) < 1e-12
        assert np.array_equal(lib.cdf_table(p.pid), np.asarray(__import__("oracle").cdf_table(o.K, o.sigma)))
    # the matrix-form id of an n that both families use stays the matrix-form set
    assert lib.params(lib.param_id(4096)).paper == 0


@pytest.mark.parametrize("n,count", [(512, 1), (512, 3), (1024, 2), (2048, 1), (4096, 1), (4096, 2)])
def test_paper_kem_full(ctx, pb, n, count):
    lib = L()
    pid = lib.param_id_paper(n)
    p = lib.params(pid)
    o = pb.params_for(n)
    g = lwe_inputs.rng(0, 7000 + n + count)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, count)
    say("paper keygen n=%d count=%d" % (n, count))
    pk = np.zeros((count, p.pk_bytes), np.uint8)
    sk = np.zeros((count, p.sk_bytes), np.uint8)
    ctx.keygen_batch(pid, count, seedA, seedSK, z, pk, sk)
    for i in range(count):
        opk, osk = pb.kem_keygen(o, seedA[i].tobytes(), seedSK[i].tobytes(), z[i].tobytes())
        assert pk[i].tobytes() == opk, ("pk", i)
        assert sk[i].tobytes() == osk, ("sk", i)
    say("paper encaps n=%d count=%d" % (n, count))
    mu = lwe_inputs.messages(g, count, 32)
    ct = np.zeros((count, p.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    ctx.encaps_batch(pid, count, pk[0], mu, ct, ss)
    for i in range(count):
        oct_, oss = pb.kem_encaps(o, pk[0].tobytes(), mu[i].tobytes())
        assert ct[i].tobytes() == oct_, ("ct", i)
        assert ss[i].tobytes() == oss, ("ss", i)
    say("paper decaps n=%d count=%d" % (n, count))
    bad = ct.copy()
    bad[count - 1, 3 * p.coef_bytes] ^= 1                 # a coefficient of u_0
    bad[0, p.ct_bytes - p.coef_bytes] ^= 2                 # v_255
    for cts, tampered in ((ct, False), (bad, True)):
        ss2 = np.zeros((count, 32), np.uint8)
        ctx.decaps_batch(pid, count, sk[0], cts, ss2)
        for i in range(count):
            if not tampered:
                assert ss2[i].tobytes() == ss[i].tobytes(), ("decaps", i)
            elif i in (0, count - 1):
                oss2, ok = pb.kem_decaps(o, sk[0].tobytes(), cts[i].tobytes())
                assert not ok and ss2[i].tobytes() == oss2 == H(z[0].tobytes() + H(cts[i].tobytes()))


@pytest.mark.parametrize("n", [8192, 16384, 32768])
def test_paper_kem_sampled(ctx, pb, n):
    import torch

    lib = L()
    pid = lib.param_id_paper(n)
    p = lib.params(pid)
    o = pb.params_for(n)
    dev = torch.device("cuda:0")
    g = lwe_inputs.rng(0, 7100 + n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    sA, sS, zz = seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes()
    say("paper keygen n=%d (device tensors)" % n)
    pk = torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev)
    sk = torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev)
    ctx.keygen(pid, seedA[0], seedSK[0], z[0], pk, sk)
    torch.cuda.synchronize()
    hpk, hsk = pk.cpu().numpy().tobytes(), sk.cpu().numpy().tobytes()
    cb = p.coef_bytes
    t = np.frombuffer(hpk[16:], "<u4" if cb == 4 else "<u2").astype(np.int64)
    assert hpk[:16] == sA
    s_ref = pb.noise(o, sS, 1, pb.BINOMIAL, n)
    assert np.array_equal(np.frombuffer(hsk[:2 * n], "<i2"), s_ref)
    assert hsk[2 * n:2 * n + p.pk_bytes] == hpk
    assert hsk[2 * n + p.pk_bytes:2 * n + p.pk_bytes + 32] == H(hpk)
    assert hsk[-32:] == zz
    for i in (0, 1, n // 2 + 3, n - 1):
        assert t[i] == pb.t_entry(o, sA, sS, i), ("t", i)
    say("paper encaps n=%d" % n)
    mu = lwe_inputs.messages(g, 1, 32)[0]
    ct = torch.empty(p.ct_bytes, dtype=torch.uint8, device=dev)
    ss = torch.empty(32, dtype=torch.uint8, device=dev)
    ctx.encaps(pid, pk, torch.from_numpy(mu).to(dev), ct, ss)
    torch.cuda.synchronize()
    hct, hss = ct.cpu().numpy().tobytes(), ss.cpu().numpy().tobytes()
    coef = np.frombuffer(hct, "<u4" if cb == 4 else "<u2").astype(np.int64)
    U, v = coef[:256 * n].reshape(256, n), coef[256 * n:]
    pkh = H(hpk)
    coins = H(b"\x01" + pkh + mu.tobytes())[:16]
    assert hss == H(H(pkh + mu.tobytes()) + H(hct))
    for (r, j) in ((0, 0), (1, n - 1), (255, 5), (128, n // 3)):
        assert U[r, j] == pb.u_entry(o, sA, coins, r, j), ("u", r, j)
    R = pb.noise(o, coins, 1, pb.GAUSSIAN, 256 * n).astype(np.int64).reshape(256, n)
    e2 = pb.noise(o, coins, 3, pb.UNIFORM, 256).astype(np.int64)
    bits = np.unpackbits(mu, bitorder="little").astype(np.int64)
    assert np.array_equal(v, (R @ t + e2 + bits * ((o.q + 1) // 2)) % o.q)
    assert U.max() < o.q and v.max() < o.q
    say("paper decaps n=%d" % n)
    ss2 = torch.empty(32, dtype=torch.uint8, device=dev)
    ctx.decaps(pid, sk, ct, ss2)
    torch.cuda.synchronize()
    assert ss2.cpu().numpy().tobytes() == hss
    ct[17] ^= 1
    ctx.decaps(pid, sk, ct, ss2)
    torch.cuda.synchronize()
    assert ss2.cpu().numpy().tobytes() == H(zz + H(ct.cpu().numpy().tobytes()))


def test_paper_hooks_refuse(ctx):
    lib = L()
    pid = lib.param_id_paper(512)
    with pytest.raises(lib.LweError) as e:
        ctx.test_sample(pid, bytes(16), 1, 0, 8, np.zeros(8, np.int16))
    assert e.value.status == lib.lwe.LWE_EUNSUPPORTED
