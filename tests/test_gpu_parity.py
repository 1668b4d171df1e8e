"""GPU parity: every stage of the HIP path against the CPU oracle, bit-exact (tolerance 0:
all arithmetic is integer).  Calls go through the C ABI (liblwe_hip.so via ctypes).

Sizes: the registry sets n = 640 (q = 2^15), 976 (ragged contraction tail: 976 = 15*64 + 16),
1344, a custom n = 200 (n = 8 mod 16: half-filled fragments), 8192 in full and 32768 at
sampled outputs; batch sizes cross the host/device hashing threshold (16) and the
streaming/strip product threshold (32 instances)."""
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


def L():
    import paper_2606_01211_amd as mod

    return mod


def _pair(orc, n):
    """(library params, oracle params) for registry n or the custom n = 200 set."""
    lib = L()
    if n == 200:
        pid = lib.register_params(200, 16, 2, 6, 1.4)
        return lib.params(pid), orc.Params(200, 16, 2, 6, 1.4)
    return lib.params(lib.param_id(n)), orc.params_for(n)


def test_keystream(ctx, orc):
    g = lwe_inputs.rng(0, 1000)
    for domain, block0, nb in [(0, 0, 4096), (1, 7, 333), (3, 2**32 - 5, 64), (2, 2**40 + 3, 17)]:
        say("keystream", domain, block0, nb)
        key = lwe_inputs.random_bytes(g, 1, 16)[0].tobytes()
        out = np.zeros(16 * nb, np.uint8)
        ctx.test_keystream(key, domain, block0, nb, out)
        assert out.tobytes() == orc.ctr_blocks(key, domain, block0, nb)


@pytest.mark.parametrize("n", [200, 640, 976, 1344])
def test_expand_A_full(ctx, orc, n):
    lp, op = _pair(orc, n)
    seedA = lwe_inputs.random_bytes(lwe_inputs.rng(0, 1100 + n), 1, 16)[0].tobytes()
    say("expand_A", n)
    out = np.zeros((n, n), np.uint16)
    ctx.test_expand_A(lp.pid, seedA, 0, n, out)
    assert np.array_equal(out, orc.expand_A_cols(op, seedA, 0, n))


def test_expand_A_sampled_32768(ctx, orc):
    lp, op = _pair(orc, 32768)
    seedA = bytes(range(3, 19))
    for col0, nc in [(0, 2), (16383, 3), (32766, 2)]:
        say("expand_A 32768", col0, nc)
        out = np.zeros((nc, 32768), np.uint16)
        ctx.test_expand_A(lp.pid, seedA, col0, nc, out)
        assert np.array_equal(out, orc.expand_A_cols(op, seedA, col0, nc))


@pytest.mark.parametrize("n", [200, 640, 976, 1344])
def test_sampler(ctx, orc, n):
    lp, op = _pair(orc, n)
    key = lwe_inputs.random_bytes(lwe_inputs.rng(0, 1200 + n), 1, 16)[0].tobytes()
    for domain, word0, cnt in [(1, 0, 8 * n), (2, 5, 3001), (3, 0, 64)]:
        say("sample", n, domain, word0, cnt)
        out = np.zeros(cnt, np.int16)
        ctx.test_sample(lp.pid, key, domain, word0, cnt, out)
        assert np.array_equal(out, orc.sample_stream(op, key, domain, word0, cnt))


@pytest.mark.parametrize("lanes", [2, 1])
@pytest.mark.parametrize("cnt", [5, 70])
@pytest.mark.parametrize("length", [0, 1, 135, 136, 137, 1000, 21632])
def test_device_sha3(ctx, length, cnt, lanes):
    """The batched SHA3-256 kernel in both layouts (two lanes per record, one record per
    thread); lengths around the rate, unaligned records, and 70 records (a ragged second
    wave for the one-per-thread layout)."""
    g = lwe_inputs.rng(0, 1300 + length + cnt)
    data = lwe_inputs.random_bytes(g, cnt, max(1, length))[:, :length].copy()
    out = np.zeros((cnt, 32), np.uint8)
    say("sha3", length, cnt, lanes)
    ctx.set_hash_lanes(lanes)
    try:
        ctx.test_sha3(cnt, length, data, out)
    finally:
        ctx.set_hash_lanes(2)
    for i in range(cnt):
        assert out[i].tobytes() == H(data[i].tobytes())


def _keypair(orc, op, g):
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    pk, sk = orc.kem_keygen(op, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())
    return pk, sk


@pytest.mark.parametrize("n", [200, 640, 976, 1344])
@pytest.mark.parametrize("count", [1, 3, 33, 40, 300])
def test_encrypt(ctx, orc, n, count):
    """B' = S'A + E' and V = S'B + E'' + enc(mu) (Alg. 2) for explicit coins; counts from 32
    take the strip (batched) product kernel, smaller ones the streaming one.  33 instances are
    264 rows: the last row block and the last row chunk of the strip kernel are ragged."""
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(0, 1400 + n + count)
    pk, _ = _keypair(orc, op, g)
    coins = lwe_inputs.coins(g, count)
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    say("encrypt", n, count)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ctx.test_encrypt(lp.pid, count, pk, coins, mus, ct)
    Bt = np.frombuffer(pk[16:], "<u2").reshape(8, n)
    for i in sorted(set([0, count - 1, count // 2, count // 3])):
        Bp, V = orc.pke_encrypt(op, pk[:16], Bt, coins[i].tobytes(), mus[i].tobytes())
        assert ct[i].tobytes() == Bp.astype("<u2").tobytes() + V.astype("<u2").tobytes(), i


@pytest.mark.parametrize("n", [200, 640, 976, 1344])
def test_decrypt(ctx, orc, n):
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(0, 1500 + n)
    pk, sk = _keypair(orc, op, g)
    count = 7
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    cts = np.stack([np.frombuffer(orc.kem_encaps(op, pk, mus[i].tobytes())[0], np.uint8) for i in range(count)])
    out = np.zeros((count, op.mu_bytes), np.uint8)
    say("decrypt", n)
    ctx.test_decrypt(lp.pid, count, sk, cts, out)
    assert np.array_equal(out, mus)


@pytest.mark.parametrize("n", [200, 640, 976, 1344, 4096])
@pytest.mark.parametrize("count", [1, 4])
def test_keygen(ctx, orc, n, count):
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(0, 1600 + n + count)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, count)
    pk = np.zeros((count, op.pk_bytes), np.uint8)
    sk = np.zeros((count, op.sk_bytes), np.uint8)
    say("keygen", n, count)
    ctx.keygen_batch(lp.pid, count, seedA, seedSK, z, pk, sk)
    for i in range(count):
        opk, osk = orc.kem_keygen(op, seedA[i].tobytes(), seedSK[i].tobytes(), z[i].tobytes())
        assert pk[i].tobytes() == opk, i
        assert sk[i].tobytes() == osk, i


@pytest.mark.parametrize("n", [200, 640, 976, 1344])
@pytest.mark.parametrize("count", [1, 20, 300])
def test_encaps_decaps(ctx, orc, n, count):
    """Encaps (Alg. 4) and Decaps (Alg. 5) against the oracle.  Decaps gets ciphertexts made
    by the oracle, a quarter of them tampered (implicit rejection)."""
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(0, 1700 + n + count)
    pk, sk = _keypair(orc, op, g)
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("encaps", n, count)
    ctx.encaps_batch(lp.pid, count, pk, mus, ct, ss)
    check = sorted(set([0, count - 1, count // 2, count // 5]))
    oracle_ct = {}
    for i in check:
        oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
        oracle_ct[i] = (oct_, oss)
        assert ct[i].tobytes() == oct_, i
        assert ss[i].tobytes() == oss, i
    # decapsulation inputs: the oracle's ciphertexts, every other one tampered; 5 of them take
    # the host-hashing path, 20 the device-hashing path
    base = [oracle_ct[i][0] for i in check]
    for nd in (5, 20):
        dec_in = np.zeros((nd, op.ct_bytes), np.uint8)
        for k in range(nd):
            c = bytearray(base[k % len(base)])
            if k % 2 == 1:
                c[(k * 97) % op.ct_bytes] ^= 1 << (k % 8)
            dec_in[k] = np.frombuffer(bytes(c), np.uint8)
        ss2 = np.zeros((nd, 32), np.uint8)
        say("decaps", n, nd)
        ctx.decaps_batch(lp.pid, nd, sk, dec_in, ss2)
        for k in range(nd):
            oss, ok = orc.kem_decaps(op, sk, dec_in[k].tobytes())
            assert ok == (k % 2 == 0)
            assert ss2[k].tobytes() == oss, (nd, k)
    # the full batch round-trips on the device (KEM invariant, no oracle involved)
    ss3 = np.zeros((count, 32), np.uint8)
    ctx.decaps_batch(lp.pid, count, sk, ct, ss3)
    assert np.array_equal(ss3, ss)


def test_device_tensors_async(ctx, orc):
    """Device-resident buffers on a torch stream: the same bytes as the host path."""
    import torch

    lp, op = _pair(orc, 1344)
    g = lwe_inputs.rng(0, 1800)
    pk, sk = _keypair(orc, op, g)
    count = 64
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    dev = torch.device("cuda:0")
    d_pk = torch.from_numpy(np.frombuffer(pk, np.uint8).copy()).to(dev)
    d_sk = torch.from_numpy(np.frombuffer(sk, np.uint8).copy()).to(dev)
    d_mu = torch.from_numpy(mus).to(dev)
    d_ct = torch.empty((count, op.ct_bytes), dtype=torch.uint8, device=dev)
    d_ss = torch.empty((count, 32), dtype=torch.uint8, device=dev)
    d_ss2 = torch.empty((count, 32), dtype=torch.uint8, device=dev)
    say("device tensors encaps/decaps")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.encaps_batch(lp.pid, count, d_pk, d_mu, d_ct, d_ss)
        ctx.decaps_batch(lp.pid, count, d_sk, d_ct, d_ss2)
    s.synchronize()
    ct = d_ct.cpu().numpy()
    ss = d_ss.cpu().numpy()
    assert np.array_equal(ss, d_ss2.cpu().numpy())
    for i in [0, 31, 63]:
        oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
        assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss


def test_batch_equals_single(ctx, orc):
    """Instance i of a batch is byte-identical to the same instance run alone."""
    lp, op = _pair(orc, 1344)
    g = lwe_inputs.rng(0, 1900)
    pk, sk = _keypair(orc, op, g)
    count = 257
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("batch vs single")
    ctx.encaps_batch(lp.pid, count, pk, mus, ct, ss)
    for i in [0, 100, 256]:
        c1 = np.zeros(op.ct_bytes, np.uint8)
        s1 = np.zeros(32, np.uint8)
        ctx.encaps(lp.pid, pk, mus[i], c1, s1)
        assert np.array_equal(c1, ct[i]) and np.array_equal(s1, ss[i])


@pytest.mark.parametrize("n", [8192])
def test_large_n_full(ctx, orc, n):
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(2, n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    pk = np.zeros(op.pk_bytes, np.uint8)
    sk = np.zeros(op.sk_bytes, np.uint8)
    say("large keygen", n)
    ctx.keygen(lp.pid, seedA[0], seedSK[0], z[0], pk, sk)
    opk, osk = orc.kem_keygen(op, seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes())
    assert pk.tobytes() == opk and sk.tobytes() == osk
    mu = lwe_inputs.messages(g, 1, op.mu_bytes)[0]
    ct = np.zeros(op.ct_bytes, np.uint8)
    ss = np.zeros(32, np.uint8)
    say("large encaps", n)
    ctx.encaps(lp.pid, pk, mu, ct, ss)
    oct_, oss = orc.kem_encaps(op, opk, mu.tobytes())
    assert ct.tobytes() == oct_ and ss.tobytes() == oss
    ss2 = np.zeros(32, np.uint8)
    say("large decaps", n)
    ctx.decaps(lp.pid, sk, ct, ss2)
    assert np.array_equal(ss2, ss)


@pytest.mark.parametrize("n", [16384, 32768])
def test_large_n_sampled(ctx, orc, n):
    """At n = 16384 and 32768: sampled entries of B^T against the oracle, the secret key in
    full, encryption with explicit coins under a public key built from seeded inputs (B' at
    sampled entries, V in full), and the KEM invariant on the device."""
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(2, n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    sA, sS, zz = seedA[0].tobytes(), seedSK[0].tobytes(), z[0].tobytes()
    pk = np.zeros(op.pk_bytes, np.uint8)
    sk = np.zeros(op.sk_bytes, np.uint8)
    say("sampled keygen", n)
    ctx.keygen(lp.pid, seedA[0], seedSK[0], z[0], pk, sk)
    Bt = np.frombuffer(pk.tobytes()[16:], "<u2").reshape(8, n)
    assert pk.tobytes()[:16] == sA
    for c, i in [(0, 0), (7, n - 1), (3, n // 2 + 5), (5, 12345 % n)]:
        assert Bt[c, i] == orc.Bt_entry(op, sA, sS, c, i), (c, i)
    St = np.frombuffer(sk.tobytes()[:16 * n], "<i2").reshape(8, n)
    assert np.array_equal(St.reshape(-1), orc.sample_stream(op, sS, 1, 0, 8 * n))
    skb = sk.tobytes()
    assert skb[16 * n:16 * n + op.pk_bytes] == pk.tobytes()
    assert skb[16 * n + op.pk_bytes:16 * n + op.pk_bytes + 32] == H(pk.tobytes()) and skb[-32:] == zz
    # encryption with explicit coins under pk' = seedA || (seeded uniform B^T)
    Bt_syn = (lwe_inputs.random_bytes(g, 8, 2 * n).view("<u2") & (op.q - 1)).astype("<u2")
    pk_syn = sA + Bt_syn.tobytes()
    coins = lwe_inputs.coins(g, 1)
    mu = lwe_inputs.messages(g, 1, op.mu_bytes)
    ct = np.zeros(op.ct_bytes, np.uint8)
    say("sampled encrypt", n)
    ctx.test_encrypt(lp.pid, 1, pk_syn, coins, mu, ct)
    Bp = np.frombuffer(ct.tobytes()[:16 * n], "<u2").reshape(8, n)
    for r, j in [(0, 0), (7, n - 1), (2, n // 3), (6, 9999 % n)]:
        assert Bp[r, j] == orc.Bp_entry(op, sA, coins[0].tobytes(), r, j), (r, j)
    V = np.frombuffer(ct.tobytes()[16 * n:], "<u2").reshape(8, 8)
    assert np.array_equal(V, orc.pke_V(op, Bt_syn, coins[0].tobytes(), mu[0].tobytes()))
    # KEM invariant and implicit rejection on the device
    ct2 = np.zeros(op.ct_bytes, np.uint8)
    ss = np.zeros(32, np.uint8)
    ss2 = np.zeros(32, np.uint8)
    say("sampled encaps/decaps", n)
    ctx.encaps(lp.pid, pk, mu[0], ct2, ss)
    ctx.decaps(lp.pid, sk, ct2, ss2)
    assert np.array_equal(ss, ss2)
    bad = ct2.copy()
    bad[5] ^= 4
    ctx.decaps(lp.pid, sk, bad, ss2)
    assert ss2.tobytes() == H(zz + H(bad.tobytes()))


@pytest.mark.parametrize("n", [640, 1344])
def test_decaps_strip_tampered(ctx, orc, n):
    """Decaps of 64 ciphertexts (512 rows: the strip kernel in compare mode) made by the
    oracle, two thirds of them tampered on instances of both parities (two instances share a
    16-row MFMA tile) in rows 0, 3 and 7 of B', in its first and last column, and in V; every
    shared secret equals the oracle's decapsulation (Alg. 5, implicit rejection)."""
    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(0, 1800 + n)
    pk, sk = _keypair(orc, op, g)
    base_mus = lwe_inputs.messages(g, 8, op.mu_bytes)
    base = [orc.kem_encaps(op, pk, base_mus[i].tobytes())[0] for i in range(8)]
    count = 64
    bp = 16 * n  # bytes of B'
    spots = [0, 2 * (n - 1) + 1, 2 * (7 * n), 2 * (7 * n + n - 1) + 1, bp, bp + 127, 2 * (3 * n + n // 2)]
    cts = np.zeros((count, op.ct_bytes), np.uint8)
    tampered = set()
    for k in range(count):
        c = bytearray(base[k % 8])
        if k % 3 != 0:
            c[spots[k % len(spots)]] ^= 1 << (k % 8)
            tampered.add(k)
        cts[k] = np.frombuffer(bytes(c), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("decaps strip tampered", n)
    ctx.decaps_batch(lp.pid, count, sk, cts, ss)
    for k in range(count):
        oss, ok = orc.kem_decaps(op, sk, cts[k].tobytes())
        assert ok == (k not in tampered), k
        assert ss[k].tobytes() == oss, k


def test_argument_checks(ctx, orc):
    """A batch of zero is a no-op; one over the maximum (65535) or an unknown parameter id is
    LWE_EINVAL, returned before any buffer is touched."""
    lib = L()
    EINVAL = lib.lwe.LWE_EINVAL
    lp, op = _pair(orc, 640)
    g = lwe_inputs.rng(0, 1900)
    pk, _ = _keypair(orc, op, g)
    mus = lwe_inputs.messages(g, 1, op.mu_bytes)
    ct = np.zeros((1, op.ct_bytes), np.uint8)
    ss = np.zeros((1, 32), np.uint8)
    ctx.encaps_batch(lp.pid, 0, pk, mus, ct, ss)  # no-op
    assert not ct.any() and not ss.any()
    pkb = np.frombuffer(pk, np.uint8).copy()
    st = ctx._lib.lwe_encaps_batch(ctx._h, lp.pid, 65536, pkb.ctypes.data, mus.ctypes.data, ct.ctypes.data,
                                   ss.ctypes.data, None)
    assert st == EINVAL
    with pytest.raises(lib.LweError) as e:
        lib.params(250)
    assert e.value.status == EINVAL


def test_full_batch_4096_sampled(ctx, orc):
    """The benchmark's batched configuration at full size: 4096 encapsulations at n = 1344 in
    one call (strip product with the tuned tile shape), checked against the oracle at 72
    instances: every 64th instance alternating between the two instances of a 16-row MFMA tile
    (so every row chunk of the strip kernel and both tile parities), both ends and the
    row-chunk boundaries; then all 4096 decapsulated on the device (KEM invariant) and a
    sample of them by the oracle."""
    lp, op = _pair(orc, 1344)
    g = lwe_inputs.rng(0, 4096)
    pk, sk = _keypair(orc, op, g)
    count = 4096
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("full batch encaps 4096")
    ctx.encaps_batch(lp.pid, count, pk, mus, ct, ss)
    picks = sorted(set([64 * k + (k % 2) for k in range(64)] + [0, 1, 511, 512, 2047, 2048, 3071, 4095]))
    assert len(picks) >= 64
    say("oracle on", len(picks), "instances")
    for i in picks:
        oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
        assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, i
    ss2 = np.zeros((count, 32), np.uint8)
    say("full batch decaps 4096")
    ctx.decaps_batch(lp.pid, count, sk, ct, ss2)
    assert np.array_equal(ss2, ss)
    for i in [5, 4094]:
        oss, ok = orc.kem_decaps(op, sk, ct[i].tobytes())
        assert ok and ss2[i].tobytes() == oss


def test_context_stream_lanes(orc):
    """Two contexts driven from device buffers on their own streams (lwe_ctx_stream), as the
    benchmark and the server run their lanes, concurrently: each lane's outputs equal the
    oracle's and do not depend on the other lane running."""
    import torch

    lib = L()
    lp, op = _pair(orc, 640)
    g = lwe_inputs.rng(0, 2100)
    pk, sk = _keypair(orc, op, g)
    count = 96
    dev = torch.device("cuda:0")
    ctxs = [lib.Context(0), lib.Context(0)]
    try:
        handles = [c.stream_handle for c in ctxs]
        assert all(handles) and handles[0] != handles[1]
        streams = [torch.cuda.ExternalStream(h, device=dev) for h in handles]
        d_pk = torch.from_numpy(np.frombuffer(pk, np.uint8).copy()).to(dev)
        d_sk = torch.from_numpy(np.frombuffer(sk, np.uint8).copy()).to(dev)
        mus = [lwe_inputs.messages(g, count, op.mu_bytes) for _ in range(2)]
        d_mus = [torch.from_numpy(m).to(dev) for m in mus]
        outs = [tuple(torch.empty(shape, dtype=torch.uint8, device=dev)
                      for shape in ((count, op.ct_bytes), (count, 32), (count, 32))) for _ in range(2)]
        torch.cuda.synchronize()  # inputs in place before either lane's stream reads them
        for lane in range(2):  # both lanes in flight at once
            d_ct, d_ss, d_ss2 = outs[lane]
            with torch.cuda.stream(streams[lane]):
                ctxs[lane].encaps_batch(lp.pid, count, d_pk, d_mus[lane], d_ct, d_ss)
                ctxs[lane].decaps_batch(lp.pid, count, d_sk, d_ct, d_ss2)
        say("context-stream lanes")
        for s in streams:
            s.synchronize()
        for lane in range(2):
            ct, ss, ss2 = (x.cpu().numpy() for x in outs[lane])
            assert np.array_equal(ss, ss2)
            for i in (0, count - 1):
                oct_, oss = orc.kem_encaps(op, pk, mus[lane][i].tobytes())
                assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, (lane, i)
    finally:
        for c in ctxs:
            c.close()


def test_decaps_side_stream_off_and_on(orc):
    """lwe_ctx_set_side_stream: a batched decapsulation with the ciphertext hash on the call's
    own stream (0) and on the context's second stream (1) gives the oracle's shared secrets,
    for valid and tampered ciphertexts alike, in either order."""
    lib = L()
    lp, op = _pair(orc, 640)
    g = lwe_inputs.rng(0, 2200)
    pk, sk = _keypair(orc, op, g)
    count = 96  # above the host-hash limit: the device hash path
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    c = lib.Context(0)
    try:
        assert c._lib.lwe_ctx_set_side_stream(c._h, 2) == lib.lwe.LWE_EINVAL
        ct = np.zeros((count, op.ct_bytes), np.uint8)
        ss = np.zeros((count, 32), np.uint8)
        c.encaps_batch(lp.pid, count, pk, mus, ct, ss)
        for i in range(1, count, 2):
            ct[i, (i * 37) % op.ct_bytes] ^= 1 << (i % 8)
        want = [orc.kem_decaps(op, sk, ct[i].tobytes()) for i in range(count)]
        for enable in (False, True, False):
            c.set_side_stream(enable)
            say("decaps side stream", enable)
            ss2 = np.zeros((count, 32), np.uint8)
            c.decaps_batch(lp.pid, count, sk, ct, ss2)
            for i in range(count):
                oss, ok = want[i]
                assert ok == (i % 2 == 0), (enable, i)
                assert ss2[i].tobytes() == oss, (enable, i)
            assert np.array_equal(ss2[0::2], ss[0::2])
    finally:
        c.close()


def test_kem_one_lane_hash(orc):
    """A context in the many-contexts configuration (one stream, one record per thread in the
    SHA3 kernels): batched KeyGen (H(pk) on the device), Encaps and Decaps, valid and tampered
    ciphertexts, against the oracle."""
    lib = L()
    lp, op = _pair(orc, 640)
    g = lwe_inputs.rng(0, 2300)
    kc = 20  # above the host-hash limit: device H(pk)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, kc)
    c = lib.Context(0)
    try:
        c.set_side_stream(False)
        c.set_hash_lanes(1)
        pks = np.zeros((kc, op.pk_bytes), np.uint8)
        sks = np.zeros((kc, op.sk_bytes), np.uint8)
        say("one-lane hash keygen", kc)
        c.keygen_batch(lp.pid, kc, seedA, seedSK, z, pks, sks)
        for i in (0, kc - 1):
            opk, osk = orc.kem_keygen(op, seedA[i].tobytes(), seedSK[i].tobytes(), z[i].tobytes())
            assert pks[i].tobytes() == opk and sks[i].tobytes() == osk, i
        pk, sk = pks[0].tobytes(), sks[0].tobytes()
        count = 96
        mus = lwe_inputs.messages(g, count, op.mu_bytes)
        ct = np.zeros((count, op.ct_bytes), np.uint8)
        ss = np.zeros((count, 32), np.uint8)
        say("one-lane hash encaps", count)
        c.encaps_batch(lp.pid, count, pk, mus, ct, ss)
        for i in (0, 47, count - 1):
            oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
            assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, i
        for i in range(1, count, 2):
            ct[i, (i * 53) % op.ct_bytes] ^= 1 << (i % 8)
        ss2 = np.zeros((count, 32), np.uint8)
        say("one-lane hash decaps", count)
        c.decaps_batch(lp.pid, count, sk, ct, ss2)
        for i in range(count):
            oss, ok = orc.kem_decaps(op, sk, ct[i].tobytes())
            assert ok == (i % 2 == 0), i
            assert ss2[i].tobytes() == oss, i
        assert c._lib.lwe_ctx_set_hash_lanes(c._h, 3) == lib.lwe.LWE_EINVAL
    finally:
        c.close()


def test_strip_split_k_8192(ctx, orc):
    """A batch of 32 encryptions at n = 8192: the strip product with its contraction split in
    two K chunks (S' in fragment order, partial sums accumulated and finished by k_finalize),
    against the oracle at both ends of the batch."""
    lp, op = _pair(orc, 8192)
    g = lwe_inputs.rng(0, 8192 + 32)
    pk, _ = _keypair(orc, op, g)
    count = 32
    coins = lwe_inputs.coins(g, count)
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    say("strip split-K 8192", count)
    ctx.test_encrypt(lp.pid, count, pk, coins, mus, ct)
    Bt = np.frombuffer(pk[16:], "<u2").reshape(8, 8192)
    for i in (0, count - 1):
        Bp, V = orc.pke_encrypt(op, pk[:16], Bt, coins[i].tobytes(), mus[i].tobytes())
        assert ct[i].tobytes() == Bp.astype("<u2").tobytes() + V.astype("<u2").tobytes(), i


def test_strip_tables_in_strip_4096(ctx, orc):
    """40 encapsulations at n = 4096 (a key size of the serving mix): the 128 KB strip leaves no
    room for the 64 KB AES table copies beside it, so the strip kernel keeps them in the first
    64 KB of the strip's own space while it regenerates A (the blocks that land there held in
    registers until the lookups are done).  Encryption and the decapsulation's compare mode
    against the oracle, one ciphertext tampered."""
    lp, op = _pair(orc, 4096)
    g = lwe_inputs.rng(0, 4096 + 40)
    pk, sk = _keypair(orc, op, g)
    count = 40
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("strip tables in strip 4096 encaps", count)
    ctx.encaps_batch(lp.pid, count, pk, mus, ct, ss)
    for i in (0, count - 1):
        oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
        assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, i
    bad = ct.copy()
    bad[7, 16 * 4096 + 5] ^= 0x10  # a V coefficient of instance 7
    ss2 = np.zeros((count, 32), np.uint8)
    say("strip tables in strip 4096 decaps", count)
    ctx.decaps_batch(lp.pid, count, sk, bad, ss2)
    for i in range(count):
        if i != 7:
            assert ss2[i].tobytes() == ss[i].tobytes(), i
    oss, ok = orc.kem_decaps(op, sk, bad[7].tobytes())
    assert not ok and ss2[7].tobytes() == oss


@pytest.mark.parametrize("n", [640, 1344])
def test_strip_tile_shapes(ctx, orc, n):
    """Every (column groups, row groups) tile the library builds for the strip product, at two
    row-chunk counts, gives the ciphertexts and shared secrets of the default tile, which are
    checked against the oracle (Alg. 2-5), and the decapsulation's compare mode rejects the
    same tampered ciphertext.  The table copies sit beside the strip (n = 640, and one or two
    column groups at 1344) or inside it (three column groups at 1344); 40 instances make
    ragged row blocks and row chunks."""
    from paper_2606_01211_amd import tune

    lp, op = _pair(orc, n)
    g = lwe_inputs.rng(0, 7100 + n)
    pk, sk = _keypair(orc, op, g)
    count = 40
    mus = lwe_inputs.messages(g, count, op.mu_bytes)
    saved = ctx.get_tuning(lp.pid)
    ct0 = np.zeros((count, op.ct_bytes), np.uint8)
    ss0 = np.zeros((count, 32), np.uint8)
    say("strip shapes: default", n)
    ctx.encaps_batch(lp.pid, count, pk, mus, ct0, ss0)
    for i in (0, count - 1):
        oct_, oss = orc.kem_encaps(op, pk, mus[i].tobytes())
        assert ct0[i].tobytes() == oct_ and ss0[i].tobytes() == oss, i
    bad = ct0.copy()
    bad[5, 2 * n + 3] ^= 0x04  # a B' coefficient of instance 5
    oss5, ok = orc.kem_decaps(op, sk, bad[5].tobytes())
    assert not ok
    try:
        for cg, rg in tune.SHAPES:
            if not tune.lds_fits(cg, n):
                continue
            for mc in (3, 8):
                say("strip shapes", n, cg, rg, mc)
                ctx.set_tuning(lp.pid, col_groups=cg, row_groups=rg, m_chunks=mc)
                ct = np.zeros_like(ct0)
                ss = np.zeros_like(ss0)
                ctx.encaps_batch(lp.pid, count, pk, mus, ct, ss)
                assert np.array_equal(ct, ct0) and np.array_equal(ss, ss0), (cg, rg, mc)
                ss2 = np.zeros_like(ss0)
                ctx.decaps_batch(lp.pid, count, sk, bad, ss2)
                keep = [i for i in range(count) if i != 5]
                assert np.array_equal(ss2[keep], ss0[keep]), (cg, rg, mc)
                assert ss2[5].tobytes() == oss5, (cg, rg, mc)
    finally:
        ctx.set_tuning(lp.pid, **saved)
