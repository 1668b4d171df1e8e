"""GPU parity of the pieces that the KEM tests reach only end to end, through the C ABI:

* the batched sampler kernel itself (both operand layouts, KeyGen and Encrypt segments),
  against the oracle's sampler over the same keystream domains (Alg. 1-2);
* the encryption product with injected operands (Alg. 2 without the sampler): unit rows of
  S' with E' = 0 select rows of A, and random S' against numpy products over the oracle's A;
* the randomised entry points (seeds and messages from the operating system), checked by
  the oracle through the KEM invariant (Alg. 4-5);
* one context driven alternately from two streams (calls reuse the context's buffers and
  must execute in call order).

Integer arithmetic throughout: tolerance 0."""
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


def frag_index(rows, ldx):
    """Byte index of element (row, k) of an int8 operand in MFMA fragment order: 16-row
    groups, then 64-column steps, then the 64 lanes of a fragment (lane = row % 16 +
    16 * (k % 64 // 16)), 16 bytes per lane."""
    r = np.arange(rows)[:, None]
    k = np.arange(ldx)[None, :]
    lane = (r % 16) + 16 * ((k % 64) // 16)
    return (((r // 16) * (ldx // 64) + k // 64) * 64 + lane) * 16 + (k % 16)


@pytest.mark.parametrize("n", [976, 1344])
@pytest.mark.parametrize("count", [3, 40])
@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_sample_batch(ctx, orc, n, count, layout, mode):
    """The hot sampler kernel: segment 0 (S^T or S', domain 1) in the requested operand layout
    with zero padding columns, segment 1 (E^T or E', domain 2), E'' (domain 3, Encrypt) and
    the int16 copy of S^T (KeyGen), each equal to the oracle's samples of that domain."""
    lib = L()
    pid = lib.param_id(n)
    op = orc.params_for(n)
    ldx = (n + 63) // 64 * 64
    g = lwe_inputs.rng(0, 5000 + n + count + 10 * layout + 100 * mode)
    keys = lwe_inputs.coins(g, count)
    rows = (count * 8 + 15) // 16 * 16 if layout else count * 8
    X = np.zeros(rows * ldx, np.int8)
    E = np.zeros(count * 8 * n, np.int8)
    E2 = np.zeros(count * 64, np.int8) if mode == 1 else None
    X16 = np.zeros(count * 8 * n, np.int16) if mode == 0 else None
    say("sample_batch", n, count, layout, mode)
    ctx.test_sample_batch(pid, count, mode, layout, keys, X, E, E2, X16)
    if layout:
        Xm = X[frag_index(rows, ldx)]
    else:
        Xm = X.reshape(count * 8, ldx)
    assert not Xm[: count * 8, n:].any()  # zero padding columns
    if layout and rows > count * 8:
        assert np.all(Xm[count * 8:].view(np.uint8) == 0x5A)  # rows the sampler does not own
    E = E.reshape(count * 8, n)
    for i in range(count):
        key = keys[i].tobytes()
        s0 = orc.sample_stream(op, key, 1, 0, 8 * n).reshape(8, n)
        s1 = orc.sample_stream(op, key, 2, 0, 8 * n).reshape(8, n)
        assert np.array_equal(Xm[8 * i:8 * i + 8, :n].astype(np.int16), s0), i
        assert np.array_equal(E[8 * i:8 * i + 8].astype(np.int16), s1), i
        if mode == 1:
            s2 = orc.sample_stream(op, key, 3, 0, 64)
            assert np.array_equal(E2[64 * i:64 * i + 64].astype(np.int16), s2), i
        else:
            assert np.array_equal(X16[8 * n * i:8 * n * (i + 1)], s0.reshape(-1)), i


def _A_rows(orc, op, seedA):
    """A as an n x n int64 array (row i, column j), from the oracle's column expansion."""
    cols = orc.expand_A_cols(op, seedA, 0, op.n)  # cols[j][i] = A[i][j]
    return cols.T.astype(np.int64)


@pytest.mark.parametrize("n,count", [(640, 2), (640, 40), (1344, 3), (1344, 33)])
def test_product_unit_rows(ctx, orc, n, count):
    """S' = unit rows, E' = 0, E'' = 0, mu = 0: row r of B' is row idx_r of A, and V[r][c] is
    B^T[c][idx_r]; both product kernels (counts below 32 stream, from 32 strip)."""
    lib = L()
    pid = lib.param_id(n)
    op = orc.params_for(n)
    g = lwe_inputs.rng(0, 5100 + n + count)
    seedA = lwe_inputs.random_bytes(g, 1, 16)[0].tobytes()
    Bt = (lwe_inputs.random_bytes(g, 8, 2 * n).view("<u2") & (op.q - 1)).astype("<u2")
    M = 8 * count
    idx = (np.arange(M) * 37 + 5) % n
    S = np.zeros((M, n), np.int8)
    S[np.arange(M), idx] = 1
    E = np.zeros((M, n), np.int8)
    E2 = np.zeros((count, 64), np.int8)
    mu = np.zeros((count, op.mu_bytes), np.uint8)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    say("product unit rows", n, count)
    ctx.test_product(pid, count, seedA, Bt, S, E, E2, mu, ct)
    A = _A_rows(orc, op, seedA)
    for i in range(count):
        Bp = np.frombuffer(ct[i, :16 * n].tobytes(), "<u2").reshape(8, n)
        V = np.frombuffer(ct[i, 16 * n:].tobytes(), "<u2").reshape(8, 8)
        for r in range(8):
            row = idx[8 * i + r]
            assert np.array_equal(Bp[r], A[row]), (i, r)
            assert np.array_equal(V[r], Bt[:, row]), (i, r)


@pytest.mark.parametrize("n,count", [(200, 5), (976, 34), (1344, 40)])
def test_product_random(ctx, orc, n, count):
    """Random int8 S' (any value, not only the sampler's support), E', E'' and messages:
    B' = S'A + E' and V = S'B + E'' + enc(mu) mod q against numpy int64 products over the
    oracle's A and the oracle's encoding."""
    lib = L()
    if n == 200:
        pid = lib.register_params(200, 16, 2, 6, 1.4)
        op = orc.Params(200, 16, 2, 6, 1.4)
    else:
        pid = lib.param_id(n)
        op = orc.params_for(n)
    g = lwe_inputs.rng(0, 5200 + n + count)
    seedA = lwe_inputs.random_bytes(g, 1, 16)[0].tobytes()
    Bt = (lwe_inputs.random_bytes(g, 8, 2 * n).view("<u2") & (op.q - 1)).astype("<u2")
    M = 8 * count
    S = lwe_inputs.random_bytes(g, M, n).view(np.int8)
    E = lwe_inputs.random_bytes(g, M, n).view(np.int8)
    E2 = lwe_inputs.random_bytes(g, count, 64).view(np.int8)
    mu = lwe_inputs.messages(g, count, op.mu_bytes)
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    say("product random", n, count)
    ctx.test_product(pid, count, seedA, Bt, S, E, E2, mu, ct)
    A = _A_rows(orc, op, seedA)
    Bmat = Bt.astype(np.int64).T  # n x 8
    Bp_all = (S.astype(np.int64) @ A + E.astype(np.int64)) % op.q
    V_all = S.astype(np.int64) @ Bmat  # M x 8
    for i in range(count):
        Bp = np.frombuffer(ct[i, :16 * n].tobytes(), "<u2").reshape(8, n)
        V = np.frombuffer(ct[i, 16 * n:].tobytes(), "<u2").reshape(8, 8)
        assert np.array_equal(Bp, Bp_all[8 * i:8 * i + 8]), i
        enc = np.array([[orc.encode_coeff(op, mu[i].tobytes(), 8 * r + c) for c in range(8)] for r in range(8)])
        want = (V_all[8 * i:8 * i + 8] + E2[i].astype(np.int64).reshape(8, 8) + enc) % op.q
        assert np.array_equal(V, want), i


def test_rand_entry_points(ctx, orc):
    """KeyGen and Encaps with seeds and messages from the operating system: two key pairs
    differ; each key pair is consistent (E^T = B^T - S^T A^T mod q lies in the error support,
    sk embeds pk, H(pk)); the oracle's encapsulations under the random key decapsulate on the
    device and in the oracle to the same secret; the device's random encapsulations decrypt
    to messages whose oracle encapsulation reproduces ciphertext and secret."""
    lib = L()
    n = 640
    pid = lib.param_id(n)
    op = orc.params_for(n)
    pk = np.zeros((2, op.pk_bytes), np.uint8)
    sk = np.zeros((2, op.sk_bytes), np.uint8)
    say("keygen_rand")
    ctx.keygen_rand(pid, 2, pk, sk)
    assert pk[0].tobytes() != pk[1].tobytes() and sk[0, -32:].tobytes() != sk[1, -32:].tobytes()
    for k in range(2):
        pkb, skb = pk[k].tobytes(), sk[k].tobytes()
        assert skb[16 * n:16 * n + op.pk_bytes] == pkb
        assert skb[16 * n + op.pk_bytes:16 * n + op.pk_bytes + 32] == H(pkb)
        A = _A_rows(orc, op, pkb[:16])
        St = np.frombuffer(skb[:16 * n], "<i2").reshape(8, n).astype(np.int64)
        Bt = np.frombuffer(pkb[16:], "<u2").reshape(8, n).astype(np.int64)
        Et = (Bt - St @ A.T) % op.q
        Et = np.where(Et > op.q // 2, Et - op.q, Et)
        assert np.abs(Et).max() <= op.K and np.abs(St).max() <= op.K
    g = lwe_inputs.rng(0, 5300)
    mus = lwe_inputs.messages(g, 3, op.mu_bytes)
    for i in range(3):
        oct_, oss = orc.kem_encaps(op, pk[0].tobytes(), mus[i].tobytes())
        ss = np.zeros(32, np.uint8)
        ctx.decaps(pid, sk[0], np.frombuffer(oct_, np.uint8), ss)
        assert ss.tobytes() == oss and orc.kem_decaps(op, sk[0].tobytes(), oct_) == (oss, True)
    count = 24  # above the host-hash limit: the device FO path
    ct = np.zeros((count, op.ct_bytes), np.uint8)
    ss = np.zeros((count, 32), np.uint8)
    say("encaps_rand", count)
    ctx.encaps_rand(pid, count, pk[0], ct, ss)
    mu2 = np.zeros((count, op.mu_bytes), np.uint8)
    ctx.test_decrypt(pid, count, sk[0], ct, mu2)
    assert len({m.tobytes() for m in mu2}) == count
    for i in (0, 11, count - 1):
        oct_, oss = orc.kem_encaps(op, pk[0].tobytes(), mu2[i].tobytes())
        assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, i


def test_one_context_two_streams(orc):
    """One context, calls alternating between two torch streams without any synchronisation
    between them: the context orders each call after the previous one, so every result
    equals the oracle's (the calls share the context's buffers)."""
    import torch

    lib = L()
    n = 640
    pid = lib.param_id(n)
    op = orc.params_for(n)
    g = lwe_inputs.rng(0, 5400)
    sa, ssk, z = lwe_inputs.keygen_seeds(g, 1)
    pk, sk = orc.kem_keygen(op, sa[0].tobytes(), ssk[0].tobytes(), z[0].tobytes())
    dev = torch.device("cuda:0")
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    d_pk = torch.from_numpy(np.frombuffer(pk, np.uint8).copy()).to(dev)
    d_sk = torch.from_numpy(np.frombuffer(sk, np.uint8).copy()).to(dev)
    counts = [96, 40, 200, 33, 64, 150]
    mus = [lwe_inputs.messages(g, c, op.mu_bytes) for c in counts]
    d_mus = [torch.from_numpy(m).to(dev) for m in mus]
    outs = [(torch.empty((c, op.ct_bytes), dtype=torch.uint8, device=dev),
             torch.empty((c, 32), dtype=torch.uint8, device=dev),
             torch.empty((c, 32), dtype=torch.uint8, device=dev)) for c in counts]
    torch.cuda.synchronize()
    c = lib.Context(0)
    try:
        # independent calls (own outputs, shared context buffers) alternating between the two
        # streams with no wait between the streams: only the context orders them
        say("one context, two streams: encaps")
        for k, cnt in enumerate(counts):
            d_ct, d_ss, _ = outs[k]
            with torch.cuda.stream(streams[k % 2]):
                c.encaps_batch(pid, cnt, d_pk, d_mus[k], d_ct, d_ss)
        torch.cuda.synchronize()
        say("one context, two streams: decaps")
        for k, cnt in enumerate(counts):
            d_ct, _, d_ss2 = outs[k]
            with torch.cuda.stream(streams[(k + 1) % 2]):
                c.decaps_batch(pid, cnt, d_sk, d_ct, d_ss2)
        torch.cuda.synchronize()
    finally:
        c.close()
    for k, cnt in enumerate(counts):
        ct, ss, ss2 = (x.cpu().numpy() for x in outs[k])
        assert np.array_equal(ss, ss2), k
        for i in (0, cnt - 1):
            oct_, oss = orc.kem_encaps(op, pk, mus[k][i].tobytes())
            assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss, (k, i)
