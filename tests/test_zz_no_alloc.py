"""The decapsulation entry point that allocates nothing (lwe_decaps_batch_noalloc) against
lwe_decaps_batch, through the C ABI: two calls in a row on the same static device array, the
second smaller than the first (stale contents from the first call must not leak into it),
both byte-equal to the context-based entry point on the same inputs, including an
implicitly rejected (tampered) ciphertext; a batch beyond the array's capacity is refused
before anything is launched.  Integer outputs: tolerance 0."""
import sys

import numpy as np
import pytest

import lwe_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [640, 1344])
def test_noalloc_matches_decaps_batch(ctx, orc, n):
    import torch

    import paper_2606_01211_amd as L

    dev = torch.device("cuda:0")
    pid = L.param_id(n)
    p = L.params(pid)
    g = lwe_inputs.rng(4, 700 + n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 1)
    big, small = 40, 5  # strip product (>= 32 instances), then the streaming product
    mu = torch.from_numpy(lwe_inputs.messages(g, big, p.mu_bytes)).to(dev)
    pk = torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev)
    sk = torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev)
    ct = torch.empty((big, p.ct_bytes), dtype=torch.uint8, device=dev)
    ss = torch.empty((big, 32), dtype=torch.uint8, device=dev)
    ctx.keygen(pid, seedA[0], seedSK[0], z[0], pk, sk)
    ctx.encaps_batch(pid, big, pk, mu, ct, ss)
    # implicit rejection paths: one coefficient of B' and one of V changed
    ct[3, 7] ^= 1
    ct[big - 2, p.ct_bytes - 1] ^= 0x40
    torch.cuda.synchronize()
    for count in (big, small):
        say("noalloc decaps n=%d count=%d" % (n, count))
        ref = torch.empty((count, 32), dtype=torch.uint8, device=dev)
        got = torch.full((count, 32), 0xA5, dtype=torch.uint8, device=dev)
        ctx.decaps_batch(pid, count, sk, ct[:count], ref)
        torch.cuda.synchronize()
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            L.decaps_batch_noalloc(pid, count, sk, ct[:count], got)
        side.synchronize()
        assert torch.equal(got, ref), "noalloc decaps differs from lwe_decaps_batch (count=%d)" % count
        # accepted instances give the encapsulated secret; tampered ones the rejection key
        assert torch.equal(got[0], ss[0])
        assert not torch.equal(got[3], ss[3])
    # one rejected instance checked against the oracle's implicit-rejection value
    op = orc.params_for(n)
    osk = sk.cpu().numpy().tobytes()
    ct3 = ct[3].cpu().numpy().tobytes()
    oss, ok = orc.kem_decaps(op, osk, ct3)
    assert not ok
    got3 = torch.empty((1, 32), dtype=torch.uint8, device=dev)
    L.decaps_batch_noalloc(pid, 1, sk, ct[3:4], got3)
    torch.cuda.synchronize()
    assert got3.cpu().numpy().tobytes() == oss


def test_noalloc_refuses_oversized_and_host_buffers():
    import torch

    import paper_2606_01211_amd as L

    dev = torch.device("cuda:0")
    n = 1344
    pid = L.param_id(n)
    p = L.params(pid)
    count = 2000  # about 21.9 KB of working memory each: more than the 32 MiB array
    sk = torch.zeros(p.sk_bytes, dtype=torch.uint8, device=dev)
    ct = torch.zeros((count, p.ct_bytes), dtype=torch.uint8, device=dev)
    ss = torch.zeros((count, 32), dtype=torch.uint8, device=dev)
    with pytest.raises(L.LweError) as e:
        L.decaps_batch_noalloc(pid, count, sk, ct, ss)
    assert e.value.status == L.lwe.LWE_ENOMEM
    assert int(ss.sum()) == 0  # nothing was launched
    with pytest.raises(ValueError):
        L.decaps_batch_noalloc(pid, 1, sk.cpu(), ct[:1], ss[:1])
