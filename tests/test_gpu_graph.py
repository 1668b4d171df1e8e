"""A step of the hot path (KeyGen + encaps_batch + decaps_batch on device buffers, above the
host-hashing batch size) captured from the library calls into a HIP graph and replayed with new
seeds in fixed slots.  Every replay must equal the same step run call by call, byte for byte
(tolerance 0: integer work), with call-by-call steps and synchronisations between the replays;
one replay is also checked against the oracle.  The host hashing of KeyGen's public key and of
Encaps' H(pk) runs as queued host functions, which the graph replays too."""
import sys

import numpy as np
import pytest

import lwe_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,batch", [(640, 40), (1344, 64)])
def test_graph_replay_equals_calls(n, batch, orc):
    import torch

    import paper_2606_01211_amd as L

    say("graph replay", n, batch)
    dev = torch.device("cuda:0")
    pid = L.param_id(n)
    p = L.params(pid)
    c = L.Context(0)
    c.set_side_stream(False)
    h = c.stream_handle
    st = torch.cuda.ExternalStream(h, device=dev)
    g = lwe_inputs.rng(4, 70 + n)
    sa, ssk, z = lwe_inputs.keygen_seeds(g, 6)
    seeds = torch.from_numpy(np.ascontiguousarray(np.concatenate([sa, ssk, z], axis=1))).to(dev)
    mus = lwe_inputs.messages(g, batch, p.mu_bytes)
    d_mu = torch.from_numpy(mus).to(dev)
    slot = torch.empty(64, dtype=torch.uint8, device=dev)
    out = {"pk": torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev),
           "sk": torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev),
           "ct": torch.empty((batch, p.ct_bytes), dtype=torch.uint8, device=dev),
           "ss": torch.empty((batch, 32), dtype=torch.uint8, device=dev),
           "ss2": torch.empty((batch, 32), dtype=torch.uint8, device=dev)}

    def load(i):
        with torch.cuda.stream(st):
            slot.copy_(seeds[i])

    def calls():
        c.keygen(pid, slot[0:16], slot[16:32], slot[32:64], out["pk"], out["sk"], stream=h)
        c.encaps_batch(pid, batch, out["pk"], d_mu, out["ct"], out["ss"], stream=h)
        c.decaps_batch(pid, batch, out["sk"], out["ct"], out["ss2"], stream=h)

    def snap():
        torch.cuda.synchronize()
        return {k: v.cpu().numpy().copy() for k, v in out.items()}

    ref = {}
    for i in range(6):
        load(i)
        calls()
        ref[i] = snap()
        assert np.array_equal(ref[i]["ss"], ref[i]["ss2"])
    gr = torch.cuda.CUDAGraph()
    load(0)
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        gr.capture_begin(capture_error_mode="relaxed")
        calls()
        gr.capture_end()
    torch.cuda.synchronize()
    for rep, i in enumerate([3, 4, 1, 5, 3]):
        load(i)
        with torch.cuda.stream(st):
            gr.replay()
        got = snap()
        for k in out:
            assert np.array_equal(got[k], ref[i][k]), (rep, i, k)
        # call-by-call work and a synchronisation between replays
        load((i + 1) % 6)
        calls()
        got = snap()
        assert np.array_equal(got["ct"], ref[(i + 1) % 6]["ct"])
    # one replay against the oracle (its inputs: the seeds and messages)
    load(2)
    with torch.cuda.stream(st):
        gr.replay()
    got = snap()
    o = orc.params_for(n)
    pk, sk = orc.kem_keygen(o, sa[2].tobytes(), ssk[2].tobytes(), z[2].tobytes())
    assert got["pk"].tobytes() == pk and got["sk"].tobytes() == sk
    for j in (0, batch - 1):
        ct, ss = orc.kem_encaps(o, pk, mus[j].tobytes())
        assert got["ct"][j].tobytes() == ct and got["ss"][j].tobytes() == ss
    c.close()
