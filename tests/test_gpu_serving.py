"""Serving on the GPU: mixed KeyGen / Encaps / Decaps requests of the serving workload's
dimensions (n = 640, 976, 1344, 4096) arrive while other groups are in flight; every result
must be byte-identical to the same request run alone (tolerance 0: the arithmetic is integer),
a sample of every dimension is checked against the oracle, and the device memory the lanes
really hold stays within the server's budget."""
import sys
import threading
import time

import numpy as np
import pytest

import lwe_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


NS = [640, 976, 1344, 4096]


@pytest.fixture(scope="module")
def keys(orc):
    """Resident key pairs made by the oracle from seeded inputs, so that every oracle check
    below starts from inputs that never went through the HIP path."""
    out = {}
    g = lwe_inputs.rng(4, 54)
    for n in NS:
        o = orc.params_for(n)
        pairs = [orc.kem_keygen(o, *(x[0].tobytes() for x in lwe_inputs.keygen_seeds(g, 1))) for _ in range(3)]
        out[n] = (np.stack([np.frombuffer(p[0], np.uint8) for p in pairs]),
                  np.stack([np.frombuffer(p[1], np.uint8) for p in pairs]))
    return out


@pytest.fixture(scope="module")
def backend(keys):
    from paper_2606_01211_amd.serve import LibraryBackend

    be = LibraryBackend(NS, keys_per_n=3, lanes=3, keys=keys)
    yield be
    be.close()


def test_mix_equals_alone(backend, keys, orc):
    from paper_2606_01211_amd.serve import DECAPS, ENCAPS, KEYGEN, Server

    ns = NS
    g = lwe_inputs.rng(4, 55)
    # Decaps inputs: ciphertexts the oracle made for the resident keys
    pool = {}
    for n in ns:
        o = orc.params_for(n)
        for key in range(3):
            pool[(n, key)] = [orc.kem_encaps(o, keys[n][0][key].tobytes(),
                                             lwe_inputs.messages(g, 1, o.mu_bytes)[0].tobytes())[0]
                              for _ in range(2)]
    reqs = []
    for i in range(240):
        op = int(g.choice(3, p=[0.2, 0.5, 0.3]))
        n = int(ns[i % len(ns)])
        key = int(g.integers(0, 3))
        p = backend.params[n]
        if op == KEYGEN:
            sa, ssk, z = lwe_inputs.keygen_seeds(g, 1)
            payload = (sa[0].tobytes(), ssk[0].tobytes(), z[0].tobytes())
        elif op == ENCAPS:
            payload = (lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes(),)
        else:
            ct = bytearray(pool[(n, key)][i % 2])
            if i % 7 == 0:
                ct[i % len(ct)] ^= 1  # some tampered ciphertexts: implicit rejection in the mix
            payload = (bytes(ct),)
        reqs.append((op, n, key, payload))
    # bursts: 40 Encaps and 40 Decaps per dimension on key 0, submitted while dispatching is
    # held, so that groups reach the batched kernels (strip product from 32 instances, device
    # FO hashing above 16) while other groups run
    for n in ns:
        p = backend.params[n]
        for k in range(40):
            reqs.append((ENCAPS, n, 0, (lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes(),)))
        for k in range(40):
            ct = bytearray(pool[(n, 0)][k % 2])
            if k % 5 == 0:
                ct[(7 * k) % len(ct)] ^= 2
            reqs.append((DECAPS, n, 0, (bytes(ct),)))
    say("serving mix of", len(reqs))
    budget = 2 << 30
    server = Server(backend, hbm_budget=budget, max_batch=64)
    futs = []
    for i, (op, n, key, payload) in enumerate(reqs[:240]):
        futs.append(server.submit(op, n, key, payload))
        if i % 20 == 19:
            time.sleep(0.002)  # arrivals spread over time: later requests join while others run
    server.pause()
    for op, n, key, payload in reqs[240:]:
        futs.append(server.submit(op, n, key, payload))
    server.resume()
    results = [f.result(timeout=300) for f in futs]
    held = sum(backend.held_bytes(lane) for lane in range(backend.lanes()))
    assert server.max_reserved <= budget and server.max_held <= budget and held <= budget
    groups = list(server.groups)
    server.close()
    assert len(groups) < len(reqs)
    assert max(gr[3] for gr in groups) >= 32
    assert server.max_in_flight_groups > 1
    for n in ns:  # every dimension ran batched groups
        assert max(gr[3] for gr in groups if gr[1] == n) >= 32, n
    say("groups", len(groups), "max concurrent", server.max_in_flight_groups, "held", held)
    # alone: each request as its own group of one
    for i, (op, n, key, payload) in enumerate(reqs):
        alone = backend.run(0, op, n, key, [payload])[0]
        assert alone == results[i], (i, op, n)
    # oracle on a sample (its inputs: seeds, messages, oracle keys and oracle ciphertexts):
    # the first 32 requests (every dimension and operation) and two of each burst
    sample = list(range(32)) + [240 + 80 * b + k for b in range(len(ns)) for k in (0, 79)]
    for i in sample:
        op, n, key, payload = reqs[i]
        o = orc.params_for(n)
        pk, sk = keys[n][0][key], keys[n][1][key]
        if op == KEYGEN:
            assert results[i] == orc.kem_keygen(o, *payload)
        elif op == ENCAPS:
            assert results[i] == orc.kem_encaps(o, pk.tobytes(), payload[0])
        else:
            assert results[i] == orc.kem_decaps(o, sk.tobytes(), payload[0])[0]


def test_small_budget_admission(backend):
    """A budget that admits only small groups still serves every request (idle lanes release
    their buffers when they block a group), the lanes' real device memory never exceeds it,
    and a request that cannot fit at all fails alone."""
    from paper_2606_01211_amd.serve import ENCAPS, LweError, Server

    lanes = backend.lanes()
    base = 1024  # the AES table every library context keeps
    # one lane running 4 Encaps at n = 1344 while the others hold only their tables
    budget = backend.call_bytes(1344, ENCAPS, 4) + (lanes - 1) * base
    g = lwe_inputs.rng(4, 56)
    with Server(backend, hbm_budget=budget, max_batch=64) as s:
        futs = [s.submit(ENCAPS, 1344, i % 3, (lwe_inputs.messages(g, 1, 32)[0].tobytes(),)) for i in range(40)]
        out = [f.result(timeout=120) for f in futs]
        held = sum(backend.held_bytes(lane) for lane in range(lanes))
        assert s.max_reserved <= budget and s.max_held <= budget and held <= budget
        assert max(gr[3] for gr in s.groups) <= 4
    assert len(out) == 40
    tiny = backend.call_bytes(640, ENCAPS, 1) + (lanes - 1) * base - 1
    with Server(backend, hbm_budget=tiny, max_batch=64) as s:
        f = s.submit(ENCAPS, 640, 0, (bytes(16),))
        with pytest.raises(LweError):
            f.result(timeout=60)


def test_call_bytes_bounds_a_call(backend):
    """lwe_ctx_call_bytes is an upper bound of what a call holds from a trimmed context, for
    every operation and dimension of the mix, host and device hashing, both product kernels."""
    from paper_2606_01211_amd.serve import DECAPS, ENCAPS, KEYGEN

    g = lwe_inputs.rng(4, 57)
    for n in NS:
        p = backend.params[n]
        for count in (1, 20, 40):
            for op in (KEYGEN, ENCAPS, DECAPS):
                backend.trim(0)
                assert backend.held_bytes(0) == 1024
                if op == KEYGEN:
                    sa, ssk, z = lwe_inputs.keygen_seeds(g, count)
                    payloads = [(sa[i].tobytes(), ssk[i].tobytes(), z[i].tobytes()) for i in range(count)]
                elif op == ENCAPS:
                    payloads = [(lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes(),) for _ in range(count)]
                else:
                    payloads = [(bytes(p.ct_bytes),) for _ in range(count)]
                need = backend.call_bytes(n, op, count)
                backend.limit_lane(0, need)  # the library refuses to hold more
                try:
                    backend.run(0, op, n, 0, payloads)
                finally:
                    backend.limit_lane(0, 0)
                assert backend.held_bytes(0) <= need, (n, count, op)
