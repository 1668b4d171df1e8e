"""The all-cores CPU comparator (cpu_comparator/) against the oracle, byte for byte: KeyGen,
batched Encaps and Decaps (including implicit rejection) at n = 640 (q = 2^15) and
n = 1344 (q = 2^16).  The comparator is a separate implementation used only for timing the
CPU side of the GPU-versus-CPU comparison; these checks make its timings those of the same
scheme."""
import hashlib

import numpy as np
import pytest

import lwe_inputs

H = lambda b: hashlib.sha3_256(b).digest()  # noqa: E731


@pytest.mark.parametrize("n,count", [(640, 5), (1344, 3)])
def test_comparator_matches_oracle(orc, n, count):
    import cpu_comparator

    o = orc.params_for(n)
    kem = cpu_comparator.Kem(o.n, o.logq, o.B, o.K, o.sigma)
    g = lwe_inputs.rng(0, 900 + n)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, 2)
    pk, sk = kem.keygen_batch(seedA, seedSK, z)
    for i in range(2):
        opk, osk = orc.kem_keygen(o, seedA[i].tobytes(), seedSK[i].tobytes(), z[i].tobytes())
        assert pk[i].tobytes() == opk and sk[i].tobytes() == osk
    mu = lwe_inputs.messages(g, count, o.mu_bytes)
    ct, ss = kem.encaps_batch(pk[0], mu)
    for i in range(count):
        oct_, oss = orc.kem_encaps(o, pk[0].tobytes(), mu[i].tobytes())
        assert ct[i].tobytes() == oct_ and ss[i].tobytes() == oss
    assert np.array_equal(kem.decaps_batch(sk[0], ct), ss)
    bad = ct.copy()
    bad[1, 10] ^= 4
    ss2 = kem.decaps_batch(sk[0], bad)
    assert ss2[1].tobytes() == H(z[0].tobytes() + H(bad[1].tobytes()))
    assert np.array_equal(np.delete(ss2, 1, 0), np.delete(ss, 1, 0))
