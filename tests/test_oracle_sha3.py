"""Pins of the oracle's SHA3-256 (the hash H of the FO transform, Alg. 4-5) against the
FIPS 202 example digests and Python's hashlib as an independent implementation."""
import hashlib
import os

import pytest

import lwe_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sha3_256_known_answers.txt")


def test_fips202_examples(orc):
    with open(GOLDEN) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for msg, digest in rows:
        m = b"" if msg == "-" else bytes.fromhex(msg)
        assert orc.sha3_256(m).hex() == digest


@pytest.mark.parametrize("length", [0, 1, 7, 8, 135, 136, 137, 271, 272, 273, 1000, 10368, 21632])
def test_matches_hashlib(orc, length):
    g = lwe_inputs.rng(0, 200 + length)
    m = lwe_inputs.random_bytes(g, 1, max(1, length))[0].tobytes()[:length]
    assert orc.sha3_256(m) == hashlib.sha3_256(m).digest()
