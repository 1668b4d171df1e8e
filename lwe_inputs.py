"""Seeded synthetic inputs for the LWE KEM workloads.

Shared by the tests, the smoke check and the benchmark; holds none of the scheme's
arithmetic (no AES, hashing, sampling or products) -- only the random seeds, secrets z
and messages mu that the KEM consumes, drawn from numpy's PCG64 so every run is
reproducible.  Production callers draw these from the operating system instead.

Workloads (the paper runs N sequential KEM iterations on random seeds, Sec. 4):
  0  n=640  q=2^15: one keygen + encaps + decaps
  1  n=1344 q=2^16: one key, encaps/decaps one instance per call
  2  n in {8192, 16384, 32768}: one keygen + encaps + decaps each
  3  n=1344: one key, 4096 encapsulations in one batch, then 4096 decapsulations
  4  serving: Poisson arrivals over n in {640, 976, 1344, 4096}, 20/50/30 keygen/encaps/decaps
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 2606012110

WORKLOADS = {
    0: {"name": "plain-n640", "n": [640]},
    1: {"name": "plain-n1344", "n": [1344]},
    2: {"name": "large-n", "n": [8192, 16384, 32768]},
    3: {"name": "batched-n1344x4096", "n": [1344], "batch": 4096},
    4: {"name": "serving-mix", "n": [640, 976, 1344, 4096], "mix": (0.2, 0.5, 0.3), "keypairs": 64},
}


def rng(workload: int, stream: int = 0) -> np.random.Generator:
    """Generator for workload `workload`; `stream` separates independent uses."""
    return np.random.Generator(np.random.PCG64([MASTER_SEED + workload, stream]))


def random_bytes(g: np.random.Generator, count: int, size: int) -> np.ndarray:
    """count x size uniformly random bytes (uint8, C-contiguous)."""
    return g.integers(0, 256, size=(count, size), dtype=np.uint8)


def keygen_seeds(g: np.random.Generator, count: int):
    """(seedA[count][16], seedSK[count][16], z[count][32])."""
    return random_bytes(g, count, 16), random_bytes(g, count, 16), random_bytes(g, count, 32)


def messages(g: np.random.Generator, count: int, mu_bytes: int) -> np.ndarray:
    return random_bytes(g, count, mu_bytes)


def coins(g: np.random.Generator, count: int) -> np.ndarray:
    return random_bytes(g, count, 16)


def poisson_arrivals(g: np.random.Generator, qps: float, count: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    return np.cumsum(g.exponential(1.0 / qps, size=count))


def request_mix(g: np.random.Generator, count: int, ns, mix=(0.2, 0.5, 0.3)):
    """(op[count] in {0 keygen, 1 encaps, 2 decaps}, n[count]) for the serving workload."""
    ops = g.choice(3, size=count, p=np.asarray(mix) / np.sum(mix))
    nsel = g.choice(np.asarray(ns), size=count)
    return ops.astype(np.int64), nsel.astype(np.int64)
