#!/usr/bin/env python3
"""Benchmark of the LWE KEM hot path on one MI355X.

Metric: encaps+decaps per second at n = 1344 (q = 2^16, nbar = mbar = 8, 4-bit coefficients),
batched (4096 encapsulations against one public key in one call, then 4096 decapsulations)
versus plain (one instance per call), with p50/p99 latencies.

One step = KeyGen of a fresh key pair + lwe_encaps_batch(4096) + lwe_decaps_batch(4096) on
device-resident buffers: every stage of the hot path (A expansion, sampling, all products,
decoding, re-encryption + comparison, FO hashing) runs inside the timed region.
`value` = 4096 * steps / wall time of the timed steps.

Also reported: the plain path (lwe_encaps / lwe_decaps one instance per call), per-kernel
device time from HIP events recorded by the library on its streams, the roofline of the
dominant kernel, and the CPU oracle timed on this host over a bounded sample of the same
workload (whose outputs are compared byte for byte with the GPU's).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encaps+decaps/sec at n=1344, batched vs plain (bit-exact); p50/p99 ms"

# MI355X peaks used for the roofline (vendor figures)
PEAK_HBM_GBS = 8000.0
PEAK_INT8_TOPS = 5000.0
# 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work per unit (see the design notes for the derivations)
AES_OPS_PER_BLOCK = 160 + 160 + 40  # 160 table lookups, 160 XORs into the state, 40 round-key XORs (10 rounds)
KECCAK_OPS_PER_PERM = 24 * (50 + 50 + 50 + 50 + 2)  # theta, rho, pi-chi (ANDN+XOR), iota per round on 32-bit halves


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1344)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--plain", type=int, default=300, help="plain encaps and decaps calls timed one by one")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU oracle leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_calibration():
    import torch

    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}), flush=True)
    return 0


def main():
    args = parse()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print("bench.py measures one GPU: the KEM hot path here runs on a single MI355X; "
              "--gpus %d is not supported (every GPU box has one GPU)" % args.gpus, file=sys.stderr)
        return 2
    import torch

    import lwe_inputs
    import paper_2606_01211_amd as L

    torch.cuda.init()
    dev = torch.device("cuda:0")
    pid = L.param_id(args.n)
    p = L.params(pid)
    B = args.batch
    K, W = args.steps, args.warmup
    ctx = L.Context(0)

    g = lwe_inputs.rng(3, 0)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, W + K)
    mus = lwe_inputs.messages(g, B, p.mu_bytes)
    d_mu = torch.from_numpy(mus).to(dev)
    d_pk = torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev)
    d_sk = torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev)
    d_ct = torch.empty((B, p.ct_bytes), dtype=torch.uint8, device=dev)
    d_ss = torch.empty((B, 32), dtype=torch.uint8, device=dev)
    d_ss2 = torch.empty((B, 32), dtype=torch.uint8, device=dev)

    def step(i):
        ctx.keygen(pid, seedA[i], seedSK[i], z[i], d_pk, d_sk)
        ctx.encaps_batch(pid, B, d_pk, d_mu, d_ct, d_ss)
        ctx.decaps_batch(pid, B, d_sk, d_ct, d_ss2)

    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    # ---------------- batched, timed ----------------
    ctx.prof_reset()
    ctx.prof_enable(True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record()
    for i in range(K):
        step(W + i)
        evs[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.prof_read()
    ctx.prof_enable(False)
    wall = t1 - t0
    value = K * B / wall
    step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(K)]
    device_agree = bool(torch.equal(d_ss, d_ss2))
    print("batched: %.1f encaps+decaps/s, %.3f ms/step" % (value, 1e3 * wall / K), file=sys.stderr, flush=True)

    # ---------------- plain: one instance per call ----------------
    P = args.plain
    enc_ms, dec_ms = [], []
    c1 = torch.empty(p.ct_bytes, dtype=torch.uint8, device=dev)
    s1 = torch.empty(32, dtype=torch.uint8, device=dev)
    s2 = torch.empty(32, dtype=torch.uint8, device=dev)
    plain_ok = True
    for i in range(min(P, B)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        ctx.encaps(pid, d_pk, d_mu[i], c1, s1)
        torch.cuda.synchronize()
        b = time.perf_counter()
        ctx.decaps(pid, d_sk, c1, s2)
        torch.cuda.synchronize()
        c = time.perf_counter()
        enc_ms.append(1e3 * (b - a))
        dec_ms.append(1e3 * (c - b))
        if i < 8:
            plain_ok &= bool(torch.equal(c1, d_ct[i])) and bool(torch.equal(s1, d_ss[i])) and bool(torch.equal(s1, s2))
    plain_rate = len(enc_ms) / (1e-3 * (sum(enc_ms) + sum(dec_ms)))
    print("plain: %.1f encaps+decaps/s" % plain_rate, file=sys.stderr, flush=True)

    # ---------------- roofline of the dominant kernel ----------------
    n = p.n
    M = 8 * B
    kern = {k: {"launches": v[0], "total_ms": v[1], "avg_us": 1e3 * v[1] / v[0]} for k, v in prof.items()}
    dominant = max(kern, key=lambda k: kern[k]["total_ms"])
    d = kern[dominant]
    avg_s = d["avg_us"] * 1e-6
    if dominant == "prod_strip":
        work = 2 * 2 * M * n * (n + 8)  # two limbs x (multiply + add) x rows x K x (A | B columns)
        roof = {"bound": "mfma", "achieved": work / avg_s / 1e12, "peak": PEAK_INT8_TOPS, "unit": "TOPS"}
    elif dominant == "sample":
        work = B * (2 * n + 8) * AES_OPS_PER_BLOCK
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": PEAK_VALU_TOPS, "unit": "Tops/s"}
    elif dominant == "hash_records":
        perms = B * (-(-(p.ct_bytes + 1) // 136))
        work = perms * KECCAK_OPS_PER_PERM
        roof = {"bound": "alu", "achieved": work / avg_s / 1e12, "peak": PEAK_VALU_TOPS, "unit": "Tops/s"}
    else:
        work = B * p.ct_bytes
        roof = {"bound": "hbm", "achieved": work / avg_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dominant
    roof["avg_us"] = d["avg_us"]
    roof["traffic"] = None

    # ---------------- CPU oracle on a bounded sample ----------------
    cpu = None
    bit_exact = device_agree and plain_ok
    if not args.no_cpu:
        import oracle

        op = oracle.params_for(n)
        # the oracle starts from the same seeds as the GPU, never from GPU outputs
        i_last = W + K - 1
        ta = time.perf_counter()
        opk, osk = oracle.kem_keygen(op, seedA[i_last].tobytes(), seedSK[i_last].tobytes(), z[i_last].tobytes())
        bit_exact &= opk == d_pk.cpu().numpy().tobytes() and osk == d_sk.cpu().numpy().tobytes()
        ct = d_ct.cpu().numpy()
        ss = d_ss.cpu().numpy()
        done = 0
        while True:
            oct_, oss = oracle.kem_encaps(op, opk, mus[done].tobytes())
            oss2, ok = oracle.kem_decaps(op, osk, oct_)
            bit_exact &= (oct_ == ct[done].tobytes()) and (oss == ss[done].tobytes()) and ok and oss2 == oss
            done += 1
            if time.perf_counter() - ta > args.cpu_seconds or done >= B:
                break
        tcpu = time.perf_counter() - ta
        cpu = {"value": done / tcpu, "unit": "encaps+decaps/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": "one keygen + %d encaps+decaps pairs of the last timed n=%d step (same seeds and mu), "
                         "compared byte for byte with the GPU outputs" % (done, n)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "encaps+decaps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "batched-n%dx%d" % (n, B), "n": n, "logq": p.logq, "B": p.B, "batch": B,
                   "nbar": 8, "mbar": 8, "step": "keygen + encaps_batch + decaps_batch"},
        "bit_exact": bit_exact,
        "batch_latency_ms": {"p50": pct(step_ms, 50), "p99": pct(step_ms, 99)},
        "plain": {"value": plain_rate, "unit": "encaps+decaps/s",
                  "encaps_ms": {"p50": pct(enc_ms, 50), "p99": pct(enc_ms, 99)},
                  "decaps_ms": {"p50": pct(dec_ms, 50), "p99": pct(dec_ms, 99)}, "calls": len(enc_ms)},
        "batched_over_plain": value / plain_rate,
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
