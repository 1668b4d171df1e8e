#!/usr/bin/env python3
"""Benchmark of the LWE KEM hot path on one MI355X.

Metric: encaps+decaps per second at n = 1344 (q = 2^16, nbar = mbar = 8, 4-bit coefficients),
batched (4096 encapsulations against one public key in one call, then 4096 decapsulations)
versus plain (one instance per call), with p50/p99 latencies.

One step = KeyGen of a fresh key pair + lwe_encaps_batch(4096) + lwe_decaps_batch(4096) on
device-resident buffers: every stage of the hot path (A expansion, sampling, all products,
decoding, re-encryption + comparison, FO hashing) runs inside the timed region.
`value` = 4096 * steps / wall time of the timed steps, with independent steps in flight on
several lanes (one library context and HIP stream per lane; each lane's context keeps all of
its work on that one stream, so every lane has a hardware queue of its own).  The lane count
is the largest divisor of --steps not above --streams (at least half of it), so every lane
runs the same number of timed steps; the feeding threads start together after the device
has drained.  `serial` is the same K steps on one lane with the same kernels, and the
per-kernel times, `roofline` and `fused_product` come from it (stand-alone times of the
kernels behind `value`); `kernels_pipelined` has the same kernels' times in the pipelined run
when the lanes are fed call by call (--eager).  By default each lane replays its step as a HIP
graph captured from the same library calls (checked byte for byte against a call-by-call step
first), so that the host work of the calls does not stagger the lanes.

Also reported: the plain path (lwe_encaps / lwe_decaps one instance per call, wall and device
time), the CPU oracle timed on this host over a bounded sample of the same workload (whose
outputs are compared byte for byte with the GPU's), and under `extras` the other workloads:
plain n = 640 KEMs with p50/p99, single large-n KEMs (fused, and unfused at the largest n) and
the serving workload at 0.5 and 0.8 of its measured capacity.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import threading
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
# Per AES block of the sampler's compiled kernel (k_sample<6>): VALU instructions (cipher, CDF
# compare and store: SQ_INSTS_VALU over the blocks of a launch, 69.9 M x 64 / 11.04 M) and LDS
# table lookups (the cipher's 148 per block with round 1's fixed part hoisted)
SAMPLE_VALU_PER_BLOCK = 405
SAMPLE_LDS_PER_BLOCK = 148
# Per absorbed block, per wave of the two-lane SHA3 kernel (k_hash_records): two passes of the
# 12-round permutation body (1317 instructions each) plus the block's load and bit
# interleaving; SQ_INSTS_VALU gives 475 K per wave for 160 blocks
HASH_VALU_PER_BLOCK = 2960
# Per absorbed block, per wave of the one-record-per-thread SHA3 kernel (k_hash_records_one):
# the 24-round permutation on the whole state of one record per lane (4343 instructions in
# the compiled loop: 2880 v_bitop3, 1392 v_alignbit, the rest XOR) plus the block's 34-word
# absorb and state moves
HASH_ONE_VALU_PER_BLOCK = 4420
# LDS: 256 CUs x 128 bytes per clock x 2.4 GHz
PEAK_LDS_TBS = 256 * 128 * 2.4e9 / 1e12


class Roctx:
    """ROCTx ranges around the benchmark's legs (no-ops when the library is absent), so that a
    rocprofv3 --marker-trace run can attribute every kernel dispatch to its leg."""

    def __init__(self):
        import ctypes

        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "/opt/rocm/lib/librocprofiler-sdk-roctx.so.1"):
            try:
                self.lib = ctypes.CDLL(name)
                self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except OSError:
                continue

    def push(self, name):
        if self.lib:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib:
            self.lib.roctxRangePop()


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=140,
                    help="timed steps (spread round-robin over the lanes)")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=1344)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--plain", type=int, default=300, help="plain encaps and decaps calls timed one by one")
    ap.add_argument("--streams", type=int, default=20,
                    help="most independent steps in flight (one library context and HIP stream each); "
                         "the lane count is the largest divisor of --steps up to this; the serial rate "
                         "(one lane) is always measured too")
    ap.add_argument("--lane-side-stream", action="store_true",
                    help="let the lanes' decapsulations hash on their context's second stream too "
                         "(two streams per lane)")
    ap.add_argument("--lane-hash-lanes", type=int, default=1, choices=(1, 2),
                    help="lanes per record of the SHA3 kernels of every lane and of the serial run: "
                         "1 (k_hash_records_one, fewer instructions per record, the better pipelined "
                         "rate) or 2 (k_hash_records, half the chain length per launch)")
    ap.add_argument("--feed-threads", action="store_true",
                    help="feed the replaying lanes from one host thread each instead of issuing every "
                         "step's replay from one thread in turn")
    ap.add_argument("--eager", action="store_true",
                    help="feed the pipelined lanes call by call instead of replaying each lane's step as "
                         "a captured HIP graph")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="HIP hardware queues of this process (GPU_MAX_HW_QUEUES, at most 32; default "
                         "streams + 3, or 2 * streams + 2 with --lane-side-stream): every stream in "
                         "use then gets a queue of its own instead of waiting behind another "
                         "stream's packets")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="budget of the CPU oracle leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--large", action="store_true",
                    help="instead of the batched benchmark: one KeyGen, Encaps and Decaps per n in "
                         "--large-n (device-resident, A regenerated on the fly), timed per phase")
    ap.add_argument("--unfused", action="store_true",
                    help="run the unfused variant (tuning a_source = 1): every call first expands A "
                         "into device memory and the products read it back instead of regenerating it")
    ap.add_argument("--large-n", default="8192,16384,32768")
    ap.add_argument("--large-reps", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (plain n=640, large n fused/unfused, serving)")
    ap.add_argument("--plain640", type=int, default=300, help="n=640 KEMs timed one by one")
    ap.add_argument("--serve-seconds", type=float, default=6.0,
                    help="duration of each serving run (0.5 and 0.8 of capacity); 0 skips serving")
    ap.add_argument("--energy-seconds", type=float, default=3.0,
                    help="duration of the pipelined run during which GPU power is sampled (0 skips it)")
    ap.add_argument("--no-comparator", action="store_true", help="skip the all-cores CPU comparator")
    ap.add_argument("--paper-n", default="512,1024,2048,4096,8192,16384,32768",
                    help="the paper's own parameter sets (Table 1) timed under extras; empty skips them")
    ap.add_argument("--paper", action="store_true",
                    help="instead of the batched benchmark: the paper's own sets (--paper-n) only")
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


def large_runs(ctx, ns, reps, unfused, log=True):
    """Single KEMs at large n on one context: per-phase wall and device time, and the AES
    keystream rate of the regeneration of A (n^2/8 blocks per product pass).  With unfused,
    the context's tuning expands A into device memory first (a_source = 1)."""
    import torch

    import lwe_inputs
    import paper_2606_01211_amd as L

    dev = torch.device("cuda:0")
    runs = {}
    for n in ns:
        pid = L.param_id(n)
        p = L.params(pid)
        g = lwe_inputs.rng(2, n)
        pk = torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev)
        sk = torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev)
        ct = torch.empty(p.ct_bytes, dtype=torch.uint8, device=dev)
        ss = torch.empty(32, dtype=torch.uint8, device=dev)
        ss2 = torch.empty(32, dtype=torch.uint8, device=dev)
        saved = ctx.get_tuning(pid)
        if unfused:
            ctx.set_tuning(pid, **dict(saved, a_source=1))
        phases = {"keygen": [], "encaps": [], "decaps": []}
        dev_ms = {"keygen": [], "encaps": [], "decaps": []}
        kern_ms = {"keygen": {}, "encaps": {}, "decaps": {}}
        ok = True
        for rep in range(reps + 1):
            sa, ssk, z = lwe_inputs.keygen_seeds(g, 1)
            mu = torch.from_numpy(lwe_inputs.messages(g, 1, p.mu_bytes)[0]).to(dev)
            calls = (("keygen", lambda: ctx.keygen(pid, sa[0], ssk[0], z[0], pk, sk)),
                     ("encaps", lambda: ctx.encaps(pid, pk, mu, ct, ss)),
                     ("decaps", lambda: ctx.decaps(pid, sk, ct, ss2)))
            for name, fn in calls:
                ctx.prof_reset()
                ctx.prof_enable(True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                prof = ctx.prof_read()
                ctx.prof_enable(False)
                if rep > 0:  # the first repetition grows the context's buffers
                    phases[name].append(1e3 * (t1 - t0))
                    dev_ms[name].append(sum(ms for _, ms in prof.values()))
                    for k, (_, ms) in prof.items():
                        kern_ms[name].setdefault(k, []).append(ms)
            ok &= bool(torch.equal(ss, ss2))
            if log:
                print("n=%d rep %d done%s" % (n, rep, " (unfused)" if unfused else ""), file=sys.stderr, flush=True)
        ctx.set_tuning(pid, **saved)
        blocks = n * n // 8
        r = {"ok": ok, "aes_blocks_per_product": blocks, "a_source": "unfused" if unfused else "fused"}
        for name in phases:
            wall = float(np.median(phases[name]))
            devt = float(np.median(dev_ms[name]))
            r[name] = {"wall_ms": wall, "device_ms": devt,
                       "kernels_ms": {k: float(np.median(v)) for k, v in kern_ms[name].items()}}
        # one product pass (A regenerated once) in keygen and encaps, two in decaps (decrypt
        # reads no A; the re-encryption regenerates it once)
        km = r["encaps"]["kernels_ms"]
        prod_ms = km.get("prod_stream")
        r["keystream_GBps_encaps"] = blocks * 16 / (r["encaps"]["device_ms"] * 1e-3) / 1e9
        if prod_ms and not unfused:
            # the fused product kernel alone: its AES keystream rate and int8 MFMA rate (8 rows
            # padded to 16 for the MFMA tile: 2 limbs x 2 ops x 16 x n x (n + 8) issued)
            r["product_ms"] = prod_ms
            r["product_keystream_GBps"] = blocks * 16 / (prod_ms * 1e-3) / 1e9
            r["product_aes_Gblocks_s"] = blocks / (prod_ms * 1e-3) / 1e9
        if unfused:
            # A (n^2 uint16) written once by the expansion and read once by the product
            a_bytes = 2 * n * n
            r["unfused"] = {
                "A_bytes": a_bytes,
                "expand_A_ms": km.get("expand_A"),
                "expand_A_write_GBps": a_bytes / (km["expand_A"] * 1e-3) / 1e9 if km.get("expand_A") else None,
                "product_ms": prod_ms,
                "product_read_GBps": a_bytes / (prod_ms * 1e-3) / 1e9 if prod_ms else None,
                "hbm_peak_GBps": PEAK_HBM_GBS,
            }
        runs[str(n)] = r
    return runs


def large(args):
    """CLI mode --large: single KEMs at large n."""
    import paper_2606_01211_amd as L

    ctx = L.Context(0)
    out = {"mode": "large", "data": "synthetic",
           "runs": large_runs(ctx, [int(x) for x in args.large_n.split(",")], args.large_reps, args.unfused)}
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


class PowerSampler:
    """Samples the GPU's board power while running: the hwmon power file of the first AMD GPU
    (microwatts) every 50 ms when the kernel exposes one, else `amd-smi metric -p --json`
    about once a second.  energy_j() integrates the samples over the sampled interval."""

    def __init__(self):
        import glob
        import shutil

        self.path = None
        for cand in sorted(glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*/power1_average")) + \
                sorted(glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*/power1_input")):
            try:
                if float(open(cand).read().strip()) > 0:
                    self.path = cand
                    break
            except (OSError, ValueError):
                continue
        self.smi = shutil.which("amd-smi") or ("/opt/rocm/bin/amd-smi" if os.path.exists("/opt/rocm/bin/amd-smi") else None)
        self.samples = []
        self._stop = threading.Event()
        self._th = None

    def source(self):
        return "hwmon:" + self.path if self.path else ("amd-smi" if self.smi else None)

    def read_w(self):
        if self.path:
            try:
                return float(open(self.path).read().strip()) * 1e-6
            except (OSError, ValueError):
                return None
        if self.smi:
            import re
            import subprocess

            try:
                r = subprocess.run([self.smi, "metric", "-p", "--json"], capture_output=True, text=True, timeout=5)
            except (OSError, subprocess.TimeoutExpired):
                return None
            # the socket power of GPU 0, whatever the nesting of this amd-smi version's JSON
            m = re.search(r'"(?:socket_power|average_socket_power|current_socket_power)"\s*:\s*\{?[^0-9]*([0-9.]+)',
                          r.stdout)
            return float(m.group(1)) if m else None
        return None

    def _run(self):
        period = 0.05 if self.path else 1.0
        while not self._stop.is_set():
            w = self.read_w()
            if w is not None:
                self.samples.append((time.perf_counter(), w))
            self._stop.wait(period)

    def start(self):
        self._th = threading.Thread(target=self._run, daemon=True)
        self._th.start()

    def stop(self):
        self._stop.set()
        if self._th:
            self._th.join()

    def mean_w(self):
        return float(np.mean([w for _, w in self.samples])) if self.samples else None


def pick_lanes(steps, want):
    """Lane count for `steps` timed steps: the largest count <= want that divides steps (and is
    at least half of want), so that every lane runs the same number of timed steps; otherwise
    want lanes with uneven shares (reported as lanes_even = false)."""
    for s in range(min(want, steps), 0, -1):
        if steps % s == 0 and s >= max(1, want // 2):
            return s, True
    return max(1, min(want, steps)), steps % max(1, min(want, steps)) == 0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    args = parse()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print("bench.py measures one GPU: the KEM hot path here runs on a single MI355X; "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2
    K, W = args.steps, args.warmup
    S, lanes_even = pick_lanes(K, max(1, args.streams))
    # before anything initialises the GPU runtime
    hwq = args.hw_queues if args.hw_queues > 0 else (2 * S + 2 if args.lane_side_stream else S + 3)
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(1, hwq)))
    if args.large:
        return large(args)
    if args.paper:
        import torch

        import paper_2606_01211_amd as L

        ctx0 = L.Context(0)
        out = {"mode": "paper", "data": "synthetic",
               "runs": paper_runs(ctx0, L, torch, torch.device("cuda:0"), [int(x) for x in args.paper_n.split(",")])}
        ctx0.close()
        print(json.dumps(out), flush=True)
        return 0
    # The serving workload runs first, in a child process, while this process holds no GPU
    # queues: the lanes' hardware queues of both processes together would exceed what the
    # hardware scheduler maps at once, and time-sliced queues would distort the latencies.
    serving = None
    if not args.no_extras and args.serve_seconds > 0:
        serving = serving_run(args)
        print("extras: serving done", file=sys.stderr, flush=True)
    import torch

    import lwe_inputs
    import paper_2606_01211_amd as L

    torch.cuda.init()
    dev = torch.device("cuda:0")
    pid = L.param_id(args.n)
    p = L.params(pid)
    B = args.batch
    ctxs = [L.Context(0) for _ in range(S)]
    # Every lane (and the serial run on lane 0) uses the same kernels: all of a context's work
    # on its one stream (unless --lane-side-stream) and --lane-hash-lanes lanes per record in
    # the SHA3 kernels, so the serial run's kernel times describe the kernels behind `value`.
    for c in ctxs:
        c.set_side_stream(args.lane_side_stream)
        c.set_hash_lanes(args.lane_hash_lanes)
    streams = [torch.cuda.ExternalStream(c.stream_handle, device=dev) for c in ctxs]
    handles = [c.stream_handle for c in ctxs]
    ctx = ctxs[0]
    if args.unfused:
        for c in ctxs:
            t = c.get_tuning(pid)
            t["a_source"] = 1
            c.set_tuning(pid, **t)

    g = lwe_inputs.rng(3, 0)
    seedA, seedSK, z = lwe_inputs.keygen_seeds(g, W + 2 * K)
    mus = lwe_inputs.messages(g, B, p.mu_bytes)
    d_mu = torch.from_numpy(mus).to(dev)
    # every input of the timed steps is resident in device memory before timing starts; a step's
    # three seeds are one 64-byte row, loaded into its lane's seed slot by one copy
    d_seeds = torch.from_numpy(np.ascontiguousarray(np.concatenate([seedA, seedSK, z], axis=1))).to(dev)
    d_seedA, d_seedSK, d_z = d_seeds[:, 0:16], d_seeds[:, 16:32], d_seeds[:, 32:64]
    slots = [torch.empty(64, dtype=torch.uint8, device=dev) for _ in range(S)]
    bufs = []
    for _ in range(S):
        bufs.append({
            "pk": torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev),
            "sk": torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev),
            "ct": torch.empty((B, p.ct_bytes), dtype=torch.uint8, device=dev),
            "ss": torch.empty((B, 32), dtype=torch.uint8, device=dev),
            "ss2": torch.empty((B, 32), dtype=torch.uint8, device=dev),
        })
    torch.cuda.synchronize()

    def lane_step(lane):
        """One step on the lane's buffers, its seeds taken from the lane's seed slot."""
        c, bf, h, sl = ctxs[lane], bufs[lane], handles[lane], slots[lane]
        c.keygen(pid, sl[0:16], sl[16:32], sl[32:64], bf["pk"], bf["sk"], stream=h)
        c.encaps_batch(pid, B, bf["pk"], d_mu, bf["ct"], bf["ss"], stream=h)
        c.decaps_batch(pid, B, bf["sk"], bf["ct"], bf["ss2"], stream=h)

    graphs = None

    def step(i, lane):
        """Step i (its seeds) on `lane`: the call sequence, or a replay of the lane's graph."""
        with torch.cuda.stream(streams[lane]):
            slots[lane].copy_(d_seeds[i])
            if graphs is not None:
                graphs[lane].replay()
        if graphs is None:
            lane_step(lane)

    for i in range(W):
        for lane in range(S):
            step(i, lane)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    issue_ms = {}  # host time from the window's start until every step was queued, per lane count

    def timed(lanes, first_seed):
        """K steps spread round-robin over `lanes` streams.  Graph replays are issued in turn
        from this thread; library calls (and --feed-threads) come from one host thread per
        stream (the library calls queue their work without waiting for the device and release
        the interpreter lock), started first and released together by a barrier.  Either way
        the window opens after the device has drained, so it holds the K steps and nothing else.  Returns wall seconds, per-step device latencies (ms) and the merged
        kernel profile (library calls only: a graph replay has no per-kernel events)."""
        for c in ctxs:
            c.prof_reset()
            c.prof_enable(graphs is None)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        errors = []
        go = threading.Barrier(lanes + 1)

        def feed(lane):
            try:
                go.wait()
                for i in range(lane, K, lanes):
                    ev[i][0].record(streams[lane])
                    step(first_seed + i, lane)
                    ev[i][1].record(streams[lane])
            except Exception as e:  # surfaced after the join
                errors.append(e)

        # Graph replays need only a seed copy and a launch per step: one thread issues them all,
        # step i on lane i mod lanes, which starts the lanes sooner than threads contending for
        # the interpreter lock (each lane's steps stay in its stream's order).
        single = graphs is not None and lanes > 1 and not args.feed_threads
        th = [] if single else [threading.Thread(target=feed, args=(lane,)) for lane in range(lanes)]
        for t in th:
            t.start()
        torch.cuda.synchronize()
        # no collector pauses inside the timed region (they stall every feeding thread)
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        if single:
            for i in range(K):
                lane = i % lanes
                ev[i][0].record(streams[lane])
                step(first_seed + i, lane)
                ev[i][1].record(streams[lane])
        else:
            go.wait()
            for t in th:
                t.join()
        t_issued = time.perf_counter()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        issue_ms[lanes] = 1e3 * (t_issued - t0)
        gc.enable()
        if errors:
            raise errors[0]
        prof = {}
        for c in ctxs:
            for k, (cnt, ms) in c.prof_read().items():
                a = prof.setdefault(k, [0, 0.0])
                a[0] += cnt
                a[1] += ms
            c.prof_enable(False)
        return t1 - t0, [e0.elapsed_time(e1) for e0, e1 in ev], prof

    # ---------------- batched, timed ----------------
    # serial: the same K steps on one lane, call by call, with every kernel bracketed by HIP
    # events (stand-alone times of the kernels behind `value`)
    tx = Roctx()
    tx.push("leg:serial")
    wall1, step_ms1, prof1 = timed(1, W)
    tx.pop()
    serial_value = K * B / wall1
    # The pipelined lanes replay their step as a HIP graph captured from the same library calls:
    # the calls' own host work (about 35 runtime calls per step) serialises across feeding
    # threads and staggers the lanes' start by about 0.25 ms per lane.  A replay runs the same
    # kernels, copies and host hashing functions; it is checked against a call-by-call step of
    # the same seeds before timing.
    graph_check = None
    if not args.eager and S > 1:
        for c in ctxs:
            c.prof_enable(False)
        torch.cuda.synchronize()
        caps = []
        for lane in range(S):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(streams[lane]):
                slots[lane].copy_(d_seeds[0])
                g.capture_begin(capture_error_mode="relaxed")
                lane_step(lane)
                g.capture_end()
            caps.append(g)
        torch.cuda.synchronize()
        i_chk = W + 2 * K - 1
        step(i_chk, 0)  # call by call (graphs not yet in use)
        torch.cuda.synchronize()
        want = [bufs[0][k].clone() for k in ("pk", "sk", "ct", "ss", "ss2")]
        graphs = caps
        step(i_chk, 0)
        torch.cuda.synchronize()
        graph_check = all(bool(torch.equal(a, bufs[0][k])) for a, k in zip(want, ("pk", "sk", "ct", "ss", "ss2")))
        if not graph_check:
            print("graph replay differs from the call sequence: timing call by call", file=sys.stderr, flush=True)
            graphs = None
    if S > 1:
        tx.push("leg:pipelined")
        wall, step_ms, prof = timed(S, W + K)
        tx.pop()
    else:
        wall, step_ms, prof = wall1, step_ms1, prof1
    value = K * B / wall
    device_agree = all(bool(torch.equal(bf["ss"], bf["ss2"])) for bf in bufs)
    d_pk, d_sk, d_ct, d_ss = bufs[0]["pk"], bufs[0]["sk"], bufs[0]["ct"], bufs[0]["ss"]
    last_seed = W + K + (K - 1) - ((K - 1) % S) if S > 1 else W + K - 1  # last step run on lane 0
    print("batched: %.1f encaps+decaps/s (%d lanes x %s steps), serial %.1f, %.3f ms/step" %
          (value, S, K // S if lanes_even else "uneven", serial_value, 1e3 * wall / K), file=sys.stderr, flush=True)

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
    # device time of the same calls (kernel events on the context's streams), in a separate
    # pass so that the events do not slow the timed one
    dev_enc, dev_dec = [], []
    for i in range(min(50, B)):
        for name, fn, acc in (("encaps", lambda: ctx.encaps(pid, d_pk, d_mu[i], c1, s1), dev_enc),
                              ("decaps", lambda: ctx.decaps(pid, d_sk, c1, s2), dev_dec)):
            ctx.prof_reset()
            ctx.prof_enable(True)
            fn()
            torch.cuda.synchronize()
            acc.append(sum(ms for _, ms in ctx.prof_read().values()))
            ctx.prof_enable(False)
    print("plain: %.1f encaps+decaps/s" % plain_rate, file=sys.stderr, flush=True)

    # ---------------- rooflines ----------------
    # Algorithmic work per timed step (one KeyGen, encaps_batch(B), decaps_batch(B)) of each
    # large kernel; achieved = K steps of work / the kernel's total device time in the serial
    # run (HIP events on the launching stream; the kernels are those of the pipelined lanes).
    n = p.n
    M = 8 * B

    def kern_table(pr):
        return {k: {"launches": v[0], "total_ms": v[1], "avg_us": 1e3 * v[1] / v[0]} for k, v in pr.items()}

    kern = kern_table(prof1)
    ct_perms = -(-(p.ct_bytes + 1) // 136)
    work_per_step = {
        # strip product: the encapsulation (encryption) and the decapsulation's re-encryption
        # (compare mode); each launch 2 limbs x (mul + add) x M x K x (n + 8)
        "prod_strip": ("mfma", 2 * 2 * M * n * (n + 8)),
        "prod_strip_cmp": ("mfma", 2 * 2 * M * n * (n + 8)),
        # sampler: KeyGen (2n AES blocks) + two batched encryptions (2n + 8 blocks per instance)
        "sample": ("alu", (2 * n + 2 * B * (2 * n + 8)) * AES_OPS_PER_BLOCK),
        # H(ct) of the encapsulated and of the received ciphertexts
        "hash_records": ("alu", 2 * B * ct_perms * KECCAK_OPS_PER_PERM),
        # decryption reads B' and V of every ciphertext once
        "decrypt": ("hbm", B * p.ct_bytes),
    }
    if "expand_A" in kern:
        # unfused variant: each expansion writes A (n^2 uint16) once
        work_per_step["expand_A"] = ("hbm", kern["expand_A"]["launches"] / K * 2 * n * n)

    def roofline_of(name):
        bound, work = work_per_step[name]
        sec = kern[name]["total_ms"] * 1e-3 / K
        if bound == "mfma":
            r = {"bound": "mfma", "achieved": work / sec / 1e12, "peak": PEAK_INT8_TOPS, "unit": "TOPS"}
        elif bound == "alu":
            r = {"bound": "alu", "achieved": work / sec / 1e12, "peak": PEAK_VALU_TOPS, "unit": "Tops/s"}
        else:
            r = {"bound": "hbm", "achieved": work / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
        r["frac"] = r["achieved"] / r["peak"]
        r["kernel"] = name
        r["avg_us"] = kern[name]["avg_us"]
        r["launches_per_step"] = kern[name]["launches"] / K
        r["traffic"] = None
        r["leg"] = "serial (one lane, the kernels of the pipelined lanes)"
        return r

    rooflines = {k: roofline_of(k) for k in work_per_step if k in kern}
    # AES keystream rates.  The sampler's blocks per step are in its work above; the strip
    # product regenerates A once per row chunk (the regeneration factor) when fused.
    if "sample" in rooflines:
        blocks = 2 * n + 2 * B * (2 * n + 8)
        rooflines["sample"]["keystream_GBps"] = blocks * 16 / (kern["sample"]["total_ms"] * 1e-3 / K) / 1e9
        rooflines["sample"]["aes_Gblocks_s"] = blocks / (kern["sample"]["total_ms"] * 1e-3 / K) / 1e9
        # The sampler against the issue bound of its own instruction stream: blocks x VALU
        # instructions per block over the chip's 32-bit VALU rate, and blocks x LDS lookups per
        # block x 4 bytes over the chip's LDS bandwidth (per-block counts of the compiled kernel).
        t_s = kern["sample"]["total_ms"] * 1e-3 / K
        valu_s = blocks * SAMPLE_VALU_PER_BLOCK / (PEAK_VALU_TOPS * 1e12)
        lds_s = blocks * SAMPLE_LDS_PER_BLOCK * 4 / (PEAK_LDS_TBS * 1e12)
        rooflines["sample"]["issue_bound"] = {
            "valu_instr_per_block": SAMPLE_VALU_PER_BLOCK, "lds_lookups_per_block": SAMPLE_LDS_PER_BLOCK,
            "valu_bound_us_per_step": 1e6 * valu_s, "lds_bound_us_per_step": 1e6 * lds_s,
            "measured_us_per_step": 1e6 * t_s, "frac": max(valu_s, lds_s) / t_s}
    if "hash_records" in rooflines:
        # Each record (one lane, or a pair of lanes) is one dependent chain of ct_perms absorbed
        # blocks; a wave issues at most one VALU instruction per 4 cycles.  The chain's issue
        # bound per launch is ct_perms x instructions per block x 4 cycles at the 2.4 GHz clock.
        per_block = HASH_VALU_PER_BLOCK if args.lane_hash_lanes == 2 else HASH_ONE_VALU_PER_BLOCK
        t_h = kern["hash_records"]["avg_us"] * 1e-6
        chain_s = ct_perms * per_block * 4 / 2.4e9
        rooflines["hash_records"]["issue_bound"] = {
            "kernel": "k_hash_records" if args.lane_hash_lanes == 2 else "k_hash_records_one",
            "valu_instr_per_block_per_wave": per_block, "blocks_per_record": ct_perms,
            "waves_per_launch": args.lane_hash_lanes * B // 64, "chain_bound_us": 1e6 * chain_s,
            "measured_us": 1e6 * t_h, "frac": chain_s / t_h}
    if "prod_strip" in rooflines:
        mch = ctx.get_tuning(pid)["m_chunks"] or 8
        fused = not args.unfused
        rooflines["prod_strip"]["A_regeneration_factor"] = mch if fused else 0
        rooflines["prod_strip"]["aes_blocks_per_launch"] = mch * n * n // 8 if fused else 0
    # HBM traffic per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes
    # (scaled by the same counters over a 1 GiB copy); only while the kernels are those the
    # counters were taken on.
    try:
        here = os.path.dirname(os.path.abspath(__file__))
        tr = json.load(open(os.path.join(here, "profiles", "traffic.json")))
        src = open(os.path.join(here, "paper_2606_01211_amd", "csrc", "kernels.hip"), "rb").read()
        if tr.get("kernels_source_sha256") == hashlib.sha256(src).hexdigest():
            tk = tr["kernels"]

            def entry(prefix):  # kernel names carry their template arguments
                keys = [k for k in sorted(tk) if k.startswith(prefix)]
                return tk[keys[0]] if keys else None

            hname = "k_hash_records_one<" if args.lane_hash_lanes == 1 else "k_hash_records<"
            by = {
                "prod_strip": [entry("k_prod_strip<3, 2, false")],
                "prod_strip_cmp": [entry("k_prod_strip<3, 2, true")],
                "sample": [entry("k_sample<6>")],
                "hash_records": [entry(hname)],
                "decrypt": [entry("k_decrypt")],
            }
            for k, ents in by.items():
                ents = [e for e in ents if e]
                if k in rooflines and ents and n == 1344 and B == 4096:
                    rooflines[k]["traffic"] = sum(e["fetch_bytes"] + (e["write_bytes"] or 0) for e in ents) / len(ents)
                    rooflines[k]["traffic_unit"] = "HBM bytes per launch"
    except (OSError, ValueError, KeyError):
        pass
    dominant = max(rooflines, key=lambda k: kern[k]["total_ms"])
    roof = rooflines[dominant]
    # the fused AES + int8 MFMA contraction (encryption and compare launches)
    fused_product = None
    if "prod_strip" in rooflines:
        fp = rooflines["prod_strip"]
        fused_product = {"kernel": "k_prod_strip (A regenerated by AES-128-CTR in LDS, int8 MFMA)",
                         "achieved_TOPS": fp["achieved"], "peak_TOPS": PEAK_INT8_TOPS, "frac": fp["frac"],
                         "target_frac": 0.5, "avg_us": fp["avg_us"]}
        if "prod_strip_cmp" in rooflines:
            fused_product["compare_frac"] = rooflines["prod_strip_cmp"]["frac"]
            fused_product["compare_avg_us"] = rooflines["prod_strip_cmp"]["avg_us"]

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
                   "nbar": 8, "mbar": 8, "step": "keygen + encaps_batch + decaps_batch",
                   "A": "expanded once per call (unfused)" if args.unfused else "regenerated in the product (fused)"},
        "bit_exact": None,
        "batch_latency_ms": {"p50": pct(step_ms, 50), "p99": pct(step_ms, 99)},
        "lanes": S,
        "steps_per_lane": K // S if lanes_even else None,
        "lanes_even": lanes_even,
        "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]),
        "lane_side_stream": bool(args.lane_side_stream),
        "lane_hash_lanes": int(args.lane_hash_lanes),
        "lane_feed": ("library calls" if graphs is None else
                      "graph replay, one feeding thread per lane" if args.feed_threads else
                      "graph replay, issued in turn from one thread"),
        # host time from the start of the timed window until the last step was queued
        "lane_feed_ms": issue_ms.get(S if S > 1 else 1),
        "graph_matches_calls": graph_check,
        "serial": {"value": serial_value, "ms_per_step": 1e3 * wall1 / K, "feed": "library calls",
                   "batch_latency_ms": {"p50": pct(step_ms1, 50), "p99": pct(step_ms1, 99)}},
        "plain": {"value": plain_rate, "unit": "encaps+decaps/s",
                  "encaps_ms": {"p50": pct(enc_ms, 50), "p99": pct(enc_ms, 99)},
                  "decaps_ms": {"p50": pct(dec_ms, 50), "p99": pct(dec_ms, 99)},
                  "encaps_device_ms": {"p50": pct(dev_enc, 50), "p99": pct(dev_enc, 99)},
                  "decaps_device_ms": {"p50": pct(dev_dec, 50), "p99": pct(dev_dec, 99)},
                  "calls": len(enc_ms)},
        "batched_over_plain": value / plain_rate,
        "kernels": kern,
        "kernels_pipelined": kern_table(prof) if graphs is None else None,
        "roofline": roof,
        "fused_product": fused_product,
        "rooflines": rooflines,
        "cpu_baseline": None,
    }
    bit_exact = device_agree and plain_ok and graph_check is not False

    # ---------------- CPU oracle on a bounded sample ----------------
    if not args.no_cpu:
        import oracle

        op = oracle.params_for(n)
        # the oracle starts from the same seeds as the GPU, never from GPU outputs
        i_last = last_seed
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
        out["cpu_baseline"] = {
            "value": done / tcpu, "unit": "encaps+decaps/s", "cores": oracle.threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "one keygen + %d encaps+decaps pairs of the last timed n=%d step (same seeds and mu), "
                      "compared byte for byte with the GPU outputs" % (done, n)}
    out["bit_exact"] = bit_exact

    # ---------------- all-cores CPU comparator on the same workload ----------------
    if not args.no_comparator:
        import cpu_comparator

        kem = cpu_comparator.Kem(n, p.logq, p.B, p.K, p.sigma)
        i_last = last_seed
        ta = time.perf_counter()
        cpk, csk = kem.keygen_batch(seedA[i_last:i_last + 1], seedSK[i_last:i_last + 1], z[i_last:i_last + 1])
        cct, css = kem.encaps_batch(cpk[0], mus)
        css2 = kem.decaps_batch(csk[0], cct)
        tc = time.perf_counter() - ta
        same = (cpk[0].tobytes() == d_pk.cpu().numpy().tobytes() and np.array_equal(cct, d_ct.cpu().numpy())
                and np.array_equal(css, d_ss.cpu().numpy()) and np.array_equal(css, css2))
        out["cpu_comparator"] = {
            "value": B / tc, "unit": "encaps+decaps/s", "cores": cpu_comparator.threads(), "cpu_model": cpu_model(),
            "kind": "all-cores OpenMP implementation (AES-NI, AVX2), not the oracle",
            "sample": "one keygen + encaps_batch(%d) + decaps_batch(%d) of the last timed lane-0 step" % (B, B),
            "bit_exact_vs_gpu": bool(same), "gpu_over_cpu": value / (B / tc)}
        print("cpu comparator: %.1f encaps+decaps/s on %d threads" % (B / tc, cpu_comparator.threads()),
              file=sys.stderr, flush=True)

    # ---------------- energy: GPU power sampled over a longer pipelined run ----------------
    if args.energy_seconds > 0:
        ps = PowerSampler()
        if ps.source() is None:
            out["energy"] = {"error": "no GPU power source (hwmon power file or amd-smi) on this host"}
        else:
            idle = []
            for _ in range(3 if ps.path else 1):
                w = ps.read_w()
                if w is not None:
                    idle.append(w)
                time.sleep(0.05)
            done = [0] * S
            stop_at = time.perf_counter() + args.energy_seconds

            def spin(lane):
                # at most two steps queued per lane, so the run ends near its time limit (graph
                # replays return at once, and the host would otherwise queue seconds of work)
                i = 0
                marks = []
                while time.perf_counter() < stop_at:
                    step(W + (i % (2 * K)), lane)
                    ev = torch.cuda.Event()
                    ev.record(streams[lane])
                    marks.append(ev)
                    if len(marks) > 2:
                        marks.pop(0).synchronize()
                    i += 1
                done[lane] = i

            ps.start()
            torch.cuda.synchronize()
            e0 = time.perf_counter()
            th = [threading.Thread(target=spin, args=(lane,)) for lane in range(S)]
            for t in th:
                t.start()
            for t in th:
                t.join()
            torch.cuda.synchronize()
            e1 = time.perf_counter()
            ps.stop()
            ops = sum(done) * B
            pw = ps.mean_w()
            out["energy"] = {
                "source": ps.source(), "seconds": e1 - e0, "samples": len(ps.samples), "mean_power_w": pw,
                "idle_power_w": float(np.mean(idle)) if idle else None, "ops": ops,
                "ops_per_s": ops / (e1 - e0),
                "energy_j": pw * (e1 - e0) if pw is not None else None,
                "j_per_encaps_decaps": pw * (e1 - e0) / ops if pw is not None and ops else None,
                "note": "board power of the GPU while the pipelined lanes run (not the host)"}
        print("energy: %s" % json.dumps(out["energy"]), file=sys.stderr, flush=True)

    # ---------------- the other workloads (plain n=640, large n, serving) ----------------
    if not args.no_extras:
        out["extras"] = extras(args, ctx, L, torch, dev)
        if serving is not None:
            out["extras"]["serving"] = serving

    for c in ctxs:
        c.close()
    print(json.dumps(out), flush=True)
    return 0


def paper_runs(ctx, L, torch, dev, ns, reps=2):
    """The paper's parameterisation: one encryption per message bit (256 rows per
    ciphertext), prime q, DRBG noise.  Per n: wall and device time of KeyGen, Encaps and
    Decaps (hashing on the host), per-kernel device time, and the product kernel's int8 MFMA
    rate (2 limbs x 2 ops x 256 x n x n per encryption)."""
    import lwe_inputs

    runs = {}
    for n in ns:
        pid = L.param_id_paper(n)
        p = L.params(pid)
        g = lwe_inputs.rng(0, 8000 + n)
        pk = torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev)
        sk = torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev)
        ct = torch.empty(p.ct_bytes, dtype=torch.uint8, device=dev)
        ss = torch.empty(32, dtype=torch.uint8, device=dev)
        ss2 = torch.empty(32, dtype=torch.uint8, device=dev)
        wall = {"keygen": [], "encaps": [], "decaps": []}
        devt = {"keygen": [], "encaps": [], "decaps": []}
        kern = {"keygen": {}, "encaps": {}, "decaps": {}}
        ok = True
        for rep in range(reps + 1):
            sa, ssk, z = lwe_inputs.keygen_seeds(g, 1)
            mu = torch.from_numpy(lwe_inputs.messages(g, 1, 32)[0]).to(dev)
            for name, fn in (("keygen", lambda: ctx.keygen(pid, sa[0], ssk[0], z[0], pk, sk)),
                             ("encaps", lambda: ctx.encaps(pid, pk, mu, ct, ss)),
                             ("decaps", lambda: ctx.decaps(pid, sk, ct, ss2))):
                ctx.prof_reset()
                ctx.prof_enable(True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                prof = ctx.prof_read()
                ctx.prof_enable(False)
                if rep:
                    wall[name].append(1e3 * (t1 - t0))
                    devt[name].append(sum(ms for _, ms in prof.values()))
                    for k, (_, ms) in prof.items():
                        kern[name].setdefault(k, []).append(ms)
            ok &= bool(torch.equal(ss, ss2))
        r = {"q": p.q, "ct_bytes": p.ct_bytes, "decaps_agree": ok}
        for name in wall:
            r[name] = {"wall_ms": float(np.median(wall[name])), "device_ms": float(np.median(devt[name])),
                       "kernels_ms": {k: float(np.median(v)) for k, v in kern[name].items()}}
        prod = r["encaps"]["kernels_ms"].get("prod_stream", 0.0) + r["encaps"]["kernels_ms"].get("finalize", 0.0)
        if prod:
            r["encaps_product_TOPS"] = 2 * 2 * 256 * n * n / (prod * 1e-3) / 1e12
            r["encaps_product_mfma_frac"] = r["encaps_product_TOPS"] / PEAK_INT8_TOPS
        runs[str(n)] = r
        print("paper n=%d done" % n, file=sys.stderr, flush=True)
    return runs


def extras(args, ctx, L, torch, dev):
    """Plain n = 640 KEMs with p50/p99 (and the oracle on the same seeds), single large-n KEMs
    fused and unfused, and the serving workload at 0.5 and 0.8 of its measured capacity (in a
    child process with its own hardware-queue setting)."""
    import lwe_inputs

    ex = {}
    # d1: n = 640, one keygen + encaps + decaps per seed set
    n = 640
    pid = L.param_id(n)
    p = L.params(pid)
    g = lwe_inputs.rng(0, 1)
    R = args.plain640
    sa, ssk, zz = lwe_inputs.keygen_seeds(g, R)
    mus = lwe_inputs.messages(g, R, p.mu_bytes)
    d_mus = torch.from_numpy(mus).to(dev)
    pk = torch.empty(p.pk_bytes, dtype=torch.uint8, device=dev)
    sk = torch.empty(p.sk_bytes, dtype=torch.uint8, device=dev)
    ct = torch.empty(p.ct_bytes, dtype=torch.uint8, device=dev)
    s1 = torch.empty(32, dtype=torch.uint8, device=dev)
    s2 = torch.empty(32, dtype=torch.uint8, device=dev)
    lat = {"keygen": [], "encaps": [], "decaps": []}
    agree = True
    for i in range(R + 1):
        for name, fn in (("keygen", lambda: ctx.keygen(pid, sa[i % R], ssk[i % R], zz[i % R], pk, sk)),
                         ("encaps", lambda: ctx.encaps(pid, pk, d_mus[i % R], ct, s1)),
                         ("decaps", lambda: ctx.decaps(pid, sk, ct, s2))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if i:  # the first round grows the context's buffers
                lat[name].append(1e3 * (time.perf_counter() - t0))
        agree &= bool(torch.equal(s1, s2))
    kem_ms = [a + b + c for a, b, c in zip(lat["keygen"], lat["encaps"], lat["decaps"])]
    d1 = {"workload": "plain-n640", "kems": R, "kem_per_s": 1e3 * R / sum(kem_ms), "decaps_agree": agree}
    for name, v in lat.items():
        d1[name + "_ms"] = {"p50": pct(v, 50), "p99": pct(v, 99)}
    d1["kem_ms"] = {"p50": pct(kem_ms, 50), "p99": pct(kem_ms, 99)}
    if not args.no_cpu:
        import oracle

        op = oracle.params_for(n)
        i = R % R  # the last round (i = R) ran the seeds and message of index 0
        ta = time.perf_counter()
        opk, osk = oracle.kem_keygen(op, sa[i].tobytes(), ssk[i].tobytes(), zz[i].tobytes())
        oct_, oss = oracle.kem_encaps(op, opk, mus[i].tobytes())
        oss2, ok = oracle.kem_decaps(op, osk, oct_)
        tcpu = time.perf_counter() - ta
        d1["bit_exact_last"] = (opk == pk.cpu().numpy().tobytes() and osk == sk.cpu().numpy().tobytes()
                                and oct_ == ct.cpu().numpy().tobytes() and oss == s1.cpu().numpy().tobytes()
                                and ok and oss2 == oss)
        d1["oracle_kem_ms"] = 1e3 * tcpu
    ex["plain_n640"] = d1
    print("extras: n=640 plain done", file=sys.stderr, flush=True)
    # d3: single large-n KEMs, fused, and the unfused comparison at the largest n
    ns = [int(x) for x in args.large_n.split(",")]
    ex["large_fused"] = large_runs(ctx, ns, 1, False)
    ex["large_unfused"] = large_runs(ctx, ns[-1:], 1, True)
    print("extras: large n done", file=sys.stderr, flush=True)
    # the paper's own sets (Table 1): single KeyGen / Encaps / Decaps per n
    if args.paper_n:
        ex["paper_sets"] = paper_runs(ctx, L, torch, dev, [int(x) for x in args.paper_n.split(",")])
        print("extras: paper sets done", file=sys.stderr, flush=True)
    return ex


def serving_run(args):
    """The serving workload (capacity, then 0.5 and 0.8 of it) in a child process with its own
    hardware-queue count."""
    import subprocess

    cmd = [sys.executable, "-m", "paper_2606_01211_amd.serve", "--duration", str(args.serve_seconds)]
    try:
        r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=300)
        line = [x for x in r.stdout.splitlines() if x.startswith("{")]
        return json.loads(line[-1]) if r.returncode == 0 and line else {"error": r.stderr[-2000:]}
    except subprocess.TimeoutExpired:
        return {"error": "timed out"}


if __name__ == "__main__":
    sys.exit(main())
