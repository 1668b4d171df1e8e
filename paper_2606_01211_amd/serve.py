"""Continuous-batching KEM server over the C ABI.

Requests (KeyGen, Encaps, Decaps) of different lattice dimensions arrive at any time.  A
scheduler thread groups the queued requests that can share one library call -- the same
operation, dimension and (for Encaps / Decaps) the same resident key pair -- and hands each
group to one of several worker lanes.  Every lane owns its own library context and HIP
stream, so batches of different lanes run concurrently on the device, and a request that
arrives while others are in flight joins the next group as soon as a lane and enough device
memory are free.  Admission is by HBM footprint: the bytes a batch needs are reserved
against the server's budget before it is dispatched and released when it completes; a group
that does not fit is split, and a single request that can never fit fails alone with
LWE_ENOMEM.

Key pairs are generated once at start-up and stay resident on the device (torch uint8
tensors); only messages, ciphertexts and shared secrets cross PCIe.

Latency of a request = completion time - arrival time (the time submit() was called, or the
arrival stamp supplied by a load generator).  The scheduler never changes the arithmetic:
each request's result is byte-identical to the same request executed alone.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import gc
import heapq
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

KEYGEN, ENCAPS, DECAPS = 0, 1, 2
OP_NAMES = {KEYGEN: "keygen", ENCAPS: "encaps", DECAPS: "decaps"}
# group sizes whose exact footprint the library backend tabulates when it starts
CALL_BYTES_TABLE = 4096


@dataclass
class Request:
    op: int
    n: int
    key: int                       # resident key pair index (Encaps / Decaps); ignored for KeyGen
    payload: Tuple                 # KeyGen: (seedA, seedSK, z); Encaps: (mu,); Decaps: (ct,)
    arrival: float = 0.0           # seconds (server clock)
    future: cf.Future = field(default_factory=cf.Future)
    start: float = 0.0             # dispatch time
    done: float = 0.0              # completion time
    batch_size: int = 0


class LweError(RuntimeError):
    pass


def footprint_bytes(n: int, op: int, count: int) -> int:
    """Device bytes one library call needs for `count` instances of `op` at dimension n
    (operand and error stacks, round keys, staged inputs and outputs; upper bound)."""
    ldx = (n + 63) // 64 * 64
    pk = 16 + 16 * n
    sk = 16 * n + pk + 64
    ct = 16 * n + 128
    per = 8 * ldx + 8 * n + 64 + 44 * 4 + 16 + 32 + 32 + 64 + 8
    if op == KEYGEN:
        per += pk + sk + 64
    elif op == ENCAPS:
        per += ct + 64 + 32
    else:
        per += 2 * ct + 64 + 32
    # split-K accumulator of the streaming product for small groups
    acc = 8 * count * (n + 8) * 4 if count * 8 < 256 else 0
    return count * per + acc + (1 << 20)


class Backend:
    """What the scheduler needs from the device side (the real one is LibraryBackend).

    Memory: a lane holds held_bytes(lane) of device memory between groups; before a group the
    server calls limit_lane(lane, cap) with the most the lane may hold until that group
    completes, and may call trim(lane) on an idle lane to release what it holds.  A backend
    without device memory of its own keeps the defaults (nothing held, no limits)."""

    def lanes(self) -> int:
        raise NotImplementedError

    def run(self, lane: int, op: int, n: int, key: int, payloads: List[Tuple]) -> List:
        raise NotImplementedError

    def held_bytes(self, lane: int) -> int:
        return 0

    def limit_lane(self, lane: int, cap: int) -> None:
        pass

    def trim(self, lane: int) -> None:
        pass

    def call_bytes(self, n: int, op: int, count: int) -> Optional[int]:
        """Device bytes one group needs starting from a trimmed lane (None: unknown)."""
        return None


class Server:
    """Continuous-batching scheduler.

    backend     executes one group on a lane and returns one result per request
    hbm_budget  bytes of device memory all lanes together may hold
    max_batch   largest group handed to one library call
    clock       time source (seconds); injectable for tests
    footprint   bytes one group needs; default: the backend's call_bytes, else an estimate

    Admission: every lane has a commitment, the device memory it holds when idle and, while
    it runs a group, the cap the backend enforces for that group (what it held plus the
    group's footprint, or the footprint alone after trimming the lane).  A group is dispatched
    only when the commitments stay within hbm_budget, so the memory the lanes really hold
    never exceeds it.
    """

    def __init__(self, backend: Backend, hbm_budget: int, max_batch: int = 4096,
                 clock: Callable[[], float] = time.perf_counter,
                 footprint: Optional[Callable[[int, int, int], int]] = None):
        self.backend = backend
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.clock = clock
        if footprint is None:
            footprint = footprint_bytes if backend.call_bytes(640, ENCAPS, 1) is None else backend.call_bytes
        self.footprint = footprint
        self._queues: Dict[Tuple[int, int, int], collections.deque] = {}
        # (arrival of the queue head, sequence, queue key) of every non-empty queue: the
        # oldest waiting request's queue is the heap minimum
        self._heads: List[Tuple[float, int, Tuple[int, int, int]]] = []
        self._seq = 0
        self._cv = threading.Condition()
        self._free_lanes = list(range(backend.lanes()))
        # Lanes may arrive holding buffers grown under an earlier server; when those exceed
        # this server's budget they are released first, so the budget bounds the memory the
        # lanes hold from the start.
        if sum(int(backend.held_bytes(lane)) for lane in range(backend.lanes())) > self.budget:
            for lane in range(backend.lanes()):
                backend.trim(lane)
        self._commit = [int(backend.held_bytes(lane)) for lane in range(backend.lanes())]
        self._reserved = sum(self._commit)
        self.max_reserved = self._reserved
        self.max_held = self._reserved  # largest total after a group completed (idle lanes' real bytes)
        self.trims = 0
        self.max_in_flight_groups = 0
        self._in_flight = 0
        self._stop = False
        self._paused = False
        self._pool = cf.ThreadPoolExecutor(max_workers=backend.lanes(), thread_name_prefix="lwe-lane")
        self._sched = threading.Thread(target=self._loop, name="lwe-scheduler", daemon=True)
        self.completed: List[Request] = []
        self.groups: List[Tuple[int, int, int, int]] = []  # (op, n, key, size) per dispatched group
        self._sched.start()

    # ---- client side ----
    def submit(self, op: int, n: int, key: int, payload: Tuple, arrival: Optional[float] = None) -> cf.Future:
        r = Request(op, n, key if op != KEYGEN else -1, payload,
                    arrival=self.clock() if arrival is None else arrival)
        with self._cv:
            if self._stop:
                raise RuntimeError("server stopped")
            k = (op, n, r.key)
            q = self._queues.get(k)
            if q is None:
                q = self._queues[k] = collections.deque()
            if not q:
                self._push_head(r.arrival, k)
            q.append(r)
            self._cv.notify_all()
        return r.future

    def _push_head(self, arrival: float, k: Tuple[int, int, int]) -> None:
        self._seq += 1
        heapq.heappush(self._heads, (arrival, self._seq, k))

    def close(self) -> None:
        with self._cv:
            self._stop = True
            self._paused = False
            self._cv.notify_all()
        self._sched.join()
        self._pool.shutdown(wait=True)
        for lane in range(self.backend.lanes()):
            self.backend.limit_lane(lane, 0)  # the lanes leave the server without a cap

    def pause(self) -> None:
        """Holds dispatching (requests keep queueing) until resume(): lets a caller submit a
        burst that the scheduler then sees whole."""
        with self._cv:
            self._paused = True

    def resume(self) -> None:
        with self._cv:
            self._paused = False
            self._cv.notify_all()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- scheduler ----
    def _pick_group(self, lane: int) -> Optional[Tuple[Tuple[int, int, int], List[Request], int, bool]]:
        """Oldest queue head first; as many of its requests as fit the budget on idle lane
        `lane`.  Returns (queue key, requests, cap for the lane, trim the lane first)."""
        while True:
            while self._heads:
                arrival, seq, best = self._heads[0]
                q = self._queues.get(best)
                if not q or q[0].arrival != arrival:  # stale entry
                    heapq.heappop(self._heads)
                    continue
                break
            else:
                return None
            op, n, key = best
            held = self._commit[lane]  # idle: what it really holds
            avail = self.budget - (self._reserved - held)
            take = min(len(q), self.max_batch)
            trim = False
            while take > 0:
                need = self.footprint(n, op, take)
                if held + need <= avail:
                    break
                if need <= avail and held > 0:
                    trim = True  # fits once the lane has released what it holds
                    break
                take //= 2
            if take > 0:
                heapq.heappop(self._heads)
                reqs = [q.popleft() for _ in range(take)]
                if q:
                    self._push_head(q[0].arrival, best)
                need = self.footprint(n, op, take)
                return best, reqs, (need if trim else held + need), trim
            if self._in_flight:
                return None  # wait for a group to complete and release its reservation
            # every lane is idle: release what idle lanes hold and try again, unless that frees
            # nothing (each lane keeps a floor, its AES table) -- then the head request can
            # never fit, and it fails alone
            idle_held = sum(self._commit[x] for x in self._free_lanes)
            if self.footprint(n, op, 1) <= self.budget - (self._reserved - idle_held) and idle_held:
                for x in self._free_lanes:
                    self._trim_lane(x)
                if sum(self._commit[x] for x in self._free_lanes) < idle_held:
                    continue
            heapq.heappop(self._heads)
            r = q.popleft()
            if q:
                self._push_head(q[0].arrival, best)
            r.future.set_exception(LweError("request needs more device memory than the budget (LWE_ENOMEM)"))

    def _trim_lane(self, lane: int) -> None:
        """Releases an idle lane's memory (caller holds the lock)."""
        self.backend.trim(lane)
        held = int(self.backend.held_bytes(lane))
        self._reserved += held - self._commit[lane]
        self._commit[lane] = held
        self.trims += 1

    def _loop(self) -> None:
        while True:
            with self._cv:
                while True:
                    if self._stop and not any(self._queues.values()) and self._in_flight == 0:
                        return
                    if self._free_lanes and not self._paused:
                        g = self._pick_group(self._free_lanes[-1])
                        if g is not None:
                            break
                    self._cv.wait(timeout=0.05)
                (op, n, key), reqs, cap, trim = g
                lane = self._free_lanes.pop()
                # The lane's worker trims it and sets its cap: no backend call here, under the
                # lock (a foreign call may wait a whole switch interval for the interpreter
                # lock, and every dispatch would wait with it).  Until the worker has trimmed
                # the lane it still holds what it held, so the reservation covers both.
                res = max(cap, self._commit[lane]) if trim else cap
                self._reserved += res - self._commit[lane]
                self._commit[lane] = res
                self._in_flight += 1
                self.max_reserved = max(self.max_reserved, self._reserved)
                self.max_in_flight_groups = max(self.max_in_flight_groups, self._in_flight)
                self.groups.append((op, n, key, len(reqs)))
                if trim:
                    self.trims += 1
            self._pool.submit(self._run_group, lane, op, n, key, reqs, cap, trim)

    def _run_group(self, lane: int, op: int, n: int, key: int, reqs: List[Request], cap: int = 0,
                   trim: bool = False) -> None:
        if trim:
            self.backend.trim(lane)
            cap = max(cap, int(self.backend.held_bytes(lane)))  # the floor trimming keeps
        self.backend.limit_lane(lane, cap)
        t0 = self.clock()
        for r in reqs:
            r.start = t0
            r.batch_size = len(reqs)
        try:
            results = self.backend.run(lane, op, n, key, [r.payload for r in reqs])
            err = None
        except Exception as e:  # the whole group failed: report it to each of its requests
            results, err = None, e
        t1 = self.clock()
        held = int(self.backend.held_bytes(lane))  # the lane is idle again: what it really holds
        with self._cv:
            self._reserved += held - self._commit[lane]
            self._commit[lane] = held
            self.max_held = max(self.max_held, self._reserved)
            self._in_flight -= 1
            self._free_lanes.append(lane)
            for i, r in enumerate(reqs):
                r.done = t1
                self.completed.append(r)
            self._cv.notify_all()
        for i, r in enumerate(reqs):
            if err is not None:
                r.future.set_exception(err)
            else:
                r.future.set_result(results[i])

    # ---- statistics ----
    def latency_ms(self, op: Optional[int] = None) -> np.ndarray:
        with self._cv:
            return np.array([1e3 * (r.done - r.arrival) for r in self.completed if op is None or r.op == op])


class LibraryBackend(Backend):
    """Runs groups through liblwe_hip: one context and one HIP stream per lane, key pairs
    resident on the device."""

    def __init__(self, ns, keys_per_n: int = 16, lanes: int = 3, device: int = 0,
                 lane_budget: int = 0, key_seed: int = 4, keys: Optional[Dict] = None):
        import torch

        import lwe_inputs
        from . import lwe

        self.torch = torch
        self.L = lwe
        self.dev = torch.device("cuda:%d" % device)
        self._lanes = [lwe.Context(device, lane_budget) for _ in range(lanes)]
        # each lane runs on its context's own stream; with the context's second stream (the
        # decapsulation hash) that is two streams per lane, each given a hardware queue
        self._streams = [c.stream_handle for c in self._lanes]
        self.pids = {n: lwe.param_id(n) for n in ns}
        # The library's exact footprint depends only on (set, op, count) and the tuning.  The
        # scheduler asks for it under its lock for every candidate group, so the table is
        # filled here: a foreign call there waits for the interpreter lock, which the other
        # threads may hold for a whole switch interval, and it stalls every dispatch.
        self._call_bytes: Dict[Tuple[int, int, int], int] = {}
        for n in ns:
            for op in (KEYGEN, ENCAPS, DECAPS):
                for count in range(1, CALL_BYTES_TABLE + 1):
                    self._call_bytes[(n, op, count)] = self._lanes[0].call_bytes(self.pids[n], op, count)
        self.params = {n: lwe.params(self.pids[n]) for n in ns}
        self.keys: Dict[int, List[Tuple]] = {}
        g = lwe_inputs.rng(key_seed, 0)
        for n in ns:
            p = self.params[n]
            if keys is not None:  # key pairs supplied by the caller: {n: (pk[k][..], sk[k][..])}
                pk, sk = (np.ascontiguousarray(x, np.uint8) for x in keys[n])
            else:
                seedA, seedSK, z = lwe_inputs.keygen_seeds(g, keys_per_n)
                pk = np.zeros((keys_per_n, p.pk_bytes), np.uint8)
                sk = np.zeros((keys_per_n, p.sk_bytes), np.uint8)
                self._lanes[0].keygen_batch(p.pid, keys_per_n, seedA, seedSK, z, pk, sk)
            self.keys[n] = [(torch.from_numpy(pk[i].copy()).to(self.dev), torch.from_numpy(sk[i].copy()).to(self.dev),
                             pk[i].copy(), sk[i].copy()) for i in range(keys_per_n)]
        torch.cuda.synchronize()

    def lanes(self) -> int:
        return len(self._lanes)

    def held_bytes(self, lane: int) -> int:
        return self._lanes[lane].device_bytes

    def limit_lane(self, lane: int, cap: int) -> None:
        self._lanes[lane].set_budget(0 if cap <= 0 else max(int(cap), 1024))

    def trim(self, lane: int) -> None:
        self._lanes[lane].trim()

    def call_bytes(self, n: int, op: int, count: int) -> Optional[int]:
        k = (n, op, count)
        b = self._call_bytes.get(k)
        if b is None:
            b = self._call_bytes[k] = self._lanes[0].call_bytes(self.pids[n], op, count)
        return b

    def host_key(self, n: int, key: int):
        return self.keys[n][key][2], self.keys[n][key][3]

    def run(self, lane: int, op: int, n: int, key: int, payloads: List[Tuple]) -> List:
        ctx, st = self._lanes[lane], self._streams[lane]
        p = self.params[n]
        c = len(payloads)
        if op == KEYGEN:
            seedA = np.stack([np.frombuffer(bytes(x[0]), np.uint8) for x in payloads])
            seedSK = np.stack([np.frombuffer(bytes(x[1]), np.uint8) for x in payloads])
            z = np.stack([np.frombuffer(bytes(x[2]), np.uint8) for x in payloads])
            pk = np.zeros((c, p.pk_bytes), np.uint8)
            sk = np.zeros((c, p.sk_bytes), np.uint8)
            ctx.keygen_batch(p.pid, c, seedA, seedSK, z, pk, sk, stream=st)
            return [(pk[i].tobytes(), sk[i].tobytes()) for i in range(c)]
        d_pk, d_sk = self.keys[n][key][0], self.keys[n][key][1]
        if op == ENCAPS:
            mu = np.stack([np.frombuffer(bytes(x[0]), np.uint8) for x in payloads])
            ct = np.zeros((c, p.ct_bytes), np.uint8)
            ss = np.zeros((c, 32), np.uint8)
            ctx.encaps_batch(p.pid, c, d_pk, mu, ct, ss, stream=st)
            return [(ct[i].tobytes(), ss[i].tobytes()) for i in range(c)]
        cts = np.stack([np.frombuffer(bytes(x[0]), np.uint8) for x in payloads])
        ss = np.zeros((c, 32), np.uint8)
        ctx.decaps_batch(p.pid, c, d_sk, cts, ss, stream=st)
        return [ss[i].tobytes() for i in range(c)]

    def close(self) -> None:
        for c in self._lanes:
            c.close()


# ---------------------------------------------------------------------------------------
# Load generator (the serving workload: Poisson arrivals, mixed ops and dimensions)
# ---------------------------------------------------------------------------------------
def run_load(server: Server, backend: LibraryBackend, qps: float, duration_s: float, ns, keys_per_n: int,
             mix=(0.2, 0.5, 0.3), seed: int = 0, ct_pool: Optional[Dict] = None) -> Dict:
    """Open-loop load: requests arrive at Poisson times regardless of completions.  Decaps
    requests use ciphertexts produced by earlier Encaps of the same key (a pool seeded
    before the run).  Returns throughput and latency percentiles."""
    import lwe_inputs

    g = lwe_inputs.rng(4, 100 + seed)
    count = max(1, int(qps * duration_s))
    arrivals = lwe_inputs.poisson_arrivals(g, qps, count)
    ops, nsel = lwe_inputs.request_mix(g, count, ns, mix)
    keys = g.integers(0, keys_per_n, size=count)
    if ct_pool is None:
        ct_pool = prime_ct_pool(backend, ns, keys_per_n)
    # every payload is drawn before the clock starts, so the generator only submits
    payloads = []
    for i in range(count):
        op, n, key = int(ops[i]), int(nsel[i]), int(keys[i])
        p = backend.params[n]
        if op == KEYGEN:
            sa, ss_, z = lwe_inputs.keygen_seeds(g, 1)
            payloads.append((sa[0].tobytes(), ss_[0].tobytes(), z[0].tobytes()))
        elif op == ENCAPS:
            payloads.append((lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes(),))
        else:
            pool = ct_pool[(n, key)]
            payloads.append((pool[i % len(pool)],))
    # The collector stays off while requests are in flight: a full collection over tens of
    # thousands of live requests and futures would stall every thread of the server.
    gc.collect()
    gc_was = gc.isenabled()
    gc.disable()
    try:
        futs = []
        t0 = server.clock()
        for i in range(count):
            target = t0 + arrivals[i]
            while True:
                now = server.clock()
                if now >= target:
                    break
                time.sleep(min(0.0005, target - now))
            futs.append((int(ops[i]), server.submit(int(ops[i]), int(nsel[i]), int(keys[i]), payloads[i],
                                                    arrival=target)))
        for _, f in futs:
            f.result()
        t1 = server.clock()
    finally:
        if gc_was:
            gc.enable()
    lat = {OP_NAMES[o]: server.latency_ms(o) for o in (KEYGEN, ENCAPS, DECAPS)}
    allat = server.latency_ms()
    return {
        "requests": count,
        "offered_qps": qps,
        "achieved_ops_per_s": count / (t1 - t0),
        "p50_ms": float(np.percentile(allat, 50)),
        "p99_ms": float(np.percentile(allat, 99)),
        "per_op": {k: {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
                       "count": int(v.size)} for k, v in lat.items() if v.size},
        "mean_group": float(np.mean([gsz[3] for gsz in server.groups])) if server.groups else 0.0,
        "max_reserved_bytes": server.max_reserved,
        "budget_bytes": server.budget,
        "max_concurrent_groups": server.max_in_flight_groups,
    }


def prime_ct_pool(backend: LibraryBackend, ns, keys_per_n: int, per_key: int = 4) -> Dict:
    """Ciphertexts for the Decaps requests: `per_key` encapsulations per resident key."""
    import lwe_inputs

    g = lwe_inputs.rng(4, 7)
    pool = {}
    for n in ns:
        p = backend.params[n]
        for key in range(keys_per_n):
            mus = [(lwe_inputs.messages(g, 1, p.mu_bytes)[0].tobytes(),) for _ in range(per_key)]
            res = backend.run(0, ENCAPS, n, key, mus)
            pool[(n, key)] = [r[0] for r in res]
    return pool


def main(argv=None) -> int:
    import argparse
    import json

    ap = argparse.ArgumentParser(description="Continuous-batching KEM serving benchmark (one GPU)")
    ap.add_argument("--ns", default="640,976,1344,4096")
    ap.add_argument("--keys-per-n", type=int, default=16)
    ap.add_argument("--lanes", type=int, default=8)
    ap.add_argument("--qps", type=float, default=0.0, help="offered load; 0 = measure capacity first")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--max-batch", type=int, default=1024)
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="HIP hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32; default "
                         "2 * lanes + 2), so that both streams of every lane have a queue of their own")
    args = ap.parse_args(argv)
    import os

    hwq = args.hw_queues if args.hw_queues > 0 else 2 * max(1, args.lanes) + 2
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(1, hwq)))  # before the GPU is used
    ns = [int(x) for x in args.ns.split(",")]
    be = LibraryBackend(ns, args.keys_per_n, args.lanes)
    pool = prime_ct_pool(be, ns, args.keys_per_n)
    out = {"ns": ns, "keys_per_n": args.keys_per_n, "lanes": args.lanes, "mix": [0.2, 0.5, 0.3],
           "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"])}
    budget = int(args.budget_gb * (1 << 30))
    if args.qps <= 0:
        # capacity: a closed burst of requests all arriving at t = 0
        with Server(be, budget, args.max_batch) as s:
            r = run_load(s, be, 1e9, 2000 / 1e9, ns, args.keys_per_n, ct_pool=pool)
        cap = r["achieved_ops_per_s"]
        out["capacity_ops_per_s"] = cap
        runs = {}
        for frac in (0.5, 0.8):
            with Server(be, budget, args.max_batch) as s:
                runs["%.1fC" % frac] = run_load(s, be, frac * cap, args.duration, ns, args.keys_per_n, ct_pool=pool)
        out["runs"] = runs
    else:
        with Server(be, budget, args.max_batch) as s:
            out["runs"] = {"qps=%g" % args.qps: run_load(s, be, args.qps, args.duration, ns, args.keys_per_n,
                                                          ct_pool=pool)}
    be.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
