"""Host logic of the continuous-batching server, on the CPU with a fake device backend:
grouping, admission by memory footprint, overlap of groups, continuous admission while
groups are in flight, and failure isolation."""
import threading
import time

import pytest

from paper_2606_01211_amd.serve import DECAPS, ENCAPS, KEYGEN, Backend, LweError, Server


class FakeBackend(Backend):
    def __init__(self, lanes=2, delay=0.02):
        self._lanes = lanes
        self.delay = delay
        self.active = 0
        self.max_active = 0
        self.calls = []
        self.lock = threading.Lock()

    def lanes(self):
        return self._lanes

    def run(self, lane, op, n, key, payloads):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.calls.append((op, n, key, len(payloads), time.perf_counter()))
        time.sleep(self.delay)
        with self.lock:
            self.active -= 1
        return [("r", op, n, key, p) for p in payloads]


def fp(n, op, count):
    return count * n


def test_groups_share_op_dim_and_key():
    be = FakeBackend(lanes=2, delay=0.01)
    with Server(be, hbm_budget=10**9, footprint=fp) as s:
        futs = []
        for i in range(200):
            op = (KEYGEN, ENCAPS, DECAPS)[i % 3]
            n = (640, 1344)[i % 2]
            key = i % 4
            futs.append(((op, n, key if op != KEYGEN else -1, ("p", i)), s.submit(op, n, key, ("p", i))))
        for (op, n, key, payload), f in futs:
            assert f.result(timeout=10) == ("r", op, n, key, payload)
    for op, n, key, size, _ in be.calls:
        assert size >= 1
    assert sum(c[3] for c in be.calls) == 200
    assert len(be.calls) < 200  # requests were batched


def test_admission_respects_budget_and_overlaps():
    be = FakeBackend(lanes=3, delay=0.03)
    budget = 640 * 40
    with Server(be, hbm_budget=budget, footprint=fp) as s:
        futs = [s.submit(ENCAPS, 640, i % 3, (i,)) for i in range(300)]
        for f in futs:
            f.result(timeout=20)
        assert s.max_reserved <= budget
        assert max(g[3] for g in s.groups) <= 40
    assert be.max_active >= 2  # groups of different lanes overlapped


def test_continuous_admission():
    """Requests that arrive while a group is in flight are dispatched on a free lane before
    that group finishes."""
    be = FakeBackend(lanes=2, delay=0.2)
    with Server(be, hbm_budget=10**9, footprint=fp) as s:
        f1 = s.submit(ENCAPS, 640, 0, (1,))
        time.sleep(0.05)
        t_submit = time.perf_counter()
        f2 = s.submit(ENCAPS, 976, 0, (2,))
        f2.result(timeout=5)
        f1.result(timeout=5)
    starts = {c[1]: c[4] for c in be.calls}
    assert starts[976] < starts[640] + 0.2  # second group started while the first was running
    assert starts[976] >= t_submit - 1e-3


def test_oversized_request_fails_alone():
    be = FakeBackend(lanes=2, delay=0.01)
    with Server(be, hbm_budget=1000, footprint=fp) as s:
        ok = s.submit(ENCAPS, 640, 0, ("small",))
        bad = s.submit(ENCAPS, 4096, 0, ("huge",))
        ok2 = s.submit(DECAPS, 976, 1, ("small2",))
        assert ok.result(timeout=5)[4] == ("small",)
        assert ok2.result(timeout=5)[4] == ("small2",)
        with pytest.raises(LweError):
            bad.result(timeout=5)


def test_latency_accounting_uses_arrival():
    t = [0.0]
    lock = threading.Lock()

    def clock():
        with lock:
            return t[0]

    class Instant(FakeBackend):
        def run(self, lane, op, n, key, payloads):
            with lock:
                t[0] += 0.004  # every group takes 4 ms of fake time
            return super().run(lane, op, n, key, payloads)

    be = Instant(lanes=1, delay=0.0)
    with Server(be, hbm_budget=10**9, clock=clock, footprint=fp) as s:
        f = s.submit(ENCAPS, 640, 0, ("x",), arrival=-0.001)
        f.result(timeout=5)
        lat = s.latency_ms()
    assert lat.size == 1 and lat[0] >= 4.9


class FakeMemBackend(FakeBackend):
    """Lanes that keep device memory between groups, as library contexts do: a group grows
    the lane's holding to at least its footprint and nothing shrinks until trim().  run()
    fails if the group would need more than the cap the server set for the lane, and the
    total held by all lanes is checked against the budget at every change."""

    def __init__(self, lanes, budget, base=1024, delay=0.005):
        super().__init__(lanes=lanes, delay=delay)
        self.budget = budget
        self.base = base
        self.held = [base] * lanes
        self.cap = [0] * lanes
        self.max_total = sum(self.held)
        self.trim_calls = 0

    def held_bytes(self, lane):
        return self.held[lane]

    def limit_lane(self, lane, cap):
        self.cap[lane] = cap

    def trim(self, lane):
        with self.lock:
            self.held[lane] = self.base
            self.trim_calls += 1

    def call_bytes(self, n, op, count):
        return self.base + count * n

    def run(self, lane, op, n, key, payloads):
        need = self.call_bytes(n, op, len(payloads))
        with self.lock:
            grown = self.held[lane] + need - self.base if self.held[lane] < need else self.held[lane]
            if self.cap[lane] and grown > self.cap[lane]:
                raise LweError("over the lane cap")
            self.held[lane] = grown
            self.max_total = max(self.max_total, sum(self.held))
            assert sum(self.held) <= self.budget
        return super().run(lane, op, n, key, payloads)


def test_admission_bounds_memory_held_between_groups():
    """Lanes keep what they allocated (the largest group they ran); the server admits by
    those real holdings, trims idle lanes when they block a group, and the memory held by
    all lanes together never exceeds the budget."""
    budget = 3 * 1024 + 4096 * 12
    be = FakeMemBackend(lanes=3, budget=budget)
    with Server(be, hbm_budget=budget, max_batch=64) as s:
        futs = []
        for i in range(400):
            n = (640, 976, 4096)[i % 3]
            futs.append(s.submit((ENCAPS, DECAPS)[i % 2], n, i % 2, (i,)))
        for f in futs:
            f.result(timeout=30)
        assert s.max_reserved <= budget and s.max_held <= budget
    assert be.max_total <= budget
    assert be.trim_calls > 0  # holdings of idle lanes had to be released
    assert max(g[3] for g in s.groups) > 1


def test_lanes_arriving_over_budget_are_released_first():
    """Lanes that still hold buffers grown under an earlier, larger server are trimmed when a
    server with a smaller budget starts, so its budget bounds the held memory from the start."""
    budget = 3 * 1024 + 4096 * 6
    be = FakeMemBackend(lanes=3, budget=10**9)
    be.held = [1024 + 4096 * 40, 1024 + 4096 * 20, 1024]  # left over from a bigger server
    be.budget = budget
    with Server(be, hbm_budget=budget, max_batch=64) as s:
        assert s.max_reserved <= budget
        futs = [s.submit(ENCAPS, 640, i % 2, (i,)) for i in range(40)]
        for f in futs:
            f.result(timeout=30)
        assert s.max_reserved <= budget and s.max_held <= budget
    assert be.trim_calls >= 3


def test_request_above_the_floor_fails_alone_without_spinning():
    """Every lane keeps a floor that trimming cannot release (its AES table).  A request that
    fits the budget only if that floor were released too fails alone with LWE_ENOMEM; the
    scheduler neither spins nor stalls, and later requests that fit are still served."""
    be = FakeMemBackend(lanes=3, budget=10**9)
    tiny = be.call_bytes(640, ENCAPS, 1) + 2 * be.base - 1
    be.budget = tiny
    with Server(be, hbm_budget=tiny, max_batch=64) as s:
        f = s.submit(ENCAPS, 640, 0, (0,))
        with pytest.raises(LweError):
            f.result(timeout=10)
        g = s.submit(ENCAPS, 320, 0, (1,))
        assert g.result(timeout=10)[0] == "r"
