"""Host logic of the serving loop (continuous batching, HBM admission, plan LRU),
driven by a simulated executor: no GPU."""
import collections

import numpy as np
import pytest

from paper_2311_14670_amd.serving import PlanKey, Request, Scheduler, serve, latency_stats, key_of
from paper_2311_14670_amd.synth import serving_trace


class FakeHandle:
    def __init__(self, requests, ready_at):
        self.requests, self.ready_at = requests, ready_at


class FakeExecutor:
    """Streams finish a batch after `cost(key, n)` simulated seconds."""

    def __init__(self, clock, n_streams=2, max_batch=4, plan_bytes=1000, ws_bytes=100):
        self.clock, self.n_streams, self.max_batch = clock, n_streams, max_batch
        self.pb, self.wb = plan_bytes, ws_bytes
        self.plans = collections.OrderedDict()
        self.ws = set()
        self.pending = []
        self.launches = []
        self.peak = 0
        self.sched = None

    def batch_limit(self, key):
        return self.max_batch

    def new_bytes(self, key):
        if key not in self.plans:
            self.plans[key] = True
            return self.wb
        return 0 if key in self.ws else self.wb

    def resident_bytes(self):
        return len(self.plans) * self.pb + len(self.ws) * self.wb

    def free_streams(self):
        return self.n_streams - len(self.pending)

    def evict(self, nbytes, busy):
        freed = 0
        for k in list(self.plans):
            if freed >= nbytes:
                break
            if k in busy:
                continue
            del self.plans[k]
            freed += self.pb
            if k in self.ws:
                self.ws.discard(k)
                freed += self.wb
        return freed

    def launch(self, key, reqs):
        assert len(self.pending) < self.n_streams
        self.plans.move_to_end(key)
        self.ws.add(key)
        h = FakeHandle(reqs, self.clock.t + 0.001 * key.L * len(reqs))
        self.pending.append(h)
        self.launches.append((key, [r.rid for r in reqs]))
        if self.sched is not None:
            self.peak = max(self.peak, self.sched.in_use + Scheduler.buffer_bytes(key, len(reqs))
                            + self.resident_bytes())
        return h

    def poll(self):
        fin = [h for h in self.pending if h.ready_at <= self.clock.t]
        for h in fin:
            self.pending.remove(h)
        return fin


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


def _req(rid, L, t=0.0, spin=0, sampling="mw"):
    key = PlanKey("s2", L, spin, 1, sampling, L // 2 if sampling == "healpix" else 0)
    return Request(rid=rid, key=key, data=np.zeros((L, 2 * L - 1), complex), t_arrival=t)


def test_batches_group_same_key_in_fifo_order():
    clk = Clock()
    ex = FakeExecutor(clk, n_streams=1, max_batch=3)
    s = Scheduler(ex, hbm_budget=1 << 40)
    reqs = [_req(0, 8), _req(1, 16), _req(2, 8), _req(3, 8), _req(4, 8), _req(5, 16)]
    serve(s, reqs, clock=clk, realtime=False, sleep=clk.sleep)
    assert [ids for _, ids in ex.launches] == [[0, 2, 3], [1, 5], [4]]
    for key, ids in ex.launches:
        assert all(reqs[i].key == key for i in ids)
    assert len(s.done) == 6 and not s.rejected


def test_admission_respects_budget_and_rejects_oversized():
    clk = Clock()
    ex = FakeExecutor(clk, n_streams=4, max_batch=8, plan_bytes=10, ws_bytes=10)
    per = Scheduler.buffer_bytes(_req(0, 16).key, 1)
    budget = 3 * per + 100
    s = Scheduler(ex, hbm_budget=budget)
    ex.sched = s
    reqs = [_req(i, 16, t=0.0) for i in range(10)] + [_req(99, 64)]   # L=64 cannot fit
    serve(s, reqs, clock=clk, realtime=False, sleep=clk.sleep)
    assert ex.peak <= budget
    assert [r.rid for r in s.rejected] == [99]
    assert sorted(r.rid for r in s.done) == list(range(10))
    assert max(len(ids) for _, ids in ex.launches) <= 3


def test_lru_eviction_makes_room_for_new_plan():
    clk = Clock()
    ex = FakeExecutor(clk, n_streams=1, max_batch=1, plan_bytes=10_000, ws_bytes=0)
    per = Scheduler.buffer_bytes(_req(0, 8).key, 1)
    s = Scheduler(ex, hbm_budget=2 * 10_000 + per + 10)
    reqs = [_req(0, 8), _req(1, 10), _req(2, 12), _req(3, 8)]
    serve(s, reqs, clock=clk, realtime=False, sleep=clk.sleep)
    assert len(s.done) == 4 and not s.rejected
    assert len(ex.plans) <= 2


def test_realtime_latency_accounting():
    clk = Clock()
    ex = FakeExecutor(clk, n_streams=2, max_batch=4)
    s = Scheduler(ex, hbm_budget=1 << 40)
    reqs = [_req(i, 8, t=0.01 * i) for i in range(20)]
    wall = serve(s, reqs, clock=clk, realtime=True, sleep=clk.sleep)
    st = latency_stats(s.done)
    assert st["n"] == 20 and st["p50_ms"] >= 0 and st["p99_ms"] >= st["p50_ms"]
    assert all(r.t_launch >= r.t_arrival and r.t_done >= r.t_launch for r in s.done)
    assert wall >= 0.19


def test_trace_keys():
    tr = serving_trace(n_requests=500, seed=3)
    keys = [key_of(t) for t in tr]
    assert all(k.L % 2 == 0 and 64 <= k.L <= 4096 for k in keys)
    so3 = [k for k in keys if k.kind == "so3"]
    assert so3 and all(k.L <= 512 and k.N in (1, 4, 8) for k in so3)
    hp = [k for k in keys if k.sampling == "healpix"]
    assert hp and all(k.nside == k.L // 2 for k in hp)
    ts = [t["t"] for t in tr]
    assert ts == sorted(ts)


def test_busy_key_waits_while_other_keys_launch():
    """A key whose single workspace is in flight waits; later requests of other
    keys take the free stream meanwhile (executor with one workspace per key)."""
    clk = Clock()

    class OneWorkspace(FakeExecutor):
        def can_launch(self, key):
            return self.free_streams() > 0 and all(h.requests[0].key != key for h in self.pending)

    ex = OneWorkspace(clk, n_streams=2, max_batch=1)
    s = Scheduler(ex, hbm_budget=1 << 40)
    reqs = [_req(0, 8), _req(1, 8), _req(2, 16)]
    serve(s, reqs, clock=clk, realtime=False, sleep=clk.sleep)
    assert [ids for _, ids in ex.launches] == [[0], [2], [1]]
    assert len(s.done) == 3 and not s.rejected


def test_waiting_key_keeps_its_plan_under_pressure():
    """A key that waits for in-flight memory keeps the plan its admission check
    built: eviction never drops the key being admitted, so the plan is created
    once, not once per pass of the serve loop."""
    clk = Clock()

    class Counting(FakeExecutor):
        def __init__(self, *a, **kw):
            super().__init__(*a, **kw)
            self.created = collections.Counter()

        def new_bytes(self, key):
            if key not in self.plans:
                self.created[key] += 1
            return super().new_bytes(key)

    ex = Counting(clk, n_streams=2, max_batch=1, plan_bytes=100, ws_bytes=0)
    small, big = _req(0, 16), _req(1, 32)
    budget = Scheduler.buffer_bytes(big.key, 1) + 2 * 100 + 50     # big fits only once small is done
    s = Scheduler(ex, hbm_budget=budget)
    serve(s, [small, big], clock=clk, realtime=False, sleep=clk.sleep)
    assert len(s.done) == 2 and not s.rejected
    assert [ids for _, ids in ex.launches] == [[0], [1]]
    assert ex.created[big.key] == 1, ex.created


class MixedExecutor(FakeExecutor):
    """A matrix-core batch below two requests runs on the key's FP64 plan."""

    def run_key(self, key, n):
        import dataclasses
        return dataclasses.replace(key, precision="fp64") if key.precision != "fp64" and n < 2 else key


def test_small_matrix_core_batches_run_on_the_fp64_plan():
    import dataclasses
    clock = Clock()
    ex = MixedExecutor(clock, n_streams=1, max_batch=4)
    sched = Scheduler(ex, hbm_budget=10 ** 9)
    ex.sched = sched
    split = PlanKey("s2", 64, 0, 1, "mw", 0, "split_bf16")
    reqs = [Request(rid=0, key=split, data=None, t_arrival=0.0),                       # alone: FP64 plan
            Request(rid=1, key=dataclasses.replace(split, L=96), data=None, t_arrival=1.0),
            Request(rid=2, key=dataclasses.replace(split, L=96), data=None, t_arrival=1.0)]  # a pair: matrix cores
    serve(sched, reqs, clock=clock, sleep=clock.sleep)
    assert len(sched.done) == 3 and not sched.rejected
    keys = [k for k, _ in ex.launches]
    assert keys[0] == dataclasses.replace(split, precision="fp64")
    assert keys[1] == dataclasses.replace(split, L=96) and ex.launches[1][1] == [1, 2]
    assert [r.run_precision for r in sorted(sched.done, key=lambda r: r.rid)] == ["fp64", "split_bf16", "split_bf16"]
    # the plan in use is the one admitted and cached
    assert dataclasses.replace(split, precision="fp64") in ex.plans
