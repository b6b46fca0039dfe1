"""Serving loop for transform requests on one GPU: continuous batching with
HBM admission control, several HIP streams, and a plan cache.

A request is one round trip -- inverse then forward -- of a spin SHT (MW or
HEALPix) or a Wigner (SO(3)) transform.  The loop

  * admits arrivals into a FIFO queue;
  * forms a batch from the oldest waiting request and every later waiting
    request with the same plan key (L, spin, N, sampling, nside, precision),
    up to the key's batch limit;
  * launches it on a free stream when its device footprint (workspace, input
    and output buffers, plus the plan's constants if the plan is not cached)
    fits the HBM budget next to what is in flight;
  * polls completion events and records submit -> complete latency.

Each request's result is independent of the batch it was served in: every
map of a batch goes through the same kernels with the same arithmetic order,
so a request gives bit-identical results alone or in any mix.

The scheduling logic (``Scheduler``) is device-free and is driven by an
executor object; ``GpuExecutor`` runs batches through the library's C ABI.
"""
import collections
import dataclasses
import itertools
import time

import numpy as np

__all__ = ["Request", "PlanKey", "Scheduler", "GpuExecutor", "serve", "latency_stats"]


@dataclasses.dataclass(frozen=True)
class PlanKey:
    kind: str          # "s2" or "so3"
    L: int
    spin: int
    N: int
    sampling: str      # "mw" or "healpix"
    nside: int
    precision: str = "fp64"


@dataclasses.dataclass
class Request:
    rid: int
    key: PlanKey
    data: np.ndarray            # complex128 coefficients ([L, 2L-1] or [2N-1, L, 2L-1])
    t_arrival: float = 0.0      # seconds, relative to the start of the run
    t_launch: float = None
    t_done: float = None
    result: np.ndarray = None
    error: str = None
    batch_size: int = 0

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival


def key_of(spec):
    """PlanKey from a trace entry (dict with kind, L, spin, sampling, N)."""
    samp = spec.get("sampling", "mw")
    nside = spec.get("nside", spec["L"] // 2 if samp == "healpix" else 0)
    return PlanKey(spec["kind"], int(spec["L"]), int(spec.get("spin", 0)), int(spec.get("N", 1)), samp,
                   int(nside), spec.get("precision", "fp64"))


def coeff_shape(key):
    s = (key.L, 2 * key.L - 1)
    return ((2 * key.N - 1,) + s) if key.kind == "so3" else s


def map_elems(key):
    if key.kind == "so3":
        return (2 * key.N - 1) * key.L * (2 * key.L - 1)
    if key.sampling == "mw":
        return key.L * (2 * key.L - 1)
    return 12 * key.nside * key.nside


class Scheduler:
    """Device-free continuous-batching scheduler.

    The executor provides:
      batch_limit(key) -> int        largest batch of one launch for the key
      new_bytes(key) -> int          device bytes a launch would newly allocate
                                     (plan constants if not cached, a workspace
                                     if the next free stream has none)
      resident_bytes() -> int        bytes held by cached plans and workspaces
      free_streams() -> int          streams with no batch in flight
      launch(key, requests) -> handle     enqueue a batch (non-blocking)
      poll() -> finished handles (each keeps its .requests)
      evict(nbytes, busy_keys) -> int     drop cached plans (LRU) not in use
    Buffers of a batch (input, inverse output, forward output) count against
    the budget while the batch is in flight.
    """

    def __init__(self, executor, hbm_budget):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.queue = collections.deque()
        self.inflight = []
        self.in_use = 0
        self.done = []
        self.rejected = []

    @staticmethod
    def buffer_bytes(key, n):
        return 16 * n * (2 * int(np.prod(coeff_shape(key))) + map_elems(key))

    def submit(self, req):
        self.queue.append(req)

    def _form_batch(self):
        head = self.queue[0]
        key = head.key
        limit = max(1, int(self.ex.batch_limit(key)))
        batch = [head]
        for r in itertools.islice(self.queue, 1, None):
            if len(batch) >= limit:
                break
            if r.key == key:
                batch.append(r)
        return key, batch

    def _need(self, key, n):
        new = self.ex.new_bytes(key)          # may bring the key's plan into the cache
        return self.in_use + self.ex.resident_bytes() + new + self.buffer_bytes(key, n)

    def _fits(self, key, n):
        return self._need(key, n) <= self.budget

    def try_launch(self, now):
        """Launch as many batches as streams and memory allow; returns the number launched."""
        launched = 0
        while self.queue and self.ex.free_streams() > 0:
            key, batch = self._form_batch()
            n = len(batch)
            while n > 0 and not self._fits(key, n):
                n -= 1
            if n == 0:
                short = self._need(key, 1) - self.budget
                busy = {h.key for h in self.inflight}
                if self.ex.evict(short, busy) > 0 and self._fits(key, 1):
                    continue
                if not self.inflight:
                    # does not fit even alone on an idle device: reject the head request
                    r = self.queue.popleft()
                    r.error = "request does not fit the HBM budget"
                    self.rejected.append(r)
                    continue
                break          # wait for in-flight work to free memory
            batch = batch[:n]
            ids = {id(r) for r in batch}
            self.queue = collections.deque(r for r in self.queue if id(r) not in ids)
            h = self.ex.launch(key, batch)
            h.footprint = self.buffer_bytes(key, n)
            h.key = key
            self.in_use += h.footprint
            for r in batch:
                r.t_launch = now
                r.batch_size = n
            self.inflight.append(h)
            launched += 1
        return launched

    def poll(self, now):
        fin = self.ex.poll()
        for h in fin:
            self.inflight.remove(h)
            self.in_use -= h.footprint
            for r in h.requests:
                if r.t_done is None:
                    r.t_done = now
                self.done.append(r)
        return len(fin)

    @property
    def idle(self):
        return not self.queue and not self.inflight


def serve(scheduler, requests, clock=time.perf_counter, realtime=True, sleep=time.sleep):
    """Run the loop over ``requests`` (sorted by t_arrival).  With realtime=False
    every request is submitted at t = 0 (saturation throughput).  Returns the
    wall time of the run in seconds."""
    pending = sorted(requests, key=lambda r: r.t_arrival)
    if not realtime:
        for r in pending:
            r.t_arrival = 0.0
    i = 0
    t0 = clock()
    while i < len(pending) or not scheduler.idle:
        now = clock() - t0
        while i < len(pending) and pending[i].t_arrival <= now:
            scheduler.submit(pending[i])
            i += 1
        progressed = scheduler.poll(clock() - t0)
        progressed += scheduler.try_launch(clock() - t0)
        if not progressed:
            if scheduler.inflight:
                sleep(0)       # yield; completion is polled on the next pass
            elif i < len(pending):
                sleep(max(0.0, min(pending[i].t_arrival - (clock() - t0), 0.01)))
    return clock() - t0


def latency_stats(requests):
    lat = np.array([r.latency for r in requests if r.latency is not None])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}


# --------------------------------------------------------------------------- GPU executor
class _Handle:
    __slots__ = ("requests", "event", "stream_idx", "out_host", "footprint", "key", "keep")


class GpuExecutor:
    """Runs batches through the C ABI on ``n_streams`` HIP streams (default
    priority), with an LRU cache of plans and one workspace per (plan, stream).

    batch_bytes: target device bytes of one batch's buffers; the batch limit of
    a key is the number of its requests that fit (at least 1, at most max_batch)."""

    def __init__(self, device="cuda:0", n_streams=4, max_batch=8, batch_bytes=2 << 30, keep_results=True):
        import torch
        from . import binding
        self.torch, self.binding = torch, binding
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        self.busy = [False] * n_streams
        self.max_batch = int(max_batch)
        self.batch_bytes = int(batch_bytes)
        self.plans = collections.OrderedDict()      # key -> Plan (LRU order)
        self.ws = {}                                # (key, stream) -> workspace tensor
        self.pending = []
        self.keep_results = keep_results

    def batch_limit(self, key):
        per = Scheduler.buffer_bytes(key, 1)
        return max(1, min(self.max_batch, self.batch_bytes // max(per, 1)))

    def _plan(self, key):
        p = self.plans.get(key)
        if p is None:
            with self.torch.cuda.device(self.device):
                p = self.binding.Plan(key.L, spin=key.spin, N=key.N, sampling=key.sampling, nside=key.nside,
                                      max_batch=self.batch_limit(key), precision=key.precision,
                                      device=self.device)
                self.torch.cuda.current_stream(self.device).synchronize()
            self.plans[key] = p
        self.plans.move_to_end(key)
        return p

    def _next_stream(self):
        return self.busy.index(False)

    def new_bytes(self, key):
        p = self.plans.get(key)
        if p is None:
            # create the plan now (host tables + constant upload) to learn its sizes; the
            # bytes are reported here once and are resident from then on
            p = self._plan(key)
            return 0 if (key, 0) in self.ws else int(p.info["workspace_bytes"])
        if False not in self.busy:
            return 0
        return 0 if (key, self._next_stream()) in self.ws else int(p.info["workspace_bytes"])

    def resident_bytes(self):
        tot = sum(int(p.info["plan_device_bytes"]) for p in self.plans.values())
        return tot + sum(int(w.numel()) for w in self.ws.values())

    def free_streams(self):
        return sum(1 for b in self.busy if not b)

    def evict(self, nbytes, busy_keys):
        freed = 0
        for key in list(self.plans):
            if freed >= nbytes:
                break
            if key in busy_keys:
                continue
            p = self.plans.pop(key)
            freed += int(p.info["plan_device_bytes"])
            for s in range(len(self.streams)):
                w = self.ws.pop((key, s), None)
                if w is not None:
                    freed += int(w.numel())
            p.close()
        return freed

    def launch(self, key, requests):
        torch = self.torch
        s = self._next_stream()
        self.busy[s] = True
        plan = self._plan(key)
        stream = self.streams[s]
        h = _Handle()
        h.requests, h.stream_idx = requests, s
        x_host = torch.from_numpy(np.stack([r.data for r in requests])).pin_memory()
        with torch.cuda.stream(stream):
            ws = self.ws.get((key, s))
            if ws is None:
                ws = plan.new_workspace()
                self.ws[(key, s)] = ws
            x = x_host.to(self.device, non_blocking=True)
            if key.kind == "so3":
                y = plan.so3_forward(plan.so3_inverse(x, workspace=ws), workspace=ws)
            else:
                y = plan.forward(plan.inverse(x, workspace=ws), workspace=ws)
            out = torch.empty(y.shape, dtype=y.dtype, pin_memory=True) if self.keep_results else None
            if out is not None:
                out.copy_(y, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        h.event, h.out_host = ev, out
        h.keep = (x_host, x, y)        # buffers stay referenced until the stream passes the event
        self.pending.append(h)
        return h

    def poll(self):
        fin = [h for h in self.pending if h.event.query()]
        for h in fin:
            self.pending.remove(h)
            self.busy[h.stream_idx] = False
            if h.out_host is not None:
                res = h.out_host.numpy()
                for i, r in enumerate(h.requests):
                    r.result = res[i]
            h.keep = None
        return fin

    def close(self):
        self.torch.cuda.synchronize(self.device)
        for p in self.plans.values():
            p.close()
        self.plans.clear()
        self.ws.clear()


def build_requests(trace, seed=3):
    """Requests with iid complex Gaussian coefficients for a serving trace."""
    from .synth import flm_gaussian, flmn_gaussian
    reqs = []
    for i, spec in enumerate(trace):
        key = key_of(spec)
        if key.kind == "so3":
            data = flmn_gaussian(key.L, key.N, seed=seed * 1000003 + i)
        else:
            data = flm_gaussian(key.L, key.spin, seed=seed * 1000003 + i)
        reqs.append(Request(rid=i, key=key, data=data, t_arrival=float(spec["t"])))
    return reqs


def run_mix(n_requests=200, seed=3, lmin=64, lmax=1024, so3_lmax=256, n_streams=4, max_batch=8,
            budget_frac=0.8, loads=(0.5, 0.7, 0.9), device="cuda:0"):
    """Saturation throughput of a request mix, then realtime runs at fractions of it.

    Returns a dict with the saturation rate (requests/s) and p50/p99 latency per load."""
    import torch
    from .synth import serving_trace
    total = torch.cuda.get_device_properties(torch.device(device)).total_memory
    trace = serving_trace(n_requests=n_requests, seed=seed, rate=1.0, lmin=lmin, lmax=lmax, so3_lmax=so3_lmax)
    ex = GpuExecutor(device=device, n_streams=n_streams, max_batch=max_batch, keep_results=False)
    out = {"requests": n_requests, "seed": seed, "L_range": [lmin, lmax], "so3_L_max": so3_lmax,
           "streams": n_streams, "max_batch": max_batch}
    try:
        # warm pass builds every plan once, then the saturation pass
        sched = Scheduler(ex, hbm_budget=budget_frac * total)
        serve(sched, build_requests(trace[: min(len(trace), 4 * n_streams)], seed), realtime=False)
        reqs = build_requests(trace, seed)
        sched = Scheduler(ex, hbm_budget=budget_frac * total)
        wall = serve(sched, reqs, realtime=False)
        lam = len(sched.done) / wall
        out["saturation_req_per_s"] = lam
        out["rejected"] = len(sched.rejected)
        for frac in loads:
            rate = frac * lam
            tr = serving_trace(n_requests=n_requests, seed=seed, rate=rate, lmin=lmin, lmax=lmax,
                               so3_lmax=so3_lmax)
            reqs = build_requests(tr, seed)
            sched = Scheduler(ex, hbm_budget=budget_frac * total)
            wall = serve(sched, reqs, realtime=True)
            st = latency_stats(sched.done)
            st["offered_req_per_s"] = rate
            st["achieved_req_per_s"] = len(sched.done) / wall
            out[f"load_{frac}"] = st
    finally:
        ex.close()
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serve a seeded mix of transform requests on one GPU")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--lmin", type=int, default=64)
    ap.add_argument("--lmax", type=int, default=1024)
    ap.add_argument("--so3-lmax", type=int, default=256)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=8)
    a = ap.parse_args(argv)
    res = run_mix(a.requests, a.seed, a.lmin, a.lmax, a.so3_lmax, a.streams, a.max_batch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
