"""Continuous-batching server for ciphertext multiplication (the Mul tensor of
section II-A) over requests of mixed N and level.

Requests arrive over time (Poisson traces in the benchmark).  The scheduler
admits a request when its HBM footprint fits the budget (56 L N bytes: two
input ciphertexts of 2 polynomials and the 3-polynomial tensor output, L
limbs of N words), groups the admitted requests of equal (N, level) into one
batched call, and keeps up to `streams` steps in flight on separate streams,
so requests that arrive while earlier ones run join the next step as soon as
a stream and memory free up.  Operand slabs come from a capacity-reusing
pool (the memory cache of section III-C-1).  Latency = completion of the
request's step minus its arrival; completion is observed with stream events,
the only host synchronisation.

The scheduling logic is backend-independent: HipBackend runs on the GPU
through the library's C ABI; the unit tests drive the same scheduler with a
CPU backend to force budget exhaustion, failed launches and cancellation.
"""
import collections
import time

import numpy as np

WORD = 8


def footprint(log_n, level):
    """HBM bytes a request holds while admitted: c, d (2 polys each) + out (3 polys)."""
    return 7 * level * (1 << log_n) * WORD


class Request:
    __slots__ = ("rid", "arrival", "log_n", "level", "c", "d", "state", "t_admit", "t_launch", "t_done",
                 "result", "error", "slot")

    def __init__(self, rid, arrival, log_n, level, c, d):
        self.rid, self.arrival, self.log_n, self.level = rid, arrival, log_n, level
        self.c, self.d = c, d          # operands at the source (device-resident for the GPU backend)
        self.state = "waiting"          # waiting -> admitted -> launched -> done | failed | rejected | cancelled
        self.t_admit = self.t_launch = self.t_done = None
        self.result = None
        self.error = None
        self.slot = None


class Scheduler:
    """Admission by footprint + continuous batching over `streams` in-flight steps."""

    def __init__(self, backend, budget_bytes, streams=2, max_group=64, clock=time.perf_counter):
        self.be = backend
        self.budget = budget_bytes
        self.reserved = 0
        self.streams = streams
        self.max_group = max_group
        self.clock = clock
        self.waiting = collections.deque()      # arrived, not yet admitted (FIFO)
        self.admitted = []                      # admitted, not yet launched
        self.inflight = []                      # (step handle, [requests])
        self.done = []
        self.steps = 0
        self.max_reserved = 0

    # -- client side -------------------------------------------------------------
    def submit(self, req):
        if footprint(req.log_n, req.level) > self.budget:
            req.state = "rejected"
            req.error = "footprint %d B exceeds the HBM budget %d B" % (footprint(req.log_n, req.level),
                                                                       self.budget)
            self.done.append(req)
            return False
        self.waiting.append(req)
        return True

    def cancel(self, req):
        """Cancel a request that has not been launched yet."""
        if req.state == "waiting":
            self.waiting.remove(req)
        elif req.state == "admitted":
            self.admitted.remove(req)
            self._release(req)
        else:
            return False
        req.state = "cancelled"
        self.done.append(req)
        return True

    # -- scheduling --------------------------------------------------------------
    def _release(self, req):
        self.reserved -= footprint(req.log_n, req.level)

    def _admit(self):
        while self.waiting:
            req = self.waiting[0]
            need = footprint(req.log_n, req.level)
            if self.reserved + need > self.budget:
                break                            # FIFO: wait until memory frees up
            self.waiting.popleft()
            self.reserved += need
            self.max_reserved = max(self.max_reserved, self.reserved)
            req.state = "admitted"
            req.t_admit = self.clock()
            self.admitted.append(req)

    def _poll(self):
        still = []
        for handle, reqs in self.inflight:
            st = self.be.poll(handle)
            if st is None:
                still.append((handle, reqs))
                continue
            now = self.clock()
            self.be.collect(handle, reqs)
            for r in reqs:
                r.t_done = now
                if st is True:
                    r.state = "done"
                else:
                    r.state = "failed"
                    r.error = str(st)
                self._release(r)
                self.done.append(r)
            self.be.release(handle)
        self.inflight = still

    def _launch(self):
        if not self.admitted or len(self.inflight) >= self.streams:
            return
        groups = collections.OrderedDict()
        for r in self.admitted:
            groups.setdefault((r.log_n, r.level), []).append(r)
        batch = []
        for key, rs in groups.items():
            for i in range(0, len(rs), self.max_group):
                batch.append((key, rs[i:i + self.max_group]))
        self.admitted = []
        now = self.clock()
        try:
            handle = self.be.launch(batch, slot=len(self.inflight))
        except Exception as e:                  # the step fails: its requests fail, memory is freed
            for _, rs in batch:
                for r in rs:
                    r.state = "failed"
                    r.error = "launch failed: %s" % e
                    r.t_done = self.clock()
                    self._release(r)
                    self.done.append(r)
            return
        reqs = [r for _, rs in batch for r in rs]
        for r in reqs:
            r.state = "launched"
            r.t_launch = now
        self.inflight.append((handle, reqs))
        self.steps += 1

    def tick(self):
        self._poll()
        self._admit()
        self._launch()

    def idle(self):
        return not (self.waiting or self.admitted or self.inflight)

    def run_trace(self, requests, time_scale=1.0):
        """Feed requests at their arrival times (seconds from start) and serve them."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        i = 0
        while i < len(reqs) or not self.idle():
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival * time_scale <= now:
                reqs[i].arrival = t0 + reqs[i].arrival * time_scale   # absolute
                self.submit(reqs[i])
                i += 1
            self.tick()
            if self.idle() and i < len(reqs):
                nxt = t0 + reqs[i].arrival * time_scale
                dt = nxt - self.clock()
                if dt > 0:
                    time.sleep(min(dt, 0.001))
        return self.clock() - t0


def latency_stats(reqs):
    lat = np.array([r.t_done - r.arrival for r in reqs if r.state == "done"])
    if lat.size == 0:
        return {"completed": 0}
    return {"completed": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}


# ============================================================ GPU backend
class HipBackend:
    """Steps on the GPU: each (N, level) group is gathered into a pooled slab
    (device-to-device copies stand in for the upload of the ciphertexts) and
    multiplied by one hentt_ct_tensor call; one stream per in-flight step."""

    def __init__(self, chain, log_ns=(14, 15, 16), streams=2, verify=False):
        import torch
        import paper_2109_14704_amd as H
        self.torch, self.H = torch, H
        self.tables = {ln: H.Tables(ln, chain) for ln in log_ns}
        self.views = {}
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.pool = collections.defaultdict(list)   # (log_n, level) -> free slabs [cap, c, d, out]
        self.keep_results = verify
        self.launches = 0

    def view(self, log_n, level):
        key = (log_n, level)
        if key not in self.views:
            self.views[key] = self.tables[log_n].view(level)
        return self.views[key]

    def _slab(self, log_n, level, count):
        torch = self.torch
        free = self.pool[(log_n, level)]
        for i, s in enumerate(free):
            if s[0] >= count:                    # any free slab with enough capacity
                return free.pop(i)
        cap = max(count, 4)
        n = 1 << log_n
        mk = lambda k: torch.empty((cap, k, level, n), dtype=torch.int64, device="cuda:0")
        return [cap, mk(2), mk(2), mk(3)]

    def launch(self, batch, slot=0):
        torch, H = self.torch, self.H
        st = self.streams[self.launches % len(self.streams)]
        self.launches += 1
        st.wait_stream(torch.cuda.current_stream())
        used = []
        with torch.cuda.stream(st):
            for (log_n, level), rs in batch:
                slab = self._slab(log_n, level, len(rs))
                cap, c, d, out = slab
                for i, r in enumerate(rs):
                    c[i].copy_(r.c[0], non_blocking=True)
                    d[i].copy_(r.d[0], non_blocking=True)
                    r.slot = (slab, i)
                b = len(rs)
                H.ct_tensor(self.view(log_n, level), c[:b], d[:b], out=out[:b], stream=st)
                used.append(((log_n, level), slab))
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, used, st)

    def poll(self, handle):
        return True if handle[0].query() else None

    def collect(self, handle, reqs):
        if self.keep_results:
            for r in reqs:
                slab, i = r.slot
                r.result = slab[3][i:i + 1].clone()

    def release(self, handle):
        for key, slab in handle[1]:
            self.pool[key].append(slab)


def serve_per_request(requests, backend, clock=time.perf_counter):
    """Baseline: each request alone (batch 1), in arrival order, one launch
    sequence per request on one stream, no overlap with later arrivals."""
    torch, H = backend.torch, backend.H
    reqs = sorted(requests, key=lambda r: r.arrival)
    st = backend.streams[0]
    t0 = clock()
    for r in reqs:
        now = clock() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.arrival = t0 + r.arrival
        with torch.cuda.stream(st):
            slab = backend._slab(r.log_n, r.level, 1)
            cap, c, d, out = slab
            c[0].copy_(r.c[0], non_blocking=True)
            d[0].copy_(r.d[0], non_blocking=True)
            H.ct_tensor(backend.view(r.log_n, r.level), c[:1], d[:1], out=out[:1], stream=st)
        st.synchronize()
        r.t_done = clock()
        r.state = "done"
        backend.pool[(r.log_n, r.level)].append(slab)
    return clock() - t0
