"""Continuous-batching server for ciphertext multiplication (the Mul tensor of
section II-A) over requests of mixed N and level.

Requests arrive over time (Poisson traces in the benchmark).  The scheduler
admits a request when its HBM footprint fits the budget, groups the
admitted requests of equal (N, level) into one batched call, and keeps up to
`streams` steps in flight on separate streams, so requests that arrive while
earlier ones run join the next step as soon as a stream and memory free up.

The footprint is what a request makes the device hold while it is in
flight: 88 L N bytes for L limbs of N words -- its two input ciphertexts (4
polynomials) and the 3-polynomial tensor output in the step's slab, plus the
4 polynomials of the library's forward-column-pass workspace.  The GPU
backend keeps what it holds within the budget: slabs are sized exactly to
their step and pooled for reuse (the memory cache of section III-C-1), idle
slabs are freed before a new one would take the slab total past its share
of the budget, and the library's workspace pool is trimmed when it holds
more than its share.  Latency = completion of the request's step minus its
arrival; completion is observed with stream events, the only host
synchronisation.

The scheduling logic is backend-independent: HipBackend runs on the GPU
through the library's C ABI; the unit tests drive the same scheduler with a
CPU backend to force budget exhaustion, failed launches and cancellation.
"""
import collections
import time

import numpy as np

WORD = 8


SLAB_POLYS = 7       # c, d (2 polynomials each) and the tensor output (3)
WORKSPACE_POLYS = 4  # the library's forward column pass over c0, c1, d0, d1


def footprint(log_n, level):
    """HBM bytes a request makes the device hold while it is admitted."""
    return (SLAB_POLYS + WORKSPACE_POLYS) * level * (1 << log_n) * WORD


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
    """Steps on the GPU: each (N, level) group is gathered into a slab
    (device-to-device copies stand in for the upload of the ciphertexts) and
    multiplied by one hentt_ct_tensor call; one stream per in-flight step.

    budget_bytes bounds what the backend holds: slabs up to the slab share
    (7/11) of it, the library's workspace pool up to the workspace share
    (4/11).  held_bytes() reports both; peak_held the largest value seen."""

    def __init__(self, chain, log_ns=(14, 15, 16), streams=2, verify=False, budget_bytes=None):
        import torch
        import paper_2109_14704_amd as H
        self.torch, self.H = torch, H
        self.tables = {ln: H.Tables(ln, chain) for ln in log_ns}
        self.views = {}
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.pool = collections.OrderedDict()   # (log_n, level, count) -> free slabs [c, d, out], oldest first
        self.keep_results = verify
        self.launches = 0
        share = SLAB_POLYS + WORKSPACE_POLYS
        self.slab_cap = None if budget_bytes is None else budget_bytes * SLAB_POLYS // share
        self.ws_cap = None if budget_bytes is None else budget_bytes * WORKSPACE_POLYS // share
        self.slab_bytes = 0                      # every slab allocated and not freed, busy or idle
        self.peak_held = 0

    def view(self, log_n, level):
        key = (log_n, level)
        if key not in self.views:
            self.views[key] = self.tables[log_n].view(level)
        return self.views[key]

    def held_bytes(self):
        return self.slab_bytes + self.H.pool_bytes()

    def _free_idle(self, need):
        """Free idle slabs, oldest first, until `need` more bytes fit the slab share."""
        while self.slab_cap is not None and self.slab_bytes + need > self.slab_cap:
            key = next((k for k, v in self.pool.items() if v), None)
            if key is None:
                break
            slab = self.pool[key].pop(0)
            self.slab_bytes -= sum(t.numel() * WORD for t in slab)
            if not self.pool[key]:
                del self.pool[key]

    def _slab(self, log_n, level, count):
        free = self.pool.get((log_n, level, count))
        if free:
            slab = free.pop(0)
            if not free:
                del self.pool[(log_n, level, count)]
            return slab
        torch = self.torch
        n = 1 << log_n
        need = SLAB_POLYS * count * level * n * WORD
        self._free_idle(need)
        mk = lambda k: torch.empty((count, k, level, n), dtype=torch.int64, device="cuda:0")
        slab = [mk(2), mk(2), mk(3)]
        self.slab_bytes += need
        return slab

    def launch(self, batch, slot=0):
        torch, H = self.torch, self.H
        st = self.streams[self.launches % len(self.streams)]
        self.launches += 1
        # largest group first: its workspace buffer serves the later groups of the step
        batch = sorted(batch, key=lambda g: -(len(g[1]) * g[0][1] << g[0][0]))
        if self.ws_cap is not None and batch:
            (log_n, level), rs = batch[0]
            need = WORKSPACE_POLYS * len(rs) * level * (1 << log_n) * WORD
            if H.pool_bytes() + need > self.ws_cap:
                H.pool_trim()                   # frees idle workspace buffers (waits for their streams)
        st.wait_stream(torch.cuda.current_stream())
        used = []
        with torch.cuda.stream(st):
            for (log_n, level), rs in batch:
                slab = self._slab(log_n, level, len(rs))
                c, d, out = slab
                for i, r in enumerate(rs):
                    c[i].copy_(r.c[0], non_blocking=True)
                    d[i].copy_(r.d[0], non_blocking=True)
                    r.slot = (slab, i)
                H.ct_tensor(self.view(log_n, level), c, d, out=out, stream=st)
                used.append(((log_n, level, len(rs)), slab))
            ev = torch.cuda.Event()
            ev.record(st)
        self.peak_held = max(self.peak_held, self.held_bytes())
        return (ev, used, st)

    def poll(self, handle):
        return True if handle[0].query() else None

    def collect(self, handle, reqs):
        if self.keep_results:
            for r in reqs:
                slab, i = r.slot
                r.result = slab[2][i:i + 1].clone()

    def release(self, handle):
        for key, slab in handle[1]:
            self.pool.setdefault(key, []).append(slab)
            self.pool.move_to_end(key)


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
            c, d, out = slab
            c[0].copy_(r.c[0], non_blocking=True)
            d[0].copy_(r.d[0], non_blocking=True)
            H.ct_tensor(backend.view(r.log_n, r.level), c, d, out=out, stream=st)
        st.synchronize()
        r.t_done = clock()
        r.state = "done"
        backend.pool.setdefault((r.log_n, r.level, 1), []).append(slab)
    return clock() - t0
