"""Continuous-batching server for ciphertext multiplication (the Mul tensor of
section II-A) over requests of mixed N and level.

Requests arrive over time (Poisson traces in the benchmark).  The scheduler
admits a request when its HBM footprint fits the budget, launches everything
admitted as one step, and keeps up to `streams` steps in flight on separate
streams, so requests that arrive while earlier ones run join the next step
as soon as a stream and memory free up.  On the GPU a step is one grouped
call (hentt_ct_tensor_grouped): one job per request, reading the request's
device-resident operands in place, all requests of one N in the same three
launches whatever their levels.

The footprint is what a request makes the device hold while it is in
flight: 88 L N bytes for L limbs of N words -- its two input ciphertexts (4
polynomials, resident from its arrival), its 3-polynomial tensor output and
the 4 polynomials of the library's forward-column-pass workspace.  The GPU
backend keeps what it holds within the budget: output buffers are pooled
for reuse (the memory cache of section III-C-1) and idle ones are freed
before a new one would take their total past the output share of the
budget, and the library's workspace pool is trimmed when it would exceed
its share.  Latency = completion of the request's step minus its arrival;
completion is observed with stream events, the only host synchronisation.

The scheduling logic is backend-independent: HipBackend runs on the GPU
through the library's C ABI; the unit tests drive the same scheduler with a
CPU backend to force budget exhaustion, failed launches and cancellation.
"""
import collections
import time

import numpy as np

WORD = 8


INPUT_POLYS = 4      # c, d (2 polynomials each), the request's own device buffers
OUTPUT_POLYS = 3     # the tensor output, from the backend's pool
WORKSPACE_POLYS = 4  # the library's forward column pass over c0, c1, d0, d1


def footprint(log_n, level):
    """HBM bytes a request makes the device hold while it is admitted."""
    return (INPUT_POLYS + OUTPUT_POLYS + WORKSPACE_POLYS) * level * (1 << log_n) * WORD


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
    """Admission by footprint + continuous batching over `streams` in-flight steps.

    A step takes the admitted requests in arrival order up to step_bytes of
    footprint (default: budget / streams), so that under a full queue the
    next step is already launched while the current one runs."""

    def __init__(self, backend, budget_bytes, streams=2, max_group=64, clock=time.perf_counter, step_bytes=None):
        self.be = backend
        self.budget = budget_bytes
        self.reserved = 0
        self.streams = streams
        self.step_bytes = step_bytes if step_bytes is not None else budget_bytes // max(1, streams)
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
        """Launch one step from the admitted requests; False if none was launched."""
        if not self.admitted or len(self.inflight) >= self.streams:
            return False
        take, size = 0, 0
        for r in self.admitted:
            fp = footprint(r.log_n, r.level)
            if take and size + fp > self.step_bytes:
                break
            take += 1
            size += fp
        step, self.admitted = self.admitted[:take], self.admitted[take:]
        groups = collections.OrderedDict()
        for r in step:
            groups.setdefault((r.log_n, r.level), []).append(r)
        batch = []
        for key, rs in groups.items():
            for i in range(0, len(rs), self.max_group):
                batch.append((key, rs[i:i + self.max_group]))
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
            return True
        reqs = [r for _, rs in batch for r in rs]
        for r in reqs:
            r.state = "launched"
            r.t_launch = now
        self.inflight.append((handle, reqs))
        self.steps += 1
        return True

    def tick(self):
        self._poll()
        self._admit()
        while self._launch():
            pass

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
    """Steps on the GPU: one hentt_ct_tensor_grouped call per step with one
    job per request (operands read in place, output into a pooled buffer);
    one stream per in-flight step.

    budget_bytes bounds what the backend holds: output buffers up to the
    output share (3/11) of it, the library's workspace pool up to the
    workspace share (4/11); the request operands (4/11) are the client's.
    held_bytes() reports outputs + workspace; peak_held the largest value
    seen."""

    def __init__(self, chain, log_ns=(14, 15, 16), streams=2, verify=False, budget_bytes=None):
        import torch
        import paper_2109_14704_amd as H
        self.torch, self.H = torch, H
        self.tables = {ln: H.Tables(ln, chain) for ln in log_ns}
        self.views = {}
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.pool = collections.OrderedDict()   # (log_n, level) -> free output buffers, oldest first
        self.keep_results = verify
        self.launches = 0
        share = INPUT_POLYS + OUTPUT_POLYS + WORKSPACE_POLYS
        self.out_cap = None if budget_bytes is None else budget_bytes * OUTPUT_POLYS // share
        self.ws_cap = None if budget_bytes is None else budget_bytes * WORKSPACE_POLYS // share
        self.out_bytes = 0                       # every output buffer allocated and not freed, busy or idle
        self.peak_held = 0

    def view(self, log_n, level):
        key = (log_n, level)
        if key not in self.views:
            self.views[key] = self.tables[log_n].view(level)
        return self.views[key]

    def held_bytes(self):
        return self.out_bytes + self.H.pool_bytes()

    def _free_idle(self, need):
        """Free idle output buffers, oldest first, until `need` more bytes fit the output share."""
        while self.out_cap is not None and self.out_bytes + need > self.out_cap:
            key = next((k for k, v in self.pool.items() if v), None)
            if key is None:
                break
            buf = self.pool[key].pop(0)
            self.out_bytes -= buf.numel() * WORD
            if not self.pool[key]:
                del self.pool[key]

    def _out(self, log_n, level):
        free = self.pool.get((log_n, level))
        if free:
            buf = free.pop(0)
            if not free:
                del self.pool[(log_n, level)]
            return buf
        need = OUTPUT_POLYS * level * (1 << log_n) * WORD
        self._free_idle(need)
        buf = self.torch.empty((1, OUTPUT_POLYS, level, 1 << log_n), dtype=self.torch.int64, device="cuda:0")
        self.out_bytes += need
        return buf

    def _put(self, key, buf):
        self.pool.setdefault(key, []).append(buf)
        self.pool.move_to_end(key)

    def launch(self, batch, slot=0):
        torch, H = self.torch, self.H
        st = self.streams[self.launches % len(self.streams)]
        self.launches += 1
        reqs = [r for _, rs in batch for r in rs]
        if self.ws_cap is not None:
            # at most every job's workspace in one launch sequence
            need = sum(WORKSPACE_POLYS * r.level * (1 << r.log_n) * WORD for r in reqs)
            if H.pool_bytes() + need > self.ws_cap:
                H.pool_trim()                   # frees idle workspace buffers (waits for their streams)
        st.wait_stream(torch.cuda.current_stream())   # the operands were written on the current stream
        used, jobs = [], []
        for r in reqs:
            out = self._out(r.log_n, r.level)
            used.append(((r.log_n, r.level), out))
            jobs.append((self.view(r.log_n, r.level), r.c, r.d, out))
            r.slot = out
        try:
            H.ct_tensor_grouped(jobs, stream=st)
        except Exception:
            for key, out in used:
                self._put(key, out)
            raise
        ev = torch.cuda.Event()
        ev.record(st)
        self.peak_held = max(self.peak_held, self.held_bytes())
        return (ev, used, st)

    def poll(self, handle):
        return True if handle[0].query() else None

    def collect(self, handle, reqs):
        if self.keep_results:
            for r in reqs:
                r.result = r.slot.clone()

    def release(self, handle):
        for key, out in handle[1]:
            self._put(key, out)


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
        st.wait_stream(torch.cuda.current_stream())
        out = backend._out(r.log_n, r.level)
        H.ct_tensor(backend.view(r.log_n, r.level), r.c, r.d, out=out, stream=st)
        st.synchronize()
        r.t_done = clock()
        r.state = "done"
        backend._put((r.log_n, r.level), out)
    return clock() - t0
