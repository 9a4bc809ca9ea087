"""Continuous-batching serving loop for decaying-turbulence runs.

Requests (grid size, method, number of steps, seed) arrive over time.  The
scheduler admits a waiting request when its device memory fits the HBM
budget and a slot is free, keeps every admitted run's populations resident
on the device, and advances all active runs together: the runs of each
method form one batch (one launch per step for all of them, on
that method's stream, so the two methods' work overlaps on the device).
The active set is re-formed whenever a run finishes or is admitted, between
chunks of steps, so requests that arrive while others are running join
without waiting for them to finish.  A run's energy spectrum and statistics
are computed on the device in the round after its last steps were issued
(while the device works on that round's steps), its memory is released, and
the latency from arrival to result is recorded.

The scheduler talks to a backend object (GPU: `GpuBackend`; tests use a fake
one) with these methods:
    bytes_of(req) -> int       device bytes the run needs while active
    prepare(req)               optional: called once for each arrived request,
                               in arrival order, before admission (the GPU
                               backend starts generating its initial field
                               in the background); returning False declines
                               for now (asked again in the next round)
    start(req) -> handle       allocate and initialise the run
    advance(handles, nsteps)   advance active runs (all of one method) by nsteps
    finish(handle) -> result   final diagnostics of a finished run
    release(handle)            release the run's device memory (the GPU
                               backend keeps the box for a later run)
    sync()                     wait for all queued work
"""
import heapq
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass(order=True)
class Request:
    arrival: float
    rid: int = field(compare=False)
    n: int = field(compare=False)
    method: str = field(compare=False)
    steps: int = field(compare=False)
    seed: int = field(compare=False)


def poisson_trace(count, rate, seed, grids=(32, 64, 128, 256), weights=(0.4, 0.3, 0.2, 0.1),
                  methods=("mrt", "dugks"), steps=(500, 2000)):
    """`count` requests with exponential inter-arrival times of mean 1/rate
    seconds; grid, method and step count drawn independently."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    w = np.asarray(weights, dtype=float)
    w = w / w.sum()
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(np.asarray(grids), p=w))
        m = methods[int(rng.integers(len(methods)))]
        k = int(rng.integers(steps[0], steps[1] + 1))
        out.append(Request(arrival=t, rid=i, n=n, method=m, steps=k, seed=1000 + i))
    return out


@dataclass
class Active:
    req: Request
    handle: object
    bytes: int
    done: int = 0
    admitted: float = 0.0


class Scheduler:
    """Admits requests by HBM budget and slot count, advances the active
    runs in chunks of at most `chunk` steps (a chunk never runs a request
    past its step count), finishes and releases completed runs."""

    def __init__(self, backend, budget_bytes, max_active=64, chunk=64):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.in_use = 0
        self.peak_in_use = 0
        self.active = []
        self.results = {}
        self._prepared = set()

    def _prepare(self, waiting, now):
        # arrived requests in arrival order; a backend may decline (return
        # False) to bound what it holds ahead, and is asked again next round
        prep = getattr(self.backend, "prepare", None)
        if prep is None:
            return
        for req in sorted(waiting):
            if req.arrival > now:
                break
            if req.rid in self._prepared:
                continue
            if prep(req) is False:
                break
            self._prepared.add(req.rid)

    def _admit(self, waiting, now):
        admitted = []
        while waiting and waiting[0].arrival <= now and len(self.active) < self.max_active:
            req = waiting[0]
            need = self.backend.bytes_of(req)
            if need > self.budget:
                raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.rid, need))
            if self.in_use + need > self.budget:
                break   # first come, first served: later arrivals wait behind it
            heapq.heappop(waiting)
            h = self.backend.start(req)
            self.in_use += need
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            a = Active(req, h, need, 0, now)
            self.active.append(a)
            admitted.append(a)
        return admitted

    def run(self, trace, clock=time.perf_counter, sleep=time.sleep, on_result=None):
        """Serves `trace`; returns the latency percentiles, the aggregate
        cell-update rate and the host time spent in each backend call
        (`host_s`: start, advance, finish, release, idle).

        Runs whose last steps were issued in one round are finished and
        released in the next, after that round's steps have been issued:
        the device works on the next chunk while their results are read."""
        waiting = list(trace)
        heapq.heapify(waiting)
        t0 = clock()
        cells_steps = 0
        spent = dict(start=0.0, advance=0.0, finish=0.0, release=0.0, idle=0.0)

        def timed(key, fn, *a):
            t = clock()
            r = fn(*a)
            spent[key] += clock() - t
            return r

        last_issued = []   # runs whose last steps were issued in the previous round
        while waiting or self.active or last_issued:
            now = clock() - t0
            self._prepare(waiting, now)
            timed("start", self._admit, waiting, now)
            issued = []
            if self.active:
                k = min(self.chunk, min(a.req.steps - a.done for a in self.active))
                groups = {}
                for a in self.active:
                    groups.setdefault(a.req.method, []).append(a)
                for method, acts in groups.items():
                    timed("advance", self.backend.advance, [a.handle for a in acts], k)
                for a in self.active:
                    a.done += k
                    cells_steps += a.req.n ** 3 * k
                issued = [a for a in self.active if a.done >= a.req.steps]
                self.active = [a for a in self.active if a.done < a.req.steps]
            elif not last_issued:
                if waiting:
                    timed("idle", sleep, max(0.0, waiting[0].arrival - (clock() - t0)))
                continue
            for a in last_issued:
                res = timed("finish", self.backend.finish, a.handle)
                t_done = clock() - t0
                self.results[a.req.rid] = dict(result=res, latency=t_done - a.req.arrival,
                                               wait=a.admitted - a.req.arrival, n=a.req.n,
                                               method=a.req.method, steps=a.req.steps)
                timed("release", self.backend.release, a.handle)
                self.in_use -= a.bytes
                if on_result:
                    on_result(a.req, self.results[a.req.rid])
            last_issued = issued
        self.backend.sync()
        wall = clock() - t0
        lat = np.array([r["latency"] for r in self.results.values()])
        return dict(requests=len(self.results), wall_s=wall,
                    p50_s=float(np.percentile(lat, 50)) if len(lat) else math.nan,
                    p99_s=float(np.percentile(lat, 99)) if len(lat) else math.nan,
                    mean_s=float(lat.mean()) if len(lat) else math.nan,
                    mlups=cells_steps / wall / 1e6 if wall > 0 else math.nan,
                    peak_bytes=self.peak_in_use, host_s={k: round(v, 3) for k, v in spent.items()})


class GpuBackend:
    """Runs requests as library boxes on the current GPU: FP32 by default,
    one batch per method on a PyTorch stream of that method, and a stream
    of its own for every box (the batch's steps wait for the box's stream
    and the box's stream for them, on the device).

    Nothing on the way from admission to release allocates or frees device
    memory once the sizes in the trace have been seen, so no call waits for
    the whole device: initial fields are generated on the device by host
    threads from the request's arrival on (at most `fields_ahead` waiting;
    fields given as host arrays are copied on a stream of their own, which
    does not wait for the steps queued on the methods' streams) and
    turned into the initial state on the box's stream by
    `init_velocity_field_device`; a finished run's box goes back to a pool
    (up to `idle_bytes` of idle boxes, the rest are closed) and the next
    run of that size and method takes it, spectrum
    work space and hipFFT plans included.  Idle pooled boxes are device
    memory outside the scheduler's budget, at most `idle_bytes` of it; a
    box released beyond that is closed (which waits for the device)."""

    def __init__(self, precision="fp32", nu=0.01, k0=4.0, u_rms=0.05, fields=None, field_workers=4,
                 idle_bytes=32e9, fields_ahead=16):
        import concurrent.futures

        import torch

        from . import Batch, Box, box_bytes, default_params, spectrum_bytes
        self._torch = torch
        self._Box, self._Batch = Box, Batch
        self._box_bytes, self._default_params = box_bytes, default_params
        self._spectrum_bytes = spectrum_bytes
        self._bytes = {}
        self.precision, self.nu, self.k0, self.u_rms = precision, nu, k0, u_rms
        self.streams = {}
        self.batches = {}   # method -> (key of its active set, Batch)
        self.idle_bytes = float(idle_bytes)
        self._idle = {}     # (n, method) -> idle boxes
        self._idle_total = 0
        self._runs = 0      # runs started (tells a reused box's runs apart in batch keys)
        self.created = 0    # boxes created (the rest of the runs reused a pooled box)
        # host seconds inside start(): waiting for initial fields, creating boxes, initial states
        self.start_s = dict(field_wait=0.0, create=0.0, init=0.0)
        if fields is None:
            import synth
            fields = lambda req: synth.dhit_field_gpu(req.n, seed=req.seed, k0=k0, u_rms=u_rms, as_tensor=True)
        self.fields = fields
        self.fields_ahead = int(fields_ahead)
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=field_workers)
        self._pending = {}   # rid -> future of the initial field (host array)
        self._upload = torch.cuda.Stream()

    def warm_up(self, grids, methods=("mrt", "dugks")):
        """What the first run of a grid size would otherwise pay at admission:
        hipFFT plans of the library's spectrum (through spectrum_bytes) and of
        the field recipe (one field made), whose kernels are compiled on first
        use in the process."""
        for n in grids:
            for m in methods:
                self.bytes_of(Request(0.0, -1, n, m, 0, 0))
            self.fields(Request(0.0, -1, n, methods[0], 0, 0))
        self._torch.cuda.synchronize()

    def prepare(self, req):
        # at most `fields_ahead` fields wait for admission (they are device
        # memory outside the scheduler's budget)
        if len(self._pending) >= self.fields_ahead:
            return False
        if req.rid not in self._pending:
            self._pending[req.rid] = self._pool.submit(self.fields, req)
        return True

    def _stream(self, method):
        if method not in self.streams:
            self.streams[method] = self._torch.cuda.Stream()
        return self.streams[method]

    def bytes_of(self, req):
        p = self._default_params(req.n, req.method, self.precision, self.nu)
        # the spectrum work space (arrays and hipFFT work areas) is allocated
        # when the run finishes; count it while the run is active
        key = (req.n, req.method)
        if key not in self._bytes:
            self._bytes[key] = self._box_bytes(p) + self._spectrum_bytes(p)
        return self._bytes[key]

    def start(self, req):
        torch = self._torch
        t0 = time.perf_counter()
        fut = self._pending.pop(req.rid, None)
        u = fut.result() if fut is not None else self.fields(req)
        t1 = time.perf_counter()
        idle = self._idle.get((req.n, req.method))
        if idle:
            b = idle.pop()
            self._idle_total -= self.bytes_of(req)
        else:
            # each box has a stream of its own: its upload, initial state and
            # spectrum wait only for the batch steps it takes part in
            b = self._Box(req.n, req.method, self.precision, self.nu, stream=self._torch.cuda.Stream())
            self.created += 1
        t2 = time.perf_counter()
        if torch.is_tensor(u) and u.is_cuda:
            b.init_velocity_field_device(u)   # made on the device, nothing to copy
        else:
            with torch.cuda.stream(self._upload):
                # a copy from pageable memory returns when it is done; the
                # box's stream then waits for the upload stream
                ud = torch.from_numpy(np.ascontiguousarray(u)).to("cuda")
                b.init_velocity_field_device(ud)
        self._runs += 1
        b.serve_run = self._runs
        t3 = time.perf_counter()
        self.start_s["field_wait"] += t1 - t0
        self.start_s["create"] += t2 - t1
        self.start_s["init"] += t3 - t2
        return b

    def advance(self, boxes, nsteps):
        # one batch per method for the whole run: when a run joins or leaves
        # the method's active set, the batch is re-formed in place (its device
        # tables are kept, nothing is freed)
        key = tuple((b.uid, b.serve_run) for b in boxes)
        method = boxes[0].method
        cur = self.batches.get(method)
        if cur is None:
            self.batches[method] = (key, self._Batch(boxes, autotune=False, stream=self._stream(method)))
        elif cur[0] != key:
            cur[1].update(boxes)
            self.batches[method] = (key, cur[1])
        self.batches[method][1].step(nsteps)

    def finish(self, box):
        E, st = box.energy_spectrum(box.n // 2)
        return dict(E=E, **st)

    def release(self, box):
        # the batch that held this run is re-formed before its next step (its
        # key no longer matches the active set), so it never steps the box
        # again for this run
        need = self._bytes[(box.n, box.method)]
        if self._idle_total + need <= self.idle_bytes:
            self._idle.setdefault((box.n, box.method), []).append(box)
            self._idle_total += need
        else:
            box.close()

    def sync(self):
        for _, bt in self.batches.values():
            bt.close()
        self.batches = {}
        for idle in self._idle.values():
            for b in idle:
                b.close()
        self._idle = {}
        self._idle_total = 0
        self._torch.cuda.synchronize()

    def close(self):
        self._pool.shutdown(wait=True)
        self._pending = {}
