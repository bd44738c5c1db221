"""Served stream of back-transformation requests on one GPU (continuous
batching).

A request is one tridiagonal->band back-transformation Q <- H ... H Q of a
problem whose Q, reflectors and tau are resident on the device.  An SCF cycle
solves a series of eigenproblems of one size whose matrix changes only
slightly from step to step, in single or double precision (Kus et al.,
Sec. 5.1 and 5.2): a sequence keeps its buffers across its consecutive solves, and the
upstream stages that refill them are not part of the timed service.

Scheduling (all of it host logic around the C ABI; every step of the
computation runs in the HIP library):

* admission by device-memory footprint: a request is launched only while
  the library's workspace for the in-flight work
  (elpa_hh_workspace_bytes_batched) stays within the budget;
* continuous batching: `slots` streams; whenever a slot is free, ready
  requests that fit the budget (oldest first, at most max_batch and at most
  an equal share of the ready requests per free slot) are launched on it as
  one elpa_hh_trafo_batched call, so requests that arrive while others run
  are admitted as soon as a slot and memory free up and their work overlaps
  on the device;
* batches are bounded by work: a request joins a batch only while the
  batch's counted flops stay within batch_flops (the first request of a
  batch always goes).  Batching pays for small problems, whose launches
  leave the device idle; a large problem fills the device alone, and putting
  it in a batch only makes the others wait for it.  Unbounded batches also
  feed on themselves: a long batch lets many requests arrive, which form the
  next long batch, and latency stays high at rates the device keeps up
  with;
* a batch of one request runs as a single call with the library's kernel
  choice; larger batches run as one elpa_hh_trafo_batched call.  Calls run
  on their slot stream alone (plan streams = `call_streams`, 1 by default):
  the slots already keep several calls in flight, and the device has few
  hardware queues (4 per process by default), so stripe groups forked onto
  further streams share queues with other slots' work and serialise behind
  it;
* each slot issues its launches from a thread of its own: a launch call can
  block its thread until the device has worked through earlier launches
  (the runtime bounds the work in flight), and the scheduler keeps feeding
  the other slots and collecting completions meanwhile;
* completion is tracked with events; a solve that depends on an earlier one
  (the next step of the same SCF sequence) becomes ready when that completes;
* graphs (optional): an SCF sequence repeats the same call on the same
  buffers, so prepare_graphs() builds, per sequence buffer set, a prepared
  batch (elpa_hh_batch_create: workspace and tables resident like the
  sequence's Q and reflectors) and captures its run into a HIP graph; a
  request that runs alone then replays that graph on its slot stream instead
  of issuing the call's launches one by one (a prepared batch of one problem
  runs the kernel and plan of the single-problem call, so the replay and the
  plain call give the same result).

Times: arrivals and readiness on the host clock of the trace; start and
completion are the device times of events recorded before and behind the
request's work, placed on the same clock through an event recorded at the
trace start (so the poll loop's granularity does not bias them; the two time
bases agree to the event timestamps' resolution, a few microseconds).  Latency of a request = completion -
max(arrival, completion of the solve it depends on).  `run_plain` serves the
same requests one call at a time on one stream, as the baseline, timed the
same way.
"""
import time
from dataclasses import dataclass

from . import binding as B

__all__ = ["Request", "Server", "run_plain", "latency_stats", "take_batch"]


@dataclass
class Request:
    rid: int
    q: object            # column-major (n, nev) device tensor, overwritten
    hh: object           # reflectors (same dtype as q)
    tau: object
    nbw: int
    arrival: float       # seconds after the trace start
    after: int = -1      # rid that must complete first (-1: none)
    seq: int = -1
    step: int = -1
    t_ready: float = None
    t_start: float = None
    t_done: float = None
    via: str = None      # "graph", "single" or "batched": how it was launched

    def flops(self):
        n, nev = self.q.shape
        return (8 if self.q.is_complex() else 2) * n * (n - 1) * nev


def _dtype_code(q):
    return B._dtype_code(q)


def footprint(r):
    """Library workspace bytes of one request, alone (a single call with the
    library's plan) or in a batched call with the library's plan, whichever is
    larger: the sum over a batch bounds what its launch allocates."""
    if getattr(r, "_fp", None) is None:
        n, nev = r.q.shape
        dt = _dtype_code(r.q)
        r._fp = max(0, B.workspace_bytes(n, nev, r.nbw, dt),
                    B.workspace_bytes_batched([(n, nev, r.nbw, dt)]))
    return r._fp


def take_batch(ready, cap, in_use, budget, batch_flops, size=None):
    """The next batch for a free slot: ready requests, oldest first, while the
    batch holds fewer than `cap`, its counted flops stay within batch_flops
    (the first request always goes) and the in-flight workspace stays within
    `budget` (an idle device, in_use == 0, always takes the oldest request).
    size(r): workspace bytes of a request (default: footprint).  Returns
    (batch, its bytes, the requests left, in order)."""
    size = size or footprint
    batch, nbytes, work, rest = [], 0, 0.0, []
    for r in ready:
        # (conservative for a request that replays its graph, whose workspace
        # is resident: it may still join a batched call)
        f = size(r)
        fits = in_use + nbytes + f <= budget
        small = not batch or work + r.flops() <= batch_flops
        if len(batch) < cap and small and (fits or (in_use == 0 and not batch)):
            batch.append(r)
            nbytes += f
            work += r.flops()
        else:
            rest.append(r)
    return batch, nbytes, rest


class _Clock:
    """Device event times on the trace's host clock: an event recorded on an
    idle device at t0 = 0."""

    def __init__(self, torch, device):
        torch.cuda.synchronize(device)
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e0.record(torch.cuda.current_stream(device))
        torch.cuda.synchronize(device)
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def at(self, ev):
        """Time of a completed event: its device time after e0, but never
        later than now (the host time at which its completion is observed)."""
        return min(self.e0.elapsed_time(ev) * 1e-3, self.now())


def _key(r):
    return (r.q.data_ptr(), r.hh.data_ptr(), r.tau.data_ptr(), tuple(r.q.shape),
            tuple(r.q.stride()), str(r.q.dtype), r.nbw)


class Server:
    def __init__(self, device, slots=3, budget_bytes=None, max_batch=32, poll_s=50e-6,
                 batch_flops=5e10, call_streams=1, threads=True):
        import torch
        from concurrent.futures import ThreadPoolExecutor
        self.torch = torch
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        # one launcher thread per slot (threads=True): a launch call can block
        # the calling thread while the device works through earlier launches,
        # and a scheduler blocked there could neither feed the other slots
        # nor see completions
        self.workers = ([ThreadPoolExecutor(max_workers=1) for _ in range(slots)]
                        if threads else [])
        self.graphs = {}        # buffer set -> (prepared batch, captured graph)
        self.replays = 0
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(device)
            budget_bytes = int(0.5 * free)
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.batch_flops = float(batch_flops)
        self.call_streams = int(call_streams)
        self.poll_s = poll_s
        self.batches = []       # (slot, size, bytes) of every launch
        self.max_in_use = 0     # peak admitted workspace bytes
        self.max_busy = 0       # peak number of slots running at once
        self._launch_s = [0.0] * slots  # host time inside launch calls, per slot

    def prepare_graphs(self, requests, capture=True):
        """Prepared batch and captured graph for every distinct buffer set of
        the requests (setup, outside the timed service); capture=False keeps
        the prepared batches only, run eagerly (their launches issued one by
        one, without per-call allocation).  Returns the device bytes the
        prepared batches hold."""
        torch = self.torch
        cap = torch.cuda.Stream(device=self.device)
        for r in requests:
            k = _key(r)
            if k in self.graphs:
                continue
            b = B.Batch([(r.q, r.hh, r.tau, r.nbw)], streams=self.call_streams)
            g = None
            if capture:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=cap):
                    b.run(cap)
            self.graphs[k] = (b, g)
        torch.cuda.synchronize(self.device)
        return sum(b.nbytes for b, _ in self.graphs.values())

    def close_graphs(self):
        self.torch.cuda.synchronize(self.device)
        for b, _ in self.graphs.values():
            b.close()
        self.graphs = {}

    def run(self, requests):
        """Replay the requests' arrival times against the wall clock; returns
        when all are done.  Requests are updated in place with their times."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        done_at = {}
        waiting, ready = [], []
        busy = [None] * len(self.streams)  # (done ev, batch, bytes, start ev, launch)
        in_use = 0
        left = len(pending)
        pi = 0
        clock = _Clock(torch, self.device)
        while left:
            now = clock.now()
            progress = False
            for i, b in enumerate(busy):
                # (an event not yet recorded by the slot's launcher queries as
                # complete: the launch call must have returned first)
                if b is not None and (b[4] is None or b[4].done()) and b[0].query():
                    if b[4] is not None:
                        b[4].result()              # re-raise a launch error
                    t = clock.at(b[0])
                    t_s = clock.at(b[3])
                    for r in b[1]:
                        r.t_start = t_s
                        r.t_done = t
                        done_at[r.rid] = t
                    in_use -= b[2]
                    left -= len(b[1])
                    busy[i] = None
                    progress = True
            while pi < len(pending) and pending[pi].arrival <= now:
                waiting.append(pending[pi])
                pi += 1
            still = []
            for r in waiting:
                if r.after < 0 or r.after in done_at:
                    r.t_ready = max(r.arrival, done_at.get(r.after, 0.0))
                    ready.append(r)
                else:
                    still.append(r)
            waiting = still
            for i, b in enumerate(busy):
                if b is not None or not ready:
                    continue
                # spread the ready requests over the free slots before
                # batching them: a request batched with larger ones waits for
                # them, while one on a slot of its own overlaps with them
                free = sum(x is None for x in busy)
                cap = min(self.max_batch, -(-len(ready) // free))
                batch, nbytes, ready = take_batch(ready, cap, in_use, self.budget,
                                                  self.batch_flops)
                if not batch:
                    break
                ev0 = torch.cuda.Event(enable_timing=True)
                ev = torch.cuda.Event(enable_timing=True)
                if len(batch) == 1 and _key(batch[0]) in self.graphs:
                    self.replays += 1
                    batch[0].via = "graph"
                else:
                    for r in batch:
                        r.via = "single" if len(batch) == 1 else "batched"
                if self.workers:
                    fut = self.workers[i].submit(self._launch, i, batch, ev0, ev)
                else:
                    self._launch(i, batch, ev0, ev)
                    fut = None
                busy[i] = (ev, batch, nbytes, ev0, fut)
                in_use += nbytes
                self.batches.append((i, len(batch), nbytes))
                self.max_in_use = max(self.max_in_use, in_use)
                self.max_busy = max(self.max_busy, sum(x is not None for x in busy))
                progress = True
            if not progress:
                time.sleep(self.poll_s)
        return requests

    def _launch(self, i, batch, ev0, ev):
        """Issue one batch on slot i between its start and done events."""
        torch = self.torch
        st = self.streams[i]
        if self.workers:
            torch.cuda.set_device(self.device)
        ev0.record(st)
        tl = time.perf_counter()
        if batch[0].via == "graph":
            b, g = self.graphs[_key(batch[0])]
            if g is None:
                b.run(st)
            else:
                with torch.cuda.stream(st):
                    g.replay()
        elif len(batch) == 1:
            r = batch[0]
            B.hh_trafo(r.q, r.hh, r.tau, r.nbw, stream=st, streams=self.call_streams)
        else:
            B.hh_trafo_batched([(r.q, r.hh, r.tau, r.nbw) for r in batch], stream=st,
                               streams=self.call_streams)
        ev.record(st)
        self._launch_s[i] += time.perf_counter() - tl

    @property
    def launch_s(self):
        """Host seconds spent inside launch calls, summed over the slots."""
        return sum(self._launch_s)

    @launch_s.setter
    def launch_s(self, v):
        self._launch_s = [float(v) / len(self.streams)] * len(self.streams)

    def close(self):
        for w in self.workers:
            w.shutdown(wait=True)
        self.workers = []


def run_plain(requests, device, poll_s=50e-6, call_streams=0):
    """Baseline: one elpa_hh_trafo call at a time on one stream, in the order
    requests become ready, each waited for before the next starts (plan
    streams = call_streams; 0: the library's choice)."""
    import torch
    st = torch.cuda.Stream(device=device)
    order = sorted(requests, key=lambda r: r.arrival)
    done_at = {}
    clock = _Clock(torch, device)
    queue = list(order)
    while queue:
        now = clock.now()
        # oldest request whose dependency is met (requests are served in order)
        r = None
        for cand in queue:
            if cand.after < 0 or cand.after in done_at:
                r = cand
                break
        if r is None or r.arrival > now:
            time.sleep(poll_s)
            continue
        queue.remove(r)
        r.t_ready = max(r.arrival, done_at.get(r.after, 0.0))
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record(st)
        B.hh_trafo(r.q, r.hh, r.tau, r.nbw, stream=st, streams=call_streams)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(st)
        ev.synchronize()
        r.t_start = clock.at(ev0)
        r.t_done = clock.at(ev)
        done_at[r.rid] = r.t_done
    return requests


def latency_stats(requests):
    """solves/s over the trace (first arrival to last completion), counted
    flops per second, p50 / p99 / max latency in ms, and the mean service
    time (start to completion on the device) in ms."""
    import numpy as np
    lat = np.array([r.t_done - r.t_ready for r in requests]) * 1e3
    svc = np.array([r.t_done - r.t_start for r in requests]) * 1e3
    span = max(r.t_done for r in requests) - min(r.arrival for r in requests)
    fl = sum(r.flops() for r in requests)
    return {"solves": len(requests), "span_s": round(span, 4),
            "solves_per_s": round(len(requests) / span, 2),
            "gflops": round(fl / span / 1e9, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "service_ms": round(float(svc.mean()), 3)}
