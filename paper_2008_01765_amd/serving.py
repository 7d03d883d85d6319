"""Serving loop for bucket oblivious sort requests on one GPU.

Requests (record tensors already in HBM) queue up in arrival order.  Between
scheduler steps the server admits queued requests while their HBM footprint
(input + output + the sort's workspace) fits under the budget; each step then
runs one bos_sort_step call over the resident requests: a budget of device
work handed out in admission order, each request running as many phases of its
sort as fit (a phase is a routing pass of the butterfly network of Section 3.2,
the tile sort or a merge pass of the comparison sort that Section 3.3 applies
to the permuted array; the overflow check closes the step).  Requests of different sizes and phases share
the step's launches, and new requests start at the next step boundary
(continuous batching).  A finished request frees its memory and records its
completion time.

Every result is the one bos.sort gives for the same input alone: the sort's
output is the sorted array whatever the seed, and each request keeps its own
seed and attempt counter through the steps.
"""
import ctypes
import time
import weakref
from collections import deque

import numpy as np
import torch

from . import bos


def admit_prefix(footprints, free_bytes):
    """How many of the queued requests, taken in order, fit in free_bytes.

    Admission is first-come first-served: it stops at the first request that
    does not fit, so a large request is not starved by smaller ones behind it.
    """
    k = 0
    for f in footprints:
        if f > free_bytes:
            break
        free_bytes -= f
        k += 1
    return k


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence."""
    v = sorted(values)
    if not v:
        raise ValueError("percentile of an empty sequence")
    rank = max(1, -(-len(v) * q // 100))
    return v[int(rank) - 1]


# layout of bos.Job (bos_job in bos.h) for a numpy view of a job array
_JOB_DTYPE = np.dtype([("in_", "<u8"), ("out", "<u8"), ("n", "<u8"), ("seed", "<u8"), ("ws", "<u8"),
                       ("ws_bytes", "<u8"), ("phase", "<u4"), ("attempt", "<u4"), ("status", "<u4"),
                       ("reserved", "<u4")])
assert _JOB_DTYPE.itemsize == ctypes.sizeof(bos.Job)


class Future:
    """Handle of one submitted request."""

    def __init__(self, server, rid, tensor, seed, arrival):
        self._server = weakref.ref(server)  # the server holds its resident futures, not the reverse
        self.id = rid
        self.input = tensor
        self.n = tensor.shape[0]
        self.seed = seed
        self.arrival = arrival
        self.admitted = None
        self.finished = None
        self.status = None
        self.out = None
        self.attempts = 0
        self.steps = 0
        self.footprint = 0
        self.phase = 0
        self._ws = None
        self._step0 = 0
        self._ready = None   # event on the submitter's stream after which the input is valid
        self._done = None    # event on the server's stream after the request's last step

    def done(self):
        return self.finished is not None

    def result(self):
        """Block (driving the server) until this request is done; returns its
        sorted tensor or raises BosError if every routing attempt overflowed."""
        while not self.done():
            server = self._server()
            if server is None:
                raise RuntimeError("the server of this request was discarded before it finished")
            server.step()
        if self.status != bos.OK:
            raise bos.BosError(self.status, "libbos: " + bos.lib().bos_status_string(self.status).decode())
        if self._done is not None:
            # the caller's stream reads the output after the server's stream
            # has written it; the output's memory is then released in the
            # caller's stream order as well
            cur = torch.cuda.current_stream(self.out.device)
            cur.wait_event(self._done)
            self.out.record_stream(cur)
        return self.out

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class Server:
    """Continuous-batching server of bucket oblivious sorts on one device.

    hbm_budget_bytes bounds the sum of the resident requests' footprints;
    z, k, tile (the comparison sort's tile), max_retries and min_security_bits
    are shared by every request (the step entry point takes one parameter
    block; 0 = the tuning table's choice per request size).  All requests must use the
    same record type.  pipeline=True drives the steps through a stepper
    (bos_sort_step_async): the device runs one step while the host plans the
    next, and a request is reported finished one call after its last step
    was enqueued, as soon as that step has completed.

    stream: the stream the steps run on (None: the current stream at each
    call).  With a stream of its own the server allocates outputs and
    workspaces on that stream (so freed blocks are reused in its order), has
    it wait for the submitter's stream before a request's first step, and
    makes the caller's stream wait for the request's last step in result().
    """

    def __init__(self, hbm_budget_bytes=64 << 30, z=0, k=0, max_retries=3, min_security_bits=80,
                 device=None, stream=None, clock=time.perf_counter, pipeline=True, tile=0):
        self.budget = int(hbm_budget_bytes)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        self.clock = clock
        self.params = bos.params(0, z, k, tile, max_retries, min_security_bits, sync=True)
        self.rec = None
        self.queue = deque()
        self.active = []
        self.used = 0
        self.peak_used = 0
        self.steps = 0
        self._next_id = 0
        self._step_ws = None
        self._jobs = None  # ctypes array of the resident requests' jobs, in self.active's order
        self._stepper = bos.Stepper() if pipeline else None
        self.completed = 0  # requests finished so far (their futures belong to the callers)

    # ---- admission ---------------------------------------------------------
    def footprint(self, n, rec):
        return 2 * n * rec + bos.workspace_bytes(n, rec, self.params) if n else 0

    def submit(self, tensor, seed=None, arrival=None):
        """Queue one request (an (n, 2) record tensor on the server's device)."""
        rec = bos.rec_bytes(tensor)
        if self.rec is None:
            self.rec = rec
        elif rec != self.rec:
            raise ValueError("all requests of a server must use the same record type")
        if tensor.device != self.device:
            raise ValueError("request tensor is on %s, server on %s" % (tensor.device, self.device))
        rid = self._next_id
        self._next_id += 1
        f = Future(self, rid, tensor, rid if seed is None else seed, self.clock() if arrival is None else arrival)
        if self.stream is not None:
            cur = torch.cuda.current_stream(self.device)
            if cur != self.stream:
                f._ready = torch.cuda.Event()
                f._ready.record(cur)
                tensor.record_stream(self.stream)  # not reused before the server's stream is done with it
        if f.n:
            bos.plan(f.n, rec, self.params.z, self.params.k, 0, self.params.min_security_bits)  # raises if Z is rejected
        f.footprint = self.footprint(f.n, rec)
        if f.footprint > self.budget:
            raise bos.BosError(bos.WORKSPACE, "request of %d records needs %d bytes, over the %d-byte budget"
                               % (f.n, f.footprint, self.budget))
        self.queue.append(f)
        return f

    def _on_stream(self):
        """Context that makes the server's stream current (allocations then
        belong to it)."""
        if self.stream is None:
            return _NoStream()
        return torch.cuda.stream(self.stream)

    def _admit(self):
        # lazily: admission stops at the first request that does not fit
        k = admit_prefix((f.footprint for f in self.queue), self.budget - self.used)
        if k == 0:
            return 0
        now = self.clock()
        new = []
        with self._on_stream():
            for _ in range(k):
                f = self.queue.popleft()
                f.admitted = now
                f._step0 = self.steps
                if f._ready is not None:
                    self.stream.wait_event(f._ready)
                f.out = torch.empty_like(f.input)
                if f.n:
                    f._ws = torch.empty(max(bos.workspace_bytes(f.n, self.rec, self.params), 256),
                                        dtype=torch.uint8, device=self.device)
                self.used += f.footprint
                new.append(f)
        # job array: the resident jobs' entries (phase and attempt as the
        # last step left them) followed by the new ones
        old = len(self.active)
        jobs = (bos.Job * (old + k))()
        if old:
            np.frombuffer(jobs, dtype=_JOB_DTYPE, count=old)[:] = np.frombuffer(self._jobs, dtype=_JOB_DTYPE,
                                                                               count=old)
        for i, f in enumerate(new):
            j = jobs[old + i]
            j.in_ = f.input.data_ptr()
            j.out = f.out.data_ptr()
            j.n = f.n
            j.seed = f.seed & 0xFFFFFFFFFFFFFFFF
            j.ws = f._ws.data_ptr() if f._ws is not None else None
            j.ws_bytes = f._ws.numel() if f._ws is not None else 0
        self._jobs = jobs
        self.active.extend(new)
        self.peak_used = max(self.peak_used, self.used)
        return k

    # ---- scheduling --------------------------------------------------------
    def idle(self):
        return not self.queue and not self.active

    def step(self):
        """Admit what fits, run one bos_sort_step over the resident requests
        and retire the finished ones; returns the requests finished in this
        step."""
        if self.queue:
            self._admit()
        if not self.active:
            return []
        cnt = len(self.active)
        jobs = self._jobs  # the step updates phase, attempt and status in place
        need = bos.step_workspace_bytes(cnt) * (2 if self._stepper else 1)
        if self._step_ws is None or self._step_ws.numel() < need:
            # a replaced buffer is released in the order of the stream it was
            # allocated on (the server's), after the step in flight that may
            # still read it
            with self._on_stream():
                self._step_ws = torch.empty(2 * need, dtype=torch.uint8, device=self.device)
        if self._stepper:
            self._stepper.step(jobs, self.rec, self.params, self._step_ws, self.stream)
        else:
            bos.sort_step(jobs, self.rec, self.params, self._step_ws, self.stream, count_left=False)
        self.steps += 1
        now = self.clock()
        view = np.frombuffer(jobs, dtype=_JOB_DTYPE, count=cnt)
        fin = view["phase"] == bos.PHASE_DONE
        if not fin.any():
            return []
        done = []
        ev = None
        if self.stream is not None:
            ev = torch.cuda.Event()
            ev.record(self.stream)  # after every step enqueued so far
        for i in np.flatnonzero(fin).tolist():
            f = self.active[i]
            f._done = ev
            f.phase = bos.PHASE_DONE
            f.attempts = int(view["attempt"][i])
            f.status = int(view["status"][i])
            f.steps = self.steps - f._step0
            f.finished = now
            f._ws = None
            self.used -= f.footprint
            done.append(f)
        keep = np.flatnonzero(~fin)
        left = (bos.Job * len(keep))()
        if len(keep):
            np.frombuffer(left, dtype=_JOB_DTYPE, count=len(keep))[:] = view[keep]
        self._jobs = left
        self.active = [self.active[i] for i in keep.tolist()]
        self.completed += len(done)
        return done

    def run_until_idle(self):
        while not self.idle():
            self.step()


class _NoStream:
    def __enter__(self):
        return None

    def __exit__(self, *exc):
        return False


def run_trace(server, tensors, arrivals, seeds=None, spin=True):
    """Replay an arrival trace (seconds from now, ascending) through `server`;
    returns the futures in submission order."""
    clock = server.clock
    t0 = clock()
    futs = []
    i = 0
    N = len(tensors)
    while i < N or not server.idle():
        now = clock() - t0
        while i < N and arrivals[i] <= now:
            futs.append(server.submit(tensors[i], seed=None if seeds is None else seeds[i], arrival=t0 + arrivals[i]))
            i += 1
        if server.idle():
            if i < N and spin:
                while clock() - t0 < arrivals[i]:
                    pass
            continue
        server.step()
    return futs


def run_trace_sequential(tensors, arrivals, z=0, k=0, seeds=None, clock=time.perf_counter, stream=None,
                         keep_outputs=True):
    """First-come first-served baseline: each request sorted alone by bos.sort
    once it has arrived and the previous one has finished.  Returns
    (latencies, outputs); outputs is None with keep_outputs=False."""
    t0 = clock()
    lat, outs = [], []
    for i, t in enumerate(tensors):
        while clock() - t0 < arrivals[i]:
            pass
        o = bos.sort(t, seed=i if seeds is None else seeds[i], z=z, k=k, stream=stream)
        torch.cuda.synchronize()
        lat.append(clock() - t0 - arrivals[i])
        if keep_outputs:
            outs.append(o)
        del o
    return lat, (outs if keep_outputs else None)


def poisson_arrivals(count, rate_per_s, seed=11):
    """Arrival times of a Poisson process (exponential gaps from splitmix64)."""
    import numpy as np

    from . import inputs

    u = (inputs.splitmix64(seed, 0, count) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps).tolist()


__all__ = ["Server", "Future", "admit_prefix", "percentile", "run_trace", "run_trace_sequential",
           "poisson_arrivals"]
