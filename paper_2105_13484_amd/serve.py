"""Serving forecast requests: continuous batching under a device-memory budget.

Requests (a mesh, parameters, an initial state and a number of steps) arrive
over time.  The engine keeps every admitted request's state resident in HBM
and advances all of them together:

* admission: first come, first served; a request is admitted as soon as it
  has arrived and its footprint (mesh image + workspace, from the library)
  fits in the remaining budget;
* one batch per precision (FP64 and mixed), each on its own HIP stream, so
  the two kinds of requests run concurrently on the device; within a batch
  one launch per step phase covers every member;
* each batch advances in chunks of at most `chunk_steps` steps, never past
  the nearest completion of its members, so that finished requests leave and
  waiting ones join between chunks; a batch gets its next chunk as soon as
  its last one has finished, without waiting for the other batch; a request
  that arrives while chunks run is set up (its mesh image built on the host
  and uploaded) meanwhile, and its batch's program is rebuilt before that
  batch's next chunk;
* a finished request's state is read back and its device memory released.

A request's result does not depend on what else runs: a batch member
computes exactly what it computes alone (the GPU tests compare them bit for
bit).  Time-to-completion is measured from arrival to the result being on
the host.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import ssprkse


@dataclass
class Request:
    rid: int
    case: object          # synthetic case: mesh, params (incl. precision), initial state
    steps: int
    arrival: float        # seconds after the start of the run
    footprint: int = 0
    admitted: float | None = None
    done: float | None = None
    status: int = 0
    result: dict | None = None

    @property
    def work(self) -> int:
        """Cell-layer updates the request asks for."""
        return int(self.case.active_cell_layers) * int(self.steps)


@dataclass
class _Active:
    req: Request
    mesh: object
    state: object
    remaining: int


@dataclass
class Engine:
    budget_bytes: int = 200 << 30
    chunk_steps: int = 10
    device: str = "cuda:0"
    keep_results: bool = True
    poll_s: float = 2e-4          # wait between checks for a finished chunk
    _streams: dict = field(default_factory=dict)
    _batches: dict = field(default_factory=dict)
    _active: dict = field(default_factory=lambda: collections.defaultdict(list))
    used_bytes: int = 0

    def _batch(self, precision: int):
        import torch
        if precision not in self._batches:
            self._streams[precision] = torch.cuda.Stream(device=self.device)
            self._batches[precision] = ssprkse.Batch(stream=self._streams[precision])
        return self._batches[precision]

    def footprint(self, req: Request) -> int:
        return ssprkse.footprint_bytes(req.case.mesh, req.case.params)

    def _admit(self, req: Request, now: float):
        prec = int(req.case.params.precision)
        b = self._batch(prec)
        dm, st = ssprkse.state_from_case(req.case, device=self.device, stream=self._streams[prec])
        b.add(st)
        req.admitted = now
        self.used_bytes += req.footprint
        self._active[prec].append(_Active(req, dm, st, int(req.steps)))

    def _finish(self, prec: int, a: _Active, now: float, status: int):
        b = self._batches[prec]
        b.remove(a.state)
        a.req.status = status
        if self.keep_results:
            a.req.result = a.state.read()
        a.state.close()
        a.mesh.close()
        a.req.done = now
        self.used_bytes -= a.req.footprint

    def run(self, requests, clock=time.perf_counter, on_progress=None) -> dict:
        """Serve `requests` (arrival times relative to the start); blocks until all finish."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        for r in pending:
            r.footprint = self.footprint(r)
            if r.footprint > self.budget_bytes:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, more than the budget")
        t0 = clock()
        finished = []
        total = len(pending)

        def admit():
            # FIFO, no overtaking
            while pending and pending[0].arrival <= clock() - t0 and \
                    self.used_bytes + pending[0].footprint <= self.budget_bytes:
                self._admit(pending.popleft(), clock() - t0)

        in_flight = {}   # precision -> (steps of the chunk, members it advances)
        while len(finished) < total:
            # every idle batch with members gets its next chunk
            for p in list(self._active):
                if self._active[p] and p not in in_flight:
                    k = min(self.chunk_steps, min(a.remaining for a in self._active[p]))
                    self._batches[p].step_async(k)
                    in_flight[p] = (k, len(self._active[p]))
            # requests that have arrived are set up while the chunks run; they
            # join their batch with its next chunk
            admit()
            if not in_flight:
                if pending and not any(self._active[p] for p in self._active):
                    time.sleep(max(0.0, min(pending[0].arrival - (clock() - t0), 0.01)))
                continue
            ready = [p for p in in_flight if self._batches[p].query()]
            if not ready:
                time.sleep(self.poll_s)
                continue
            for p in ready:
                k, joined = in_flight.pop(p)
                rc = self._batches[p].sync()
                now = clock() - t0
                still = []
                ran, newcomers = self._active[p][:joined], self._active[p][joined:]
                for a in ran:
                    a.remaining -= k
                    if rc != 0:
                        st_rc = a.state.sync()
                        if st_rc != 0:
                            self._finish(p, a, now, st_rc)
                            finished.append(a.req)
                            continue
                    if a.remaining <= 0:
                        self._finish(p, a, now, 0)
                        finished.append(a.req)
                    else:
                        still.append(a)
                self._active[p] = still + newcomers   # admitted during the chunk, not stepped yet
            if on_progress:
                on_progress(len(finished), total)
        wall = clock() - t0
        lat = sorted(r.done - r.arrival for r in finished)

        def pct(q):
            # linear interpolation between the two nearest order statistics
            x = q * (len(lat) - 1)
            i = min(int(x), len(lat) - 1)
            j = min(i + 1, len(lat) - 1)
            return lat[i] + (x - i) * (lat[j] - lat[i])

        work = sum(r.work for r in finished)
        return {"requests": total, "wall_s": wall, "p50_s": pct(0.50), "p99_s": pct(0.99), "max_s": lat[-1],
                "mean_s": sum(lat) / len(lat), "cell_layer_updates_per_s": work / wall,
                "failed": sum(1 for r in finished if r.status != 0)}

    def close(self):
        for b in self._batches.values():
            b.close()
        self._batches.clear()


def poisson_arrivals(n: int, rate_per_s: float, seed: int):
    """n arrival times of a Poisson process of the given rate (seeded)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n)).tolist()
