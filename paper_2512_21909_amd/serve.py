"""Continuous-batching request loop for ladder-residual evaluations on one GPU.

Requests arrive over time, each with its inputs (Cholesky vectors and
amplitudes) already resident in device memory.  The server

* admits a waiting request when its device footprint (result buffers) fits the
  HBM budget that is left after resident workspaces and other admitted
  requests; a request that can never fit is rejected at submission;
* launches every batch of admitted requests as ONE batched library call
  (``cdcc_ladder_t2`` / ``cdcc_ladder_lambda`` with nsys = batch size) on a
  free stream, so that batches on different streams overlap on the device; a
  request of at least ``solo_flops`` runs as a batch of its own, so that the
  small requests of a batch never wait for a large one;
  before launching it reserves the batch's library workspace (queried with
  ``cdcc_workspace_bytes``; the library keeps a grow-only workspace per stream);
* retires batches by polling their completion events and records per-request
  latency (arrival -> result complete on the device, observed on the host).

On an allocation failure inside a batch the batch is split and its requests are
retried one by one, so one failing request does not fail the others.  Tile
shapes are chosen per system by the library, never per batch, so every result
is bitwise the same alone and in a mix.
"""
from __future__ import annotations

import collections
import dataclasses
import time

from . import _lib
from .ladder import ladder_lambda, ladder_t2, release, workspace_bytes
from .layout import Layout


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds on the server clock
    layout: Layout
    B: object                      # device tensor (resident)
    X: object                      # device tensor (resident)
    kind: str = "t2"               # "t2" or "lambda"
    Bvo: object = None
    t1: object = None
    flops: float = 0.0
    R: object = None
    pair_energy: object = None
    want_energy: bool = False
    solo: bool = False             # launch alone (after a batch hit an allocation failure)
    status: str = "new"            # new, waiting, admitted, running, done, rejected, failed
    error: str = ""
    t_admit: float = -1.0
    t_launch: float = -1.0
    t_done: float = -1.0

    def out_bytes(self) -> int:
        n = self.layout.amp_size * 8
        if self.want_energy:
            n += self.layout.nocc_tot ** 2 * 8
        return n

    def problem(self) -> dict:
        p = {"layout": self.layout, "B": self.B, "X": self.X, "R": self.R}
        if self.want_energy:
            p["pair_energy"] = self.pair_energy
        if self.kind == "lambda" and self.Bvo is not None:
            p["Bvo"], p["t1"] = self.Bvo, self.t1
        return p


class LadderServer:
    def __init__(self, hbm_budget_bytes: int, n_streams: int = 3, precision: str = "fp64",
                 max_batch: int = 16, batch_bytes: int = 256 << 20, clock=time.perf_counter,
                 solo_flops: float | None = 1e11):
        import torch
        self.torch = torch
        # a request of at least this many flops (1e11: about 1.5-2.5 ms of
        # device time, enough to fill the GPU alone) runs as a batch of its
        # own, and batches of smaller requests never wait for one; None
        # batches every request alike
        self.solo_flops = solo_flops
        self.budget = int(hbm_budget_bytes)
        self.precision = precision
        self.max_batch = max_batch
        self.batch_bytes = int(batch_bytes)
        self.clock = clock
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]   # default priority
        self.free = collections.deque(range(n_streams))
        self.ws_reserved = [0] * n_streams      # library workspace held per stream (grow-only)
        self.out_reserved = 0                   # result buffers of admitted / running requests
        self.waiting: collections.deque[Request] = collections.deque()
        self.ready: list[Request] = []
        self.running = []                       # (stream, event, [requests])
        self.finished: list[Request] = []
        self.t0 = None

    # -- accounting -------------------------------------------------------
    def _free_bytes(self) -> int:
        return self.budget - self.out_reserved - sum(self.ws_reserved)

    def submit(self, req: Request) -> None:
        lone_ws = workspace_bytes(req.problem() | {"R": req.X}, req.kind == "lambda", self.precision,
                                  batch_bytes=self.batch_bytes)
        if req.out_bytes() + lone_ws > self.budget:
            req.status, req.error = "rejected", "footprint exceeds the HBM budget"
            self.finished.append(req)
            return
        req.status = "waiting"
        self.waiting.append(req)

    # -- the loop ---------------------------------------------------------------
    def _retire(self, now: float) -> None:
        keep = []
        for s, ev, reqs in self.running:
            if ev.query():
                for r in reqs:
                    r.t_done, r.status = now, "done"
                    self.finished.append(r)
                self.free.append(s)
            else:
                keep.append((s, ev, reqs))
        self.running = keep

    def _admit(self, now: float) -> None:
        torch = self.torch
        while self.waiting and self.waiting[0].out_bytes() <= self._free_bytes():
            r = self.waiting.popleft()
            r.R = torch.empty(r.layout.amp_size, dtype=torch.float64, device="cuda")
            if r.want_energy:
                r.pair_energy = torch.empty(r.layout.nocc_tot ** 2, dtype=torch.float64, device="cuda")
            self.out_reserved += r.out_bytes()
            r.t_admit, r.status = now, "admitted"
            self.ready.append(r)

    def _launch(self) -> None:
        while self.ready and self.free:
            head = self.ready[0]
            if head.solo or self._heavy(head):
                batch = [head]
            else:
                batch = [r for r in self.ready
                         if r.kind == head.kind and not r.solo and not self._heavy(r)][:self.max_batch]
            probs = [r.problem() for r in batch]
            need = workspace_bytes(probs, head.kind == "lambda", self.precision, batch_bytes=self.batch_bytes)
            s = self.free[0]
            if max(0, need - self.ws_reserved[s]) > self._free_bytes():
                if self.running:
                    break                          # wait until memory frees up
                # nothing in flight will free memory: drop the cached workspaces
                release()
                self.ws_reserved = [0] * len(self.streams)
                if need > self._free_bytes():
                    if len(batch) > 1:
                        for r in batch:
                            r.solo = True
                        continue
                    head.status, head.error = "failed", "workspace exceeds the HBM budget"
                    self.out_reserved -= head.out_bytes()
                    head._released = True
                    self.finished.append(head)
                    self.ready.pop(0)
                    continue
            self.free.popleft()
            ids = {id(r) for r in batch}
            self.ready = [r for r in self.ready if id(r) not in ids]
            stream = self.streams[s]
            # the inputs were written on the current stream: order after it
            stream.wait_stream(self.torch.cuda.current_stream())
            try:
                fn = ladder_t2 if head.kind == "t2" else ladder_lambda
                fn(probs, precision=self.precision, stream=stream, batch_bytes=self.batch_bytes)
            except _lib.CdccError as e:
                self.free.appendleft(s)
                if e.status == _lib.ENOMEM and len(batch) > 1:
                    for r in batch:
                        r.solo = True             # retry alone: one failure must not fail the rest
                    self.ready = batch + self.ready
                    continue
                for r in batch:
                    r.status, r.error = "failed", str(e)
                    self.out_reserved -= r.out_bytes()
                    r._released = True
                    self.finished.append(r)
                continue
            self.ws_reserved[s] = max(self.ws_reserved[s], need)
            ev = self.torch.cuda.Event()
            ev.record(stream)
            now = self.clock() - self.t0
            for r in batch:
                r.t_launch, r.status = now, "running"
            self.running.append((s, ev, batch))

    def _heavy(self, r: Request) -> bool:
        return self.solo_flops is not None and r.flops >= self.solo_flops

    def _release_done(self) -> None:
        for r in self.finished:
            if r.status == "done" and r.R is not None and not getattr(r, "_released", False):
                self.out_reserved -= r.out_bytes()
                r._released = True

    def serve(self, requests: list[Request], poll_sleep: float = 0.0) -> list[Request]:
        """Run until every request is finished.  ``requests`` carry arrival
        times relative to the start; they are submitted when their time comes."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = self.clock()
        i = 0
        while i < len(pending) or self.waiting or self.ready or self.running:
            now = self.clock() - self.t0
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            self._retire(now)
            self._release_done()
            self._admit(now)
            self._launch()
            if poll_sleep:
                time.sleep(poll_sleep)
        self.torch.cuda.synchronize()
        return self.finished


def latency_stats(reqs: list[Request]) -> dict:
    import numpy as np
    done = [r for r in reqs if r.status == "done"]
    if not done:
        return {"done": 0}
    lat = np.array([r.t_done - r.arrival for r in done])
    span = max(r.t_done for r in done) - min(r.arrival for r in done)
    fl = sum(r.flops for r in done)
    return {"done": len(done), "rejected": sum(r.status == "rejected" for r in reqs),
            "failed": sum(r.status == "failed" for r in reqs),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "tflops": fl / span / 1e12 if span > 0 else 0.0,
            "requests_per_s": len(done) / span if span > 0 else 0.0}


def make_stream(pool, n: int, rate_hz: float, seed: int = 5, p_large: float = 0.1, want_energy=True):
    """Poisson arrivals; each request takes a pool shape (large with
    probability p_large, else a uniformly drawn small shape)."""
    import numpy as np
    rng = np.random.default_rng([seed, 7])
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n)) if rate_hz > 0 else np.zeros(n)
    small = [p for p in pool if not p["large"]]
    large = [p for p in pool if p["large"]]
    reqs = []
    for k in range(n):
        p = large[0] if (large and rng.random() < p_large) else small[int(rng.integers(len(small)))]
        reqs.append(Request(rid=k, arrival=float(t[k]), layout=p["layout"], B=p["B"], X=p["X"],
                            flops=p["flops"], want_energy=want_energy))
    return reqs


def measure(pool, precision="fp64", n_requests=2000, warmup=200, load=0.7, n_streams=3, max_batch=16, seed=5,
            **server_kw):
    """Warm-up (``warmup`` requests at t=0, at least two per pool shape, not
    counted), saturation throughput of the mix (``n_requests`` at t=0), then a
    Poisson stream of ``n_requests`` at ``load`` times that rate.  ``pool``:
    device-resident request inputs (dicts with layout, B, X, flops, large)."""
    out = measure_sweep(pool, precision, n_requests, (load,), n_streams, max_batch, seed, warmup, **server_kw)
    st = out.pop("streams")[0]
    out["load"], out["rate_hz"] = st.pop("load"), st.pop("rate_hz")
    out["stream"] = st
    return out


def measure_sweep(pool, precision="fp64", n_requests=2000, loads=(0.3, 0.5, 0.7, 0.9), n_streams=3,
                  max_batch=16, seed=5, warmup=200, log=None, **server_kw):
    """Warm-up (``warmup`` requests at t=0, at least two per pool shape, not
    counted), saturation throughput of the mix, then one Poisson stream of
    ``n_requests`` per entry of ``loads`` (a fraction of the saturation
    rate).  ``log(str)`` is called after each measured run; ``server_kw``
    go to every ``LadderServer``."""
    import torch
    free, total = torch.cuda.mem_get_info()
    budget = int(free * 0.6)

    def server():
        return LadderServer(budget, n_streams, precision, max_batch, **server_kw)

    server().serve(make_stream(pool, max(warmup, 2 * len(pool)), 0, seed + 1))
    sat = latency_stats(server().serve(make_stream(pool, n_requests, 0.0, seed)))
    if log:
        log(f"{precision} saturation: {sat.get('requests_per_s', 0):.1f} requests/s")
    out = {"precision": precision, "requests": n_requests, "warmup": warmup, "saturation": sat, "streams": [],
           "n_streams": n_streams, "max_batch": max_batch, "hbm_budget_bytes": budget}
    for load in loads:
        rate = load * sat["requests_per_s"]
        st = latency_stats(server().serve(make_stream(pool, n_requests, rate, seed)))
        out["streams"].append({"load": load, "rate_hz": rate, **st})
        if log:
            log(f"{precision} load {load}: p50 {st.get('p50_ms', 0):.2f} ms, p99 {st.get('p99_ms', 0):.2f} ms")
    return out
