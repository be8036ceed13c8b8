"""Serving loop: continuous batching of adiabatic-evolution solve requests.

Requests arrive over time (e.g. a Poisson process).  Each request is a full
solve psi(0) = |+>^n -> psi(T) of an interpolated Hamiltonian, followed by the
ground-state fidelity at T (Sec. III.B).  The server

  * admits a request as soon as a slot is free and its state plus workspace fit
    the HBM budget (requests wait in arrival order otherwise);
  * keeps every admitted state resident on the device until it finishes;
  * runs one batch (aqc_batch_*) per size class, each on its own stream and
    host thread, so that small solves keep stepping while a large one occupies
    the device, and the classes' kernels overlap on the GPU;
  * lets requests join and leave the running batch between ticks (continuous
    batching), and records arrival, admission and finish times.

A solve's arithmetic does not depend on the batch it runs in (the batch engine
replays the single-solve launch sequence), so each result equals the result
of solving the request alone.
"""
from __future__ import annotations

import math
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import engine

STAB_H_RHO = 0.1   # step from the stability guard: h * rho = 0.1


@dataclass
class Request:
    rid: int
    inst: object              # instances.Instance
    arrival: float = 0.0      # seconds after the start of the run
    n: int = 0
    T: float = 0.0

    def __post_init__(self):
        self.n = int(self.inst.n)
        self.T = float(self.inst.path["T"])


@dataclass
class Result:
    rid: int
    n: int
    steps: int
    fidelity: float
    e_min: float
    arrival: float
    admitted: float
    finished: float
    klass: int
    extra: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.finished - self.arrival


def choose_plan(ctx, ham, inst, dtype, autotune=False, wide_register_passes=True):
    """The pass plan a served solve runs: the plan tuned by batch tick time
    (cached per kind of problem), or else the default tiling with wide register
    passes when asked.  In a batch the workgroups of all solves fill the GPU
    together, so wide passes (fewer passes, fewer bytes) win even where a
    single small solve would not fill it.  A solve run alone with the same
    plan gives the same result bit for bit."""
    from . import autotune as at
    if autotune:
        return at.tune_cached(ctx, ham, inst, dtype, batch=True)[0]
    tiling = at.default_tiling(dtype)
    if wide_register_passes:
        tiling = (*tiling[:3], (tiling[3] & 4) | 3)
        ham.set_tiling(dtype, *tiling)
    return tiling


def warm_plans(requests, dtype=torch.complex64, device=0):
    """Tune (by batch tick time) every kind of problem among the requests once,
    so admissions find the plan in the tuning cache; returns the number of
    kinds tuned."""
    from . import autotune as at
    ctx = engine.Context(device)
    seen = set()
    dt = engine.dtype_code(torch.empty(0, dtype=dtype))
    for req in requests:
        key = at.structure_key(req.inst, dt)
        if key in seen:
            continue
        seen.add(key)
        ham = engine.Hamiltonian(ctx, req.inst)
        at.tune_cached(ctx, ham, req.inst, dtype, batch=True)
        ham.free()
    ctx.close()
    return len(seen)


def solve_plan(ctx, ham, T):
    """Step count and shift of a full solve on [0, T]: centred shift, h rho = 0.1."""
    lo, hi = ham.spectral_bounds(0.0, T)
    rho = 0.5 * (hi - lo)
    K = max(4, int(math.ceil(T * rho / STAB_H_RHO)))
    return K, 0.5 * (lo + hi)


def state_bytes(n, dtype):
    es = 8 if dtype == torch.complex64 else 16
    return (1 << n) * es


class _Class:
    def __init__(self, server, idx, max_n, capacity):
        self.server = server
        self.idx = idx
        self.max_n = max_n
        self.stream = torch.cuda.Stream(device=server.device)   # default priority
        self.ctx = engine.Context(server.device.index or 0, stream=self.stream)
        self.batch = engine.Batch(self.ctx, server.dtype, capacity=capacity, graph=server.graph,
                                  resident_max_n=min(server.resident_max_n, max_n))
        self.queue = []
        self.live = {}      # slot -> (request, ham, bytes, admitted time)
        self.lock = threading.Lock()
        self.thread = None
        self.ticks_done = 0

    def run(self):
        srv = self.server
        with torch.cuda.stream(self.stream):
            while True:
                now = srv.now()
                # admit arrived requests in order while memory and slots allow
                with self.lock:
                    while self.queue and self.queue[0].arrival <= now and len(self.live) < self.batch.capacity:
                        req = self.queue[0]
                        need = srv.request_bytes(req.n)
                        if not srv.reserve(need):
                            break
                        self.queue.pop(0)
                        self._admit(req, need)
                if self.live:
                    self.batch.step(srv.ticks)
                    self.ticks_done += srv.ticks
                    for slot in self.batch.poll():
                        self._finish(slot)
                    srv.report_ticks(self)
                else:
                    with self.lock:
                        empty = not self.queue
                        nxt = self.queue[0].arrival if self.queue else None
                    if empty and srv.closed.is_set():
                        return
                    wait = 0.002 if nxt is None else max(0.0, min(0.05, nxt - srv.now()))
                    time.sleep(wait)

    def _admit(self, req, need):
        srv = self.server
        ham = engine.Hamiltonian(self.ctx, req.inst)
        choose_plan(self.ctx, ham, req.inst, srv.dtype, srv.autotune, srv.wide_register_passes)
        K, shift = solve_plan(self.ctx, ham, req.T)
        N = 1 << req.n
        psi = torch.full((N,), 1.0 / math.sqrt(N), dtype=srv.dtype, device=srv.device)
        slot = self.batch.admit(ham, psi, 0.0, req.T, K, shift)
        self.live[slot] = (req, ham, need, srv.now())
        srv.n_admitted += 1
        if srv.progress and srv.n_admitted % (8 * srv.progress) == 0:
            srv.log(f"{srv.n_admitted} admitted, t={srv.now():.1f}s")

    def _finish(self, slot):
        srv = self.server
        psi, st = self.batch.retire(slot)
        req, ham, need, t_adm = self.live.pop(slot)
        mass, emin = engine.ground_mass(self.ctx, ham, req.T, psi)
        t_fin = srv.now()
        res = Result(req.rid, req.n, int(st["steps"]), mass, emin, req.arrival, t_adm, t_fin,
                     self.idx)
        if srv.keep_states:
            res.extra["psi"] = psi.detach().cpu().numpy()
        ham.free()
        del psi
        srv.release(need)
        srv.add_result(res)


class Server:
    """size_classes: ((max_n, capacity), ...) in increasing max_n.
    resident_max_n: solves of at most this many qubits run as resident solves
    of their batch (aqc_batch_set_resident), 0 for none."""

    def __init__(self, device=0, dtype=torch.complex64, hbm_budget_bytes=200e9,
                 size_classes=((20, 256), (34, 8)), ticks=8, graph=True, keep_states=False,
                 autotune=False, progress=0, wide_register_passes=True, resident_max_n=0):
        self.device = torch.device("cuda", device)
        self.dtype = dtype
        self.budget = float(hbm_budget_bytes)
        self.used = 0.0
        self.ticks = ticks
        self.graph = graph
        self.keep_states = keep_states
        self.autotune = autotune
        self.wide_register_passes = wide_register_passes
        # solves up to this size run as resident solves (one workgroup each)
        self.resident_max_n = resident_max_n
        self.progress = progress     # print a line every `progress` results (0: quiet)
        self.n_admitted = 0
        self._last_report = 0.0
        self._mem = threading.Lock()
        self._res = threading.Lock()
        self.results = []
        self.closed = threading.Event()
        self.t_start = None
        self.classes = [_Class(self, i, mx, cap) for i, (mx, cap) in enumerate(size_classes)]

    def now(self):
        return time.perf_counter() - self.t_start

    def request_bytes(self, n):
        # the state plus the predictor-corrector workspace (at most 8 vectors:
        # y^p and its second buffer, four history vectors, the partial
        # product of the high passes and the compensation part)
        return 9 * state_bytes(n, self.dtype)

    def reserve(self, b):
        with self._mem:
            if self.used + b > self.budget:
                return False
            self.used += b
            return True

    def release(self, b):
        with self._mem:
            self.used -= b

    def log(self, msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    def add_result(self, r):
        with self._res:
            self.results.append(r)
            if self.progress and len(self.results) % self.progress == 0:
                active = sum(len(c.live) for c in self.classes)
                self.log(f"{len(self.results)} done, {active} running, t={self.now():.1f}s")

    def report_ticks(self, klass):
        """A progress line after a batch step, at most every 20 seconds."""
        if not self.progress:
            return
        with self._res:
            now = self.now()
            if now - self._last_report < 20.0:
                return
            self._last_report = now
            self.log(f"class {klass.idx}: {klass.ticks_done} ticks, {len(klass.live)} running, "
                     f"{len(self.results)} done, t={now:.1f}s")

    def run(self, requests):
        """Serve the requests (arrival times relative to the start); returns
        (results sorted by id, wall seconds)."""
        for r in sorted(requests, key=lambda q: q.arrival):
            if self.request_bytes(r.n) > self.budget:
                raise ValueError(f"request {r.rid} (n={r.n}) exceeds the HBM budget")
            k = next(i for i, c in enumerate(self.classes) if r.n <= c.max_n)
            self.classes[k].queue.append(r)
        self.t_start = time.perf_counter()
        self.closed.set()   # every request is queued; workers stop when drained
        for c in self.classes:
            c.thread = threading.Thread(target=c.run, daemon=True)
            c.thread.start()
        for c in self.classes:
            c.thread.join()
        torch.cuda.synchronize()
        wall = self.now()
        return sorted(self.results, key=lambda r: r.rid), wall

    def close(self):
        for c in self.classes:
            c.batch.close()
            c.ctx.close()


def poisson_arrivals(n_requests, qps, seed=4):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=n_requests))


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=float), q)) if len(xs) else float("nan")


def sequential_plain(requests, device=0, dtype=torch.complex128, progress=False):
    """The plain path: each request solved alone with aqc_evolve, one after the
    other in arrival order.  Returns per-request (service seconds, fidelity)."""
    ctx = engine.Context(device)
    out = []
    for req in requests:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ham = engine.Hamiltonian(ctx, req.inst)
        K, shift = solve_plan(ctx, ham, req.T)
        N = 1 << req.n
        psi = torch.full((N,), 1.0 / math.sqrt(N), dtype=dtype, device="cuda")
        engine.evolve(ctx, ham, psi, 0.0, req.T, method="pc4", n_steps=K, shift=shift)
        mass, _ = engine.ground_mass(ctx, ham, req.T, psi)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0, mass, K))
        if progress:
            print(f"[serve] sequential {len(out)}/{len(requests)} (n={req.n}, {out[-1][0]:.2f} s)",
                  file=sys.stderr, flush=True)
        ham.free()
        del psi
    ctx.close()
    return out


def fifo_latencies(arrivals, services):
    """Latencies of a single server processing jobs in arrival order."""
    lat = []
    free_at = 0.0
    for a, s in zip(arrivals, services):
        start = max(a, free_at)
        free_at = start + s
        lat.append(free_at - a)
    return lat
