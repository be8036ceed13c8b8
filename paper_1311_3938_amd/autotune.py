"""Autotuner for the tile-pass plan of H|psi>.

For a Hamiltonian and a dtype it times H|psi> (aqc_apply, HIP events) under a
set of candidate tilings (aqc_ham_set_tiling): the last pass's tile bits, the
high-pass tile bits and contiguous low bits, register hypercube passes (wide,
narrow or none), and whether the last pass applies the remaining high flips
itself by reading their partners from memory (stream groups).  The fastest candidate is applied to the Hamiltonian and cached in a
JSON file keyed by the GPU architecture, the dtype, n and the flip-group
structure, so the search runs once per kind of problem.

For solves that run inside a batch the right measure is the batch's tick time,
not one solve's latency (a small solve alone cannot fill the GPU, so timing it
alone favours plans that are worse in a full batch): ``tune_batch`` times
ticks of a batch of replicas of the problem, enough to fill the device.
"""
from __future__ import annotations

import json
import os
import threading

import torch

from . import _lib as L
from . import engine

# options: register passes 3 wide, 2 narrow, 0 none (flips in tile passes);
# + 4: the remaining flips above the last tile as stream groups of the last
# pass (then the high-pass tile shape does not matter, so it is not varied)
def _candidates(tbfs, shapes):
    out = [(tbf, tbh, lh, reg) for tbf in tbfs for (tbh, lh) in shapes for reg in (3, 2, 0)]
    out += [(tbf, shapes[0][0], shapes[0][1], 4 | reg) for tbf in tbfs for reg in (3, 2, 0)]
    return out


CANDIDATES = {
    L.C64: _candidates((12, 13, 14), ((13, 4), (13, 5), (12, 4), (14, 6))),
    L.C128: _candidates((11, 12, 13), ((12, 3), (12, 4), (11, 3), (13, 5))),
}

BATCH_CANDIDATES = {
    L.C64: [(tbf, tbh, lh, reg) for tbf in (12, 13) for (tbh, lh) in ((13, 4), (13, 5), (13, 6), (12, 4))
            for reg in (3, 2, 0)] + [(tbf, 13, 4, 7) for tbf in (12, 13)],
    L.C128: [(tbf, tbh, lh, reg) for tbf in (11, 12) for (tbh, lh) in ((12, 3), (12, 4), (12, 5), (11, 3))
             for reg in (3, 2, 0)] + [(tbf, 12, 3, 7) for tbf in (11, 12)],
}

_lock = threading.Lock()


def default_tiling(dtype):
    """The library's default (tbf, tbh, lh, options) for a dtype."""
    return (13, 13, 4, 1) if dtype in (torch.complex64, L.C64) else (12, 12, 3, 1)


_memo = {}


def cache_path():
    base = os.environ.get("AQC_TUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "aqc", "tiling.json")


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def structure_key(inst, dtype_code):
    """n, dtype and the multiset of flip patterns' bit counts."""
    from collections import Counter
    flips = Counter(bin(int(x)).count("1") for x in inst.x if int(x) != 0)
    pats = len({int(x) for x in inst.x if int(x) != 0})
    return f"{_arch()}|{dtype_code}|n{inst.n}|groups{pats}|" + ",".join(
        f"{k}:{v}" for k, v in sorted(flips.items()))


def time_apply(ctx, ham, psi, out, reps=5):
    ws = engine.workspace(ctx, L.lib().aqc_apply_workspace_bytes(ham.handle, engine.dtype_code(psi)))
    engine.apply(ctx, ham, 0.37, psi, out, ws)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(ctx.stream)
    for _ in range(reps):
        engine.apply(ctx, ham, 0.37, psi, out, ws)
    e.record(ctx.stream)
    e.synchronize()
    return s.elapsed_time(e) / reps


def tune(ctx, ham, inst, dtype=torch.complex64, candidates=None, reps=5):
    """Time every candidate tiling; apply and return the best
    ((tbf, tbh, lh, reg), ms, {candidate: ms})."""
    dt = engine.dtype_code(torch.empty(0, dtype=dtype))
    cands = candidates if candidates is not None else CANDIDATES[dt]
    N = 1 << inst.n
    psi = torch.randn(N, dtype=dtype, device=ctx.device)
    out = torch.empty_like(psi)
    times = {}
    for c in cands:
        tbf, tbh, lh, reg = c
        try:
            ham.set_tiling(dtype, tbf, tbh, lh, reg)
        except L.AqcError:
            continue
        times[c] = time_apply(ctx, ham, psi, out, reps)
    best = min(times, key=times.get)
    ham.set_tiling(dtype, *best)
    return best, times[best], times


def time_batch(ctx, ham, dtype, copies, warm=16, ticks=32):
    """Seconds per tick of a batch of `copies` solves of this Hamiltonian."""
    import time
    b = engine.Batch(ctx, dtype, capacity=copies, graph=True)
    try:
        N = 1 << ham.n
        for _ in range(copies):
            psi = torch.randn(N, dtype=dtype, device=ctx.device)
            psi /= torch.linalg.vector_norm(psi)
            b.admit(ham, psi, 0.0, 1.0, 10 ** 6, 0.0)
        b.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(ticks)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / ticks
    finally:
        b.close()


def tune_batch(ctx, ham, inst, dtype=torch.complex64, candidates=None, fill_amps=1 << 23, max_copies=64):
    """Time batch ticks of replicas of the problem (about fill_amps amplitudes in
    all) under every candidate plan; apply and return the best
    ((tbf, tbh, lh, options), s per tick, {candidate: s})."""
    dt = engine.dtype_code(torch.empty(0, dtype=dtype))
    cands = candidates if candidates is not None else BATCH_CANDIDATES[dt]
    copies = max(1, min(max_copies, fill_amps >> inst.n))
    times = {}
    for c in cands:
        try:
            ham.set_tiling(dtype, *c)
        except L.AqcError:
            continue
        times[c] = time_batch(ctx, ham, dtype, copies)
    best = min(times, key=times.get)
    ham.set_tiling(dtype, *best)
    return best, times[best], times


def tune_cached(ctx, ham, inst, dtype=torch.complex64, path=None, batch=False):
    """Use the cached choice for this kind of problem, or tune and store it
    (batch=True: by batch tick time, cached under its own key)."""
    path = path or cache_path()
    dt = engine.dtype_code(torch.empty(0, dtype=dtype))
    key = ("batch|" if batch else "") + structure_key(inst, dt)
    with _lock:
        hit = _memo.get((path, key))
        if hit is not None:
            ham.set_tiling(dtype, *hit)
            return tuple(hit), None, False
        cache = {}
        if os.path.exists(path):
            try:
                cache = json.load(open(path))
            except ValueError:
                cache = {}
        if key in cache:
            c = cache[key]["tiling"]
            ham.set_tiling(dtype, *c)
            _memo[(path, key)] = list(c)
            return tuple(c), cache[key]["ms"], False
        if batch:
            best, s_tick, _ = tune_batch(ctx, ham, inst, dtype)
            ms = 1e3 * s_tick   # milliseconds per batch tick
        else:
            best, ms, _ = tune(ctx, ham, inst, dtype)
        cache[key] = {"tiling": list(best), "ms": ms}
        _memo[(path, key)] = list(best)
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
        return best, ms, True
