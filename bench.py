#!/usr/bin/env python3
"""Benchmark of the time-stepped Schroedinger evolution on one MI355X.

Workload: the Sherrington-Kirkpatrick annealing run with n = 30 qubits
(2^30 amplitudes, 8 GiB per complex64 vector): H(s) = (1 - s) H_x + s H_SK,
H_x = sum (1 - sigma^x)/2, H_SK = sum J_ij sz_i sz_j + sum h_i sz_i with
J_ij ~ N(0, 1/n), h_i ~ N(0, 0.1), s(t) = sin^2(pi t / 2T), T = 30, psi(0) = |+>^30.
The integrator is the one-evaluation 4th-order predictor-corrector (Sec. II.B of
the paper) with a centred spectral shift; the step h comes from the stability
guard h * rho <= 0.1.  Complex64 state, float32 products, float64 reductions.

One benchmark step = one aqc_evolve call over the next window of `--window`
integration steps of the path (RK4 bootstrap, predictor-corrector steps, norm
guard, shift phase) followed by the ground-state mass of the diagonal at T.
The metric is amplitude updates per second: 2^n x integration steps / seconds.
The workspace is picked among a few fresh allocations by a short timed window
(the last pass's speed depends on where the allocation lands in HBM).

Beside it, the same JSON line carries: complex64-vs-complex128 accuracy (the
whole path at n = 24, the first window at n = 30); a compact batched run and a
compact served run (continuous batching, Poisson arrivals) on the generators
of the batched and serving workloads, each against the plain single-instance
complex128 path on the same solves (solves/s, p50/p99 latency, |dF|); and the
oracle timed on the host on a whole 13-qubit solve, with the library's
complex64 and complex128 errors against it.

Prints one JSON line (rank 0, N = 1 only)."""
import argparse
import json
import math
import os
import sys
import time


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sk_plan(ham, T):
    """(steps, shift) of a full solve: centred shift, h rho = 0.1."""
    lo, hi = ham.spectral_bounds(0.0, T)
    return int(math.ceil(T * 0.5 * (hi - lo) / 0.1)), 0.5 * (lo + hi)


def cpu_baseline(ctx, n=13, T=30.0):
    """The oracle (NumPy complex128, one thread) on a whole solve of the same
    workload family at n = 13 (the full path from |+>, fixed-step pc4 with the
    library's step and shift), timed; the library solves the same problem in
    complex64 and complex128, and their errors against the oracle's state and
    ground-state mass at T are reported with it."""
    import numpy as np
    import torch
    from oracle import integrate, observables
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    inst = I.workload_sk_sin2(n=n, T=T, seed=I.seed_for(2))
    ham = engine.Hamiltonian(ctx, inst)
    K, shift = sk_plan(ham, T)
    psi0 = I.plus_state(n)
    t0 = time.perf_counter()
    ref = integrate.evolve(inst, psi0, 0.0, T, K, "pc4", shift)
    dt = time.perf_counter() - t0
    F_ref, _ = observables.ground_mass(inst, T, ref)
    err = {}
    for name, tdt in (("c64", torch.complex64), ("c128", torch.complex128)):
        psi = torch.from_numpy(psi0).to(device="cuda", dtype=tdt)
        engine.evolve(ctx, ham, psi, 0.0, T, method="pc4", n_steps=K, shift=shift)
        F, _ = engine.ground_mass(ctx, ham, T, psi)
        got = psi.cpu().to(torch.complex128).numpy()
        err[name] = {"dpsi": float(np.linalg.norm(got - ref)), "dF": abs(F - F_ref)}
    ham.free()
    return {"value": (1 << n) * K / dt, "unit": "amp-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one whole solve of the SK workload at n={n} (same generator, 2^{n} amplitudes, "
                      f"T={T:g}, {K} pc4 steps with the library's step and shift, 3 RK4 bootstrap "
                      f"steps included), {dt:.1f} s, NumPy complex128 single thread; n=30 does not fit "
                      "the oracle",
            "gpu_error_vs_oracle": {"n": n, "steps": K, "F_T_oracle": F_ref, **err}}


def kernel_source_hash():
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "paper_1311_3938_amd", "csrc", "aqc_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(args):
    """HBM bytes per last-pass launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), when
    it was taken on this kernel source and this configuration; else None."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "k_pass_last_sk30_c64_traffic.txt")
    if not os.path.exists(path):
        return None
    try:
        rec = json.loads(open(path).read().split("JSON:", 1)[1])
    except (ValueError, IndexError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    chained = args.method == "pc4" and not args.no_carry
    if (rec.get("n"), rec.get("window"), rec.get("dtype"), rec.get("method"), rec.get("chained")) != (
            args.n, args.window, args.dtype, args.method, chained):
        return None
    return rec.get("traffic_bytes_per_launch")


def error_summary(dFs, reqs, res):
    """Fidelity differences to the complex128 plain path: how many exceed 1e-6
    and the largest ones with their size and step count."""
    order = sorted(range(len(dFs)), key=lambda i: -dFs[i])
    return {"n": len(dFs), "above_1e-6": sum(d > 1e-6 for d in dFs),
            "max_steps": max(r.steps for r in res[:len(dFs)]),
            "worst": [{"rid": reqs[i].rid, "n": reqs[i].n, "steps": res[i].steps, "T": reqs[i].T,
                       "dF": dFs[i]} for i in order[:8]]}


def run_batch_mode(args):
    """Mixed batch of independent solves (EC3 and SK, n uniform in 14..22, XX
    catalysts, T uniform in 10..100) admitted together into one batch;
    complex64 state, float64 reductions, ticks launched as graphs."""
    import numpy as np
    import torch
    from paper_1311_3938_amd import engine, serve
    from paper_1311_3938_amd import instances as I
    insts = [I.workload_batch_member(i, n_lo=args.batch_n_lo, n_hi=args.batch_n_hi)
             for i in range(args.instances)]
    ctx = engine.Context(0)
    reqs = [serve.Request(i, inst) for i, inst in enumerate(insts)]
    srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=args.hbm_budget * 1e9,
                       size_classes=((34, args.instances),), ticks=args.ticks, graph=True,
                       autotune=not args.no_autotune, progress=8, resident_max_n=args.resident_max_n)
    log(f"batch: {len(reqs)} solves, n in [{min(r.n for r in reqs)}, {max(r.n for r in reqs)}], "
        f"resident up to n = {args.resident_max_n}")
    tune_s = 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        kinds = serve.warm_plans(reqs)
        tune_s = time.perf_counter() - t0
        log(f"autotuned {kinds} kinds of problem by batch tick time in {tune_s:.1f} s")
    t0 = time.perf_counter()
    res, wall = srv.run(reqs)
    amp_steps = sum((1 << r.n) * r.steps for r in res)
    srv.close()
    log(f"batch done in {wall:.1f} s")
    sub = reqs[:args.baseline_subset]
    # the same subset as a batch of its own, for a like-for-like rate
    srv_sub = serve.Server(dtype=torch.complex64, hbm_budget_bytes=args.hbm_budget * 1e9,
                           size_classes=((34, max(1, len(sub))),), ticks=args.ticks, graph=True,
                           autotune=not args.no_autotune, resident_max_n=args.resident_max_n)
    res_sub, wall_sub = srv_sub.run([serve.Request(q.rid, q.inst) for q in sub])
    srv_sub.close()
    log(f"the first {len(sub)} solves as a batch of their own: {wall_sub:.1f} s")
    log(f"sequential complex128 on {len(sub)} of the solves")
    seq = serve.sequential_plain(sub, progress=True)
    seq_time = sum(s[0] for s in seq) or float("nan")
    seq_lat = serve.fifo_latencies([0.0] * len(sub), [s_[0] for s_ in seq])
    dFs = [abs(seq[i][1] - res[i].fidelity) for i in range(len(sub))]
    dF = max(dFs) if dFs else None
    out = {
        "metric": "batched solves/s", "value": len(res) / wall, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"{len(res)} mixed EC3/SK solves, n {args.batch_n_lo}..{args.batch_n_hi}, "
                               "XX catalysts, T 10..100, pc4, batch ticks launched as graphs"
                               + (f", solves up to n = {args.resident_max_n} resident (one workgroup each, "
                                  "one launch)" if args.resident_max_n else ""),
                   "solves": len(res), "resident_max_n": args.resident_max_n},
        "amp_updates_per_s": amp_steps / wall,
        "autotune_s_before_timing": tune_s,
        "baseline_plain_c128_sequential": {
            "solves": len(sub), "seconds": seq_time, "solves_per_s": len(sub) / seq_time,
            "latency_s": {"p50": serve.percentile(seq_lat, 50), "p99": serve.percentile(seq_lat, 99)},
            "batched_solves_per_s_on_same": len(res_sub) / wall_sub,
            "batched_latency_s_on_same": {"p50": serve.percentile([r.latency for r in res_sub], 50),
                                          "p99": serve.percentile([r.latency for r in res_sub], 99)}},
        "max_abs_dF_vs_c128_plain": dF,
        "dF_vs_c128_plain": error_summary(dFs, sub, res) if dFs else None,
        "latency_s": {"p50": serve.percentile([r.latency for r in res], 50),
                      "p99": serve.percentile([r.latency for r in res], 99)},
    }
    print(json.dumps(out), flush=True)


def run_serve_mode(args):
    """Poisson-arriving requests, n in [12, n_max] with P(n) ~ 2^-(n-12)/2,
    EC3 or SK, linear or catalysed path, T uniform in 10..100; admitted by HBM
    budget, states resident, continuous batching in two size classes."""
    import numpy as np
    import torch
    from paper_1311_3938_amd import engine, serve
    from paper_1311_3938_amd import instances as I
    arr = serve.poisson_arrivals(args.requests, args.qps)
    reqs = [serve.Request(i, I.workload_serving_request(i, n_hi=args.n_max), float(arr[i]))
            for i in range(args.requests)]
    srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=args.hbm_budget * 1e9,
                       size_classes=((20, 256), (34, 8)), ticks=args.ticks, graph=True,
                       autotune=not args.no_autotune, progress=8)
    log(f"serve: {len(reqs)} requests at {args.qps} qps, n in "
        f"[{min(r.n for r in reqs)}, {max(r.n for r in reqs)}]")
    tune_s = 0.0
    if not args.no_autotune:
        t0 = time.perf_counter()
        kinds = serve.warm_plans(reqs)
        tune_s = time.perf_counter() - t0
        log(f"autotuned {kinds} kinds of problem by batch tick time in {tune_s:.1f} s")
    res, wall = srv.run(reqs)
    srv.close()
    lat = [r.latency for r in res]
    log(f"served in {wall:.1f} s")
    log("sequential complex128 on the same requests")
    seq = serve.sequential_plain(reqs, progress=True)
    seq_lat = serve.fifo_latencies([r.arrival for r in reqs], [s[0] for s in seq])
    dFs = [abs(seq[i][1] - res[i].fidelity) for i in range(len(reqs))]
    dF = max(dFs)
    out = {
        "metric": "served solves/s", "value": len(res) / wall, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"{len(res)} Poisson requests at {args.qps} qps, n 12..{args.n_max}, "
                               "EC3/SK, linear or catalysed, T 10..100; continuous batching",
                   "requests": len(res), "qps": args.qps},
        "latency_s": {"p50": serve.percentile(lat, 50), "p99": serve.percentile(lat, 99)},
        "autotune_s_before_timing": tune_s,
        "baseline_plain_c128_sequential": {
            "solves_per_s": len(reqs) / sum(s[0] for s in seq),
            "latency_s": {"p50": serve.percentile(seq_lat, 50), "p99": serve.percentile(seq_lat, 99)}},
        "max_abs_dF_vs_c128_plain": dF,
        "dF_vs_c128_plain": error_summary(dFs, reqs, res),
    }
    print(json.dumps(out), flush=True)


def run_adaptive_mode(args):
    """The 24-qubit EC3 run with an XX catalyst: complex128 chooses the grid with
    the adaptive predictor-corrector, complex64 (float64 reductions) replays it;
    the path is done in ten pieces so progress is visible."""
    import torch
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    inst = I.workload_ec3_catalyst()
    T = inst.path["T"]
    ctx = engine.Context(0)
    ham = engine.Hamiltonian(ctx, inst)
    # the plan of each dtype chosen by timing H|psi> under the autotuner's
    # candidate tilings, before the timed region
    plans, tune_s = {}, 0.0
    if not args.no_autotune:
        from paper_1311_3938_amd import autotune
        t_tune = time.perf_counter()
        for name, dt in (("c64", torch.complex64), ("c128", torch.complex128)):
            plans[name] = list(autotune.tune(ctx, ham, inst, dt)[0])
        tune_s = time.perf_counter() - t_tune
        log(f"tuned plans {plans} in {tune_s:.1f} s")
    lo, hi = ham.spectral_bounds(0.0, T)
    shift = 0.5 * (lo + hi)
    N = 1 << inst.n
    p128 = torch.full((N,), N ** -0.5, dtype=torch.complex128, device="cuda")
    p64 = torch.full((N,), N ** -0.5, dtype=torch.complex64, device="cuda")
    out = {"c64": {"seconds": 0.0, "steps": 0}, "c128": {"seconds": 0.0, "steps": 0, "rejected": 0}}
    h0 = 0.01
    pieces = 10
    for i in range(pieces):
        ta, tb = T * i / pieces, T * (i + 1) / pieces
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, segs = engine.evolve(ctx, ham, p128, ta, tb, method="pc4", n_steps=0, atol=args.atol,
                                 h0=h0, window=8, shift=shift, stab_limit=0.2155,
                                 check_every=256, norm_tol=1e-2, record_cap=1 << 16)
        torch.cuda.synchronize()
        out["c128"]["seconds"] += time.perf_counter() - t0
        out["c128"]["steps"] += st["steps"]
        out["c128"]["rejected"] += st["rejected"]
        h0 = st["h_last"]
        t0 = time.perf_counter()
        st64, _ = engine.evolve(ctx, ham, p64, ta, tb, method="pc4", replay=segs, shift=shift,
                                check_every=256, norm_tol=1e-2)
        torch.cuda.synchronize()
        out["c64"]["seconds"] += time.perf_counter() - t0
        out["c64"]["steps"] += st64["steps"]
        log(f"piece {i}: t=[{ta:g},{tb:g}] c128 steps {st['steps']} (rejected {st['rejected']}), "
            f"h_last {st['h_last']:.4g}")
    for name, p in (("c64", p64), ("c128", p128)):
        mass, emin = engine.ground_mass(ctx, ham, T, p)
        out[name]["fidelity"] = mass
        out[name]["amp_updates_per_s"] = N * out[name]["steps"] / out[name]["seconds"]
    dpsi = torch.linalg.vector_norm(p64.to(torch.complex128) - p128).item()
    res = {
        "metric": "amp-updates/s", "value": out["c64"]["amp_updates_per_s"], "unit": "amp-updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": out["c64"]["seconds"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "EC3 n=24, 20 clauses, 24 XX catalyst pairs, T=50, adaptive pc4 "
                               f"(atol {args.atol:g}) in complex128, grid replayed in complex64"},
        "c64": out["c64"], "c128": out["c128"],
        "plans": plans or "library default", "autotune_s_before_timing": tune_s,
        "abs_dF_c64_vs_c128": abs(out["c64"]["fidelity"] - out["c128"]["fidelity"]),
        "dpsi_c64_vs_c128": dpsi,
    }
    print(json.dumps(res), flush=True)


def run_paths_mode(args):
    """The three paths of Sec. IV.A (straight line, nonlinear, clause-by-clause)
    from H^xy to an EC3 H_f at n qubits, started in a Dicke state: fixed-step
    pc4 windows per path, with the kernel times of each."""
    import numpy as np
    import torch
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    n = args.n_paths
    m = int(round(0.8 * n))
    T = 20.0
    N = 1 << n
    W = args.window
    weight = n // 3
    dicke = torch.from_numpy(I.dicke_state(n, weight, dtype=np.complex64)).to("cuda")
    ctx = engine.Context(0)
    out = {}
    for kind in args.paths_kinds.split(","):
        inst = I.workload_ec3_paths(n=n, m=m, T=T, kind=kind, seed=I.seed_for(5))
        ham = engine.Hamiltonian(ctx, inst)
        tuned = None
        if args.paths_autotune:
            from paper_1311_3938_amd import autotune
            t_tune = time.perf_counter()
            tuned = list(autotune.tune(ctx, ham, inst, torch.complex64)[0])
            log(f"{kind}: tuned plan {tuned} in {time.perf_counter() - t_tune:.1f} s")
        lo, hi = ham.spectral_bounds(0.0, T)
        rho = 0.5 * (hi - lo)
        K = int(math.ceil(T * rho / 0.1))
        h = T / K
        psi = dicke.clone()
        opts = dict(method="pc4", n_steps=W, shift=0.5 * (lo + hi), check_every=W, norm_tol=1e-2,
                    stab_limit=0.2155)
        o, _, _ = engine.evolve_opts(**opts)
        ws = engine.workspace(ctx, engine.evolve_workspace_bytes(ham, engine.dtype_code(psi), o))
        carry = engine.new_carry()
        # the middle of the path, where every clause ramp of the cbc path is on
        t_a = 0.5 * T - 0.5 * (args.steps + args.warmup) * W * h
        for i in range(args.warmup):
            engine.evolve(ctx, ham, psi, t_a, t_a + W * h, ws=ws, carry=carry, **opts)
            t_a += W * h
        engine.profile_enable(ctx, True)
        engine.profile_reset(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        for i in range(args.steps):
            st, _ = engine.evolve(ctx, ham, psi, t_a, t_a + W * h, ws=ws, carry=carry, **opts)
            t_a += W * h
            steps += st["steps"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = engine.profile_read(ctx)
        engine.profile_enable(ctx, False)
        last_ms, last_n, last_b = prof["last_pass"]
        high_ms, high_n, high_b = prof["high_pass"]
        info = ham.info()
        out[kind] = {
            "amp_updates_per_s": N * steps / el, "ms_per_integration_step": 1e3 * el / steps,
            "K_path": K, "h": h, "n_terms": inst.n_terms, "n_schedules": len(inst.scheds),
            "tile_passes_per_matvec": info["n_passes"][0],
            "last_pass": {"avg_ms": last_ms / max(last_n, 1),
                          "GBps": last_b / (last_ms * 1e-3) / 1e9 if last_ms > 0 else None},
            "high_passes": {"launches_per_step": high_n / max(steps, 1),
                            "avg_ms": high_ms / max(high_n, 1),
                            "GBps": high_b / (high_ms * 1e-3) / 1e9 if high_ms > 0 else None},
            "bytes_per_amp_step": (last_b + high_b) / max(steps, 1) / N,
            "hbm_frac_whole_step": (last_b + high_b) / el / 8.0e12,
            "norm": engine.norm2(ctx, psi),
            "plan": tuned if tuned is not None else "default",
        }
        log(f"{kind}: {out[kind]}")
        del ws, psi
        ham.free()
        torch.cuda.empty_cache()
    lin = out[next(iter(out))]
    res = {
        "metric": "amp-updates/s", "value": lin["amp_updates_per_s"], "unit": "amp-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": lin["ms_per_integration_step"] * W, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"EC3 n={n}, m={m}, H^xy start (Dicke weight {weight}), T={T:g}, "
                               f"pc4 windows of {W} steps in the middle of each path"},
        "paths": out,
    }
    print(json.dumps(res), flush=True)


def run_sector_mode(args):
    """The paths of Sec. IV.A in one Hamming-weight sector (Sec. III.A.2-3):
    EC3 with m = round(0.8 n) clauses from H^xy, the C(n, w) states of weight
    w only, from their Dicke state; chained pc4 windows in the middle of each
    path, timed with the library's kernel timers."""
    import torch
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    n = args.n_sector
    w = args.w_sector if args.w_sector >= 0 else n // 2
    m = int(round(0.8 * n))
    T = 20.0
    W = args.window
    ctx = engine.Context(0)
    tdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    out = {}
    for kind in args.sector_paths.split(","):
        inst = I.workload_ec3_paths(n=n, m=m, T=T, kind=kind, seed=I.seed_for(5))
        ham = engine.Hamiltonian(ctx, inst)
        sec = engine.Sector(ctx, ham, w)
        D = sec.dim
        t_b = time.perf_counter()
        lo, hi = sec.spectral_bounds(0.0, T)
        bounds_s = time.perf_counter() - t_b
        rho = 0.5 * (hi - lo)
        K = int(math.ceil(T * rho / 0.1))
        h = T / K
        log(f"{kind}: n={n} w={w} dim={D} enclosure=[{lo:.3f},{hi:.3f}] ({bounds_s:.2f} s) K={K}")
        psi = sec.dicke(tdt)
        opts = dict(method="pc4", n_steps=W, shift=0.5 * (lo + hi), check_every=W, norm_tol=1e-2,
                    stab_limit=0.2155)
        o, _, _ = engine.evolve_opts(**opts)
        ws = engine.workspace(ctx, engine.evolve_workspace_bytes(sec, engine.dtype_code(psi), o))
        carry = engine.new_carry()
        t_a = 0.5 * T - 0.5 * (args.steps + args.warmup) * W * h
        for i in range(args.warmup):
            engine.evolve(ctx, sec, psi, t_a, t_a + W * h, ws=ws, carry=carry, **opts)
            t_a += W * h
            log(f"{kind}: warmup window {i} done")
        engine.profile_enable(ctx, True)
        engine.profile_reset(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        for i in range(args.steps):
            st, _ = engine.evolve(ctx, sec, psi, t_a, t_a + W * h, ws=ws, carry=carry, **opts)
            t_a += W * h
            steps += st["steps"]
            log(f"{kind}: window {i} done")
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = engine.profile_read(ctx)
        engine.profile_enable(ctx, False)
        k_ms, k_n, k_b = prof["last_pass"]
        out[kind] = {
            "dim": D, "full_space_amplitudes": 1 << n,
            "sector_amp_updates_per_s": D * steps / el,
            "ms_per_integration_step": 1e3 * el / steps,
            "K_path": K, "h": h, "enclosure": [lo, hi], "enclosure_seconds": bounds_s,
            "kernel": {"avg_ms": k_ms / max(k_n, 1),
                       "algorithmic_GBps": k_b / (k_ms * 1e-3) / 1e9 if k_ms > 0 else None,
                       "bytes_per_amp": k_b / max(k_n, 1) / D},
            "norm2": engine.norm2(ctx, psi),
            "workspace_GiB": ws.numel() / 2 ** 30,
        }
        log(f"{kind}: {out[kind]}")
        del ws, psi
        sec.free()
        ham.free()
        torch.cuda.empty_cache()
    first = out[next(iter(out))]
    res = {
        "metric": "amp-updates/s", "value": first["sector_amp_updates_per_s"], "unit": "amp-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": first["ms_per_integration_step"] * W, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"EC3 n={n}, m={m}, H^xy start, Hamming-weight sector w={w} "
                               f"(C({n},{w}) amplitudes), T={T:g}, pc4 windows of {W} steps"},
        "sector": out,
    }
    print(json.dumps(res), flush=True)


def run_gap_mode(args):
    """Gap curve E_1(s) - E_0(s) of a path of Sec. IV.A (the analysis behind
    the paper's bottom panels): the two lowest levels by aqc_lowest_eigs at
    evenly spaced s, in the Hamming-weight sector of the Dicke start (or the
    full space with --w-sector -2)."""
    import numpy as np
    import torch
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    n = args.n_gap
    m = int(round(0.8 * n))
    w = args.w_sector if args.w_sector >= 0 else n // 3
    ctx = engine.Context(0)
    inst = I.workload_ec3_paths(n=n, m=m, T=1.0, kind=args.gap_path, seed=I.seed_for(5))
    ham = engine.Hamiltonian(ctx, inst)
    op = ham if args.w_sector == -2 else engine.Sector(ctx, ham, w)
    dtype = torch.complex128 if args.dtype == "c128" else torch.complex64
    tol = 1e-10 if args.dtype == "c128" else 1e-5
    pts = []
    ws = None
    t_all = time.perf_counter()
    for i in range(args.gap_points):
        s_ = (i + 0.5) / args.gap_points
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, res, nmv = engine.lowest_eigs(ctx, op, s_, k=2, dtype=dtype, tol=tol, max_basis=24,
                                          max_matvecs=20000)
        el = time.perf_counter() - t0
        pts.append({"s": s_, "E0": ev[0], "E1": ev[1], "gap": ev[1] - ev[0], "matvecs": nmv,
                    "seconds": el, "resid": res.tolist()})
        log(f"s={s_:.3f}: E0={ev[0]:.6f} gap={ev[1] - ev[0]:.6f} ({nmv} products, {el:.2f} s)")
    wall = time.perf_counter() - t_all
    dim = op.dim
    mv = sum(p["matvecs"] for p in pts)
    gmin = min(pts, key=lambda p: p["gap"])
    res_ = {
        "metric": "gap points/s", "value": len(pts) / wall, "unit": "points/s", "n_gpus": 1,
        "steps": len(pts), "warmup": 0, "ms_per_step": 1e3 * wall / len(pts), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"EC3 n={n}, m={m}, {args.gap_path} path from H^xy, "
                               + (f"sector w={w} ({dim} states)" if op is not ham else f"full space ({dim})")
                               + f", {len(pts)} values of s"},
        "products": mv, "products_per_s": mv / wall, "amp_products_per_s": mv * dim / wall,
        "min_gap": {"s": gmin["s"], "gap": gmin["gap"]}, "points": pts,
    }
    print(json.dumps(res_), flush=True)


def run_tsearch_mode(args):
    """Successful runtimes T_s (E(T_s) = 1/2, Sec. III.B) of hard instances
    with a unique solution (Sec. II.D) for the X and XY algorithms, each round
    of the bracket-and-bisect search solved as one batch (the methodology of
    the paper's runtime-scaling figure, on synthetic instances)."""
    import numpy as np
    import torch
    from paper_1311_3938_amd import engine, tsearch
    from paper_1311_3938_amd import instances as I
    ctx = engine.Context(0)
    sizes = [int(v) for v in args.ts_sizes.split(",")]
    out = {}
    t_all = time.perf_counter()
    n_solves = 0
    for alg in args.ts_algorithms.split(","):
        for n in sizes:
            insts = [I.workload_usa(n, i, alg) for i in range(args.ts_instances)]
            states = []
            for inst in insts:
                if alg == "x":
                    states.append(I.plus_state(n))
                    continue
                ham = engine.Hamiltonian(ctx, inst)
                sec = engine.Sector(ctx, ham, inst.meta["weight"])
                g = torch.empty(sec.dim, dtype=torch.complex128, device="cuda")
                engine.lowest_eigs(ctx, sec, 0.0, k=1, max_basis=16, tol=1e-10, ground=g)
                states.append(sec.expand(g))
                sec.free()
                ham.free()
            t0 = time.perf_counter()
            S = tsearch.find_ts(ctx, insts, states, T0=4.0, rel=args.ts_rel, dtype=torch.complex64,
                                log=log, batched=args.ts_batched)
            el = time.perf_counter() - t0
            ts = [s.T_s for s in S]
            ns = sum(len(s.evals) for s in S)
            n_solves += ns
            out[f"{alg}-{n}"] = {"T_s_median": float(np.nanmedian(ts)),
                                 "T_s_quartiles": [float(np.nanpercentile(ts, 25)),
                                                   float(np.nanpercentile(ts, 75))],
                                 "T_s": ts, "solves": ns, "seconds": el,
                                 "m": [len(i.meta["clauses"]) for i in insts]}
            log(f"{alg} n={n}: median T_s {out[f'{alg}-{n}']['T_s_median']:.3g}, {ns} solves in {el:.1f} s")
    wall = time.perf_counter() - t_all
    res = {
        "metric": "solves/s", "value": n_solves / wall, "unit": "solves/s", "n_gpus": 1, "steps": n_solves,
        "warmup": 0, "ms_per_step": 1e3 * wall / max(n_solves, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"T_s search, hard EC3 instances with a unique solution, n in {sizes}, "
                               f"{args.ts_instances} per size, algorithms {args.ts_algorithms}, "
                               f"bracket ratio {1 + args.ts_rel:g}, "
                               + ("batched rounds" if args.ts_batched else "sequential solves")},
        "runs": out,
    }
    print(json.dumps(res), flush=True)


def run_scaling_mode(args):
    """Step time against n for the SK workload family (sin^2 path, transverse
    field, pc4, c64 with float64 reductions): the library (median of 5
    windows of 50 chained steps) beside the oracle (NumPy complex128, one
    thread), with the versions of the software stack."""
    import numpy as np
    import torch
    from oracle import integrate, sqh
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    ctx = engine.Context(0)
    rows = []
    for n in [int(v) for v in args.scaling_sizes.split(",")]:
        inst = I.workload_sk_sin2(n=n, T=30.0, seed=I.seed_for(2))
        ham = engine.Hamiltonian(ctx, inst)
        lo, hi = ham.spectral_bounds(0.0, 30.0)
        K = int(math.ceil(30.0 * 0.5 * (hi - lo) / 0.1))
        h = 30.0 / K
        N = 1 << n
        psi = torch.full((N,), N ** -0.5, dtype=torch.complex64, device="cuda")
        opts = dict(method="pc4", n_steps=50, shift=0.5 * (lo + hi))
        o, _, _ = engine.evolve_opts(**opts)
        ws = engine.workspace(ctx, engine.evolve_workspace_bytes(ham, engine.dtype_code(psi), o))
        carry = engine.new_carry()
        t = 0.0
        engine.evolve(ctx, ham, psi, t, t + 50 * h, ws=ws, carry=carry, **opts)
        t += 50 * h
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            engine.evolve(ctx, ham, psi, t, t + 50 * h, ws=ws, carry=carry, **opts)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) / 50)
            t += 50 * h
        gpu = float(np.median(times))
        row = {"n": n, "gpu_ms_per_step": 1e3 * gpu, "gpu_amp_updates_per_s": N / gpu}
        del ws, psi
        ham.free()
        torch.cuda.empty_cache()
        if n <= args.scaling_oracle_max:
            psi0 = I.plus_state(n)
            steps = 4 if n <= 16 else 1
            seg = integrate.Segment(inst, psi0, 0.0, h, "pc4", 0.5 * (lo + hi))
            seg.advance(3)                     # the RK4 bootstrap
            t0 = time.perf_counter()
            seg.advance(steps)
            o_dt = (time.perf_counter() - t0) / steps
            row.update({"oracle_ms_per_step": 1e3 * o_dt, "oracle_amp_updates_per_s": N / o_dt,
                        "ratio": o_dt / gpu})
        rows.append(row)
        log(f"n={n}: {row}")
    fit = [r for r in rows if "oracle_ms_per_step" in r]
    per_amp = fit[-1]["oracle_ms_per_step"] / (1 << fit[-1]["n"]) if fit else None
    versions = {"torch": torch.__version__, "hip": getattr(torch.version, "hip", None),
                "device": torch.cuda.get_device_properties(0).name,
                "arch": torch.cuda.get_device_properties(0).gcnArchName}
    res = {
        "metric": "amp-updates/s", "value": rows[-1]["gpu_amp_updates_per_s"], "unit": "amp-updates/s",
        "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": rows[-1]["gpu_ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "SK + transverse field, sin^2 path, T=30, pc4, chained windows of 50 steps"},
        "rows": rows, "versions": versions,
        "oracle_n30_extrapolated_s_per_step": per_amp * (1 << 30) * 1e-3 if per_amp else None,
    }
    print(json.dumps(res), flush=True)


def calibrated_workspace(ctx, ham, psi, nbytes, opts, h, trials):
    """The workspace of the timed run.  On MI355X the speed of the last pass
    (eleven concurrent streams) depends on where in HBM the allocation lands:
    a fresh allocation runs it in one of two modes about 7 % apart, while each
    vector alone streams at the same rate in both (measured; address
    translation misses are equal in both modes).  Like a long-running service
    that allocates once, the benchmark tries a few allocations, times a short
    chained window on each, and keeps the fastest.  Returns (workspace, the
    last-pass ms of every trial)."""
    import torch
    from paper_1311_3938_amd import engine
    N = psi.numel()
    Wc = 16
    copts = dict(opts, n_steps=Wc)
    best, best_ms, tried = None, math.inf, []
    for _ in range(max(1, trials)):
        ws = engine.workspace(ctx, nbytes)
        carry = engine.new_carry()
        psi.fill_(1.0 / math.sqrt(N))
        engine.evolve(ctx, ham, psi, 0.0, Wc * h, ws=ws, carry=carry, **copts)
        engine.profile_enable(ctx, True)
        engine.profile_reset(ctx)
        engine.evolve(ctx, ham, psi, Wc * h, 2 * Wc * h, ws=ws, carry=carry, **copts)
        ms, nl, _ = engine.profile_read(ctx)["last_pass"]
        engine.profile_enable(ctx, False)
        ms /= max(nl, 1)
        tried.append(round(ms, 3))
        if ms < best_ms:
            if best is not None:
                del best
                torch.cuda.empty_cache()
            best, best_ms = ws, ms
        else:
            del ws
            torch.cuda.empty_cache()
    psi.fill_(1.0 / math.sqrt(N))
    return best, tried


def accuracy_checks(ctx, inst30, W, h, opts):
    """Complex64 (float64 reductions) against complex128 on the GPU:
    * the whole path of the same workload at n = 24 (T = 30, fixed pc4 steps
      from the step guard): |dF| of the ground-state mass at T and ||dpsi||
      at T, where F is not small;
    * the first window of the 30-qubit run: ||dpsi|| (F is ~1e-9 there, so no
      fidelity figure is taken from it).
    The errors against the oracle itself come with the CPU baseline (n = 13)."""
    import torch
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I
    out = {}
    n, T = 24, 30.0
    inst = I.workload_sk_sin2(n=n, T=T, seed=I.seed_for(2))
    ham = engine.Hamiltonian(ctx, inst)
    K, shift = sk_plan(ham, T)
    res = {}
    for name, tdt in (("c64", torch.complex64), ("c128", torch.complex128)):
        psi = torch.full((1 << n,), 1.0 / math.sqrt(1 << n), dtype=tdt, device="cuda")
        engine.evolve(ctx, ham, psi, 0.0, T, method="pc4", n_steps=K, shift=shift)
        F, _ = engine.ground_mass(ctx, ham, T, psi)
        res[name] = (psi.to(torch.complex128), F)
    d = res["c64"][0] - res["c128"][0]
    out["full_path_n24"] = {"steps": K, "T": T, "reference": "GPU complex128, same steps and shift",
                            "F_T_c128": res["c128"][1], "dF": abs(res["c64"][1] - res["c128"][1]),
                            "dpsi": float(torch.linalg.vector_norm(d).item())}
    del res, d
    ham.free()
    torch.cuda.empty_cache()
    ham30 = engine.Hamiltonian(ctx, inst30)
    N = 1 << inst30.n
    p64 = torch.full((N,), 1.0 / math.sqrt(N), dtype=torch.complex64, device="cuda")
    engine.evolve(ctx, ham30, p64, 0.0, W * h, **opts)
    p128 = torch.full((N,), 1.0 / math.sqrt(N), dtype=torch.complex128, device="cuda")
    engine.evolve(ctx, ham30, p128, 0.0, W * h, **opts)
    p64c = p64.to(torch.complex128)
    del p64
    a2, b2 = engine.norm2(ctx, p64c), engine.norm2(ctx, p128)
    ov = engine.overlap(ctx, p64c, p128)
    out["first_window_n30"] = {"t": [0.0, W * h], "steps": W, "reference": "GPU complex128",
                               "dpsi": math.sqrt(max(a2 + b2 - 2.0 * ov.real, 0.0))}
    del p64c, p128
    ham30.free()
    torch.cuda.empty_cache()
    return out


def compact_batch_and_serve(args):
    """The batched and served forms on the configs' generators, small enough
    for the default run: a batch of mixed EC3/SK solves (n 14..22, XX
    catalysts, T 10..100) admitted at once, and Poisson requests (n 12..28
    weighted toward small n, linear or catalysed, T 10..100) at a fixed QPS;
    complex64 with float64 reductions, continuous batching.  The same solves
    are then run one after the other on the plain single-instance complex128
    path, which gives the baseline rate, its (first-in-first-out) latencies and
    the reference for |dF|."""
    import torch
    from paper_1311_3938_amd import serve
    from paper_1311_3938_amd import instances as I
    out = {}
    # batch
    reqs = [serve.Request(i, I.workload_batch_member(i)) for i in range(args.leg_batch)]
    srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=args.hbm_budget * 1e9,
                       size_classes=((34, max(1, len(reqs))),), ticks=args.ticks, graph=True)
    res, wall = srv.run(reqs)
    srv.close()
    log(f"batch leg: {len(res)} solves in {wall:.1f} s")
    seq = serve.sequential_plain(reqs)
    seq_t = sum(s_[0] for s_ in seq)
    dFs = [abs(seq[i][1] - res[i].fidelity) for i in range(len(reqs))]
    out["batch"] = {
        "workload": f"{len(reqs)} mixed EC3/SK solves (the 512-solve generator's first members), "
                    "n 14..22, XX catalysts, T 10..100, admitted at once, ticks as graphs",
        "n_range": [min(r.n for r in reqs), max(r.n for r in reqs)],
        "solves_per_s": len(res) / wall, "seconds": wall,
        "latency_s": {"p50": serve.percentile([r.latency for r in res], 50),
                      "p99": serve.percentile([r.latency for r in res], 99)},
        "baseline_plain_c128_sequential": {
            "solves": len(reqs), "seconds": seq_t, "solves_per_s": len(reqs) / seq_t,
            "latency_s": {"p50": serve.percentile(serve.fifo_latencies([0.0] * len(reqs),
                                                                        [s_[0] for s_ in seq]), 50),
                          "p99": serve.percentile(serve.fifo_latencies([0.0] * len(reqs),
                                                                        [s_[0] for s_ in seq]), 99)}},
        "max_abs_dF_vs_c128_plain": max(dFs), "above_1e-6": sum(d_ > 1e-6 for d_ in dFs)}
    log(f"batch leg baseline: {seq_t:.1f} s")
    # serve
    arr = serve.poisson_arrivals(args.leg_serve, args.leg_qps)
    reqs = [serve.Request(i, I.workload_serving_request(i), float(arr[i])) for i in range(args.leg_serve)]
    srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=args.hbm_budget * 1e9,
                       size_classes=((20, 256), (34, 8)), ticks=args.ticks, graph=True)
    res, wall = srv.run(reqs)
    srv.close()
    log(f"serve leg: {len(res)} requests in {wall:.1f} s")
    seq = serve.sequential_plain(reqs)
    seq_lat = serve.fifo_latencies([r.arrival for r in reqs], [s_[0] for s_ in seq])
    dFs = [abs(seq[i][1] - res[i].fidelity) for i in range(len(reqs))]
    lat = [r.latency for r in res]
    out["serve"] = {
        "workload": f"{len(reqs)} Poisson requests at {args.leg_qps:g} qps (the serving generator's first "
                    "requests), n 12..28 with P(n) ~ 2^-(n-12)/2, EC3/SK, linear or catalysed, T 10..100; "
                    "two size classes, admission by HBM budget",
        "n_range": [min(r.n for r in reqs), max(r.n for r in reqs)],
        "solves_per_s": len(res) / wall, "seconds": wall,
        "latency_s": {"p50": serve.percentile(lat, 50), "p99": serve.percentile(lat, 99)},
        "baseline_plain_c128_sequential": {
            "solves_per_s": len(reqs) / sum(s_[0] for s_ in seq),
            "latency_s": {"p50": serve.percentile(seq_lat, 50), "p99": serve.percentile(seq_lat, 99)}},
        "max_abs_dF_vs_c128_plain": max(dFs), "above_1e-6": sum(d_ > 1e-6 for d_ in dFs)}
    log(f"serve leg baseline done")
    return out


def run_single_mode(args):
    import torch
    from paper_1311_3938_amd import engine
    from paper_1311_3938_amd import instances as I

    n = args.n
    N = 1 << n
    T = 30.0
    tdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    inst = I.workload_sk_sin2(n=n, T=T, seed=I.seed_for(2))
    ctx = engine.Context(0)
    ham = engine.Hamiltonian(ctx, inst)
    lo, hi = ham.spectral_bounds(0.0, T)
    rho = 0.5 * (hi - lo)
    k_total = int(math.ceil(T * rho / 0.1))
    h = T / k_total
    W = args.window
    log(f"n={n} dtype={args.dtype} method={args.method} enclosure=[{lo:.3f},{hi:.3f}] "
        f"rho={rho:.3f} K_total={k_total} h={h:.6g} window={W}")

    psi = torch.full((N,), 1.0 / math.sqrt(N), dtype=tdt, device="cuda")
    # one shift for the whole path: the centre of its spectral enclosure
    opts = dict(method=args.method, n_steps=W, shift=0.5 * (lo + hi), check_every=W,
                norm_tol=1e-2, stab_limit=0.2155)
    o, _, _ = engine.evolve_opts(**opts)
    nbytes = engine.evolve_workspace_bytes(ham, engine.dtype_code(psi), o)
    ws, placement = calibrated_workspace(ctx, ham, psi, nbytes, opts, h, args.placement_trials)
    log(f"workspace placement: last-pass ms of the trials {placement}")

    n_windows_total = k_total // W
    # consecutive windows form one chain of pc4 calls (the multistep history
    # carries over); the chain restarts from |+> when the path is done
    carry = engine.new_carry() if (args.method == "pc4" and not args.no_carry) else None

    def bench_step(i):
        w = i % n_windows_total
        if w == 0 and i > 0:
            psi.fill_(1.0 / math.sqrt(N))
            if carry is not None:
                carry.valid = 0
        t_a, t_b = w * W * h, (w + 1) * W * h
        st, _ = engine.evolve(ctx, ham, psi, t_a, t_b, ws=ws, carry=carry, **opts)
        mass, emin = engine.ground_mass(ctx, ham, T, psi)   # |psi|^2: the frame phase does not matter
        return st, mass, t_b

    for i in range(args.warmup):
        bench_step(i)
        log(f"warmup step {i} done")
    info = ham.info()
    log(f"plan: {info}; workspace {ws.numel() / 2**30:.1f} GiB")
    engine.profile_enable(ctx, True)
    engine.profile_reset(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(bench_step(args.warmup + i))
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = engine.profile_read(ctx)
    engine.profile_enable(ctx, False)
    int_steps = sum(s_[0]["steps"] for s_ in stats)
    value = N * int_steps / elapsed
    last_ms, last_n, last_bytes = prof["last_pass"]
    high_ms, high_n, high_bytes = prof["high_pass"]
    peak = 8.0e12
    achieved = last_bytes / (last_ms * 1e-3) if last_ms > 0 else 0.0
    result = {
        "metric": "amp-updates/s",
        "value": value,
        "unit": "amp-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"SK spin glass n={n} (2^{n} amplitudes), transverse-field start, "
                        f"sin^2 path, T={T:g}; {args.method} with centred shift, "
                        f"{args.dtype} state, fp64 reductions",
            "n_qubits": n, "integration_steps_per_step": W, "h": h, "k_total": k_total,
            "windows_chained": carry is not None,
            "tile_passes_per_matvec": info["n_passes"][0 if args.dtype == "c64" else 1],
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved / 1e9,
            "peak": peak / 1e9,
            "unit": "GB/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(args),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": "k_pass<last> (diagonal + low flips + fused stage update)",
            "avg_launch_ms": last_ms / max(last_n, 1),
            "algorithmic_bytes_per_launch": last_bytes / max(last_n, 1),
        },
        "high_pass": {
            "launches": high_n, "avg_launch_ms": high_ms / max(high_n, 1),
            "achieved_GBps": (high_bytes / (high_ms * 1e-3) / 1e9) if high_ms > 0 else None,
        },
        "effective_frac": None,
        "workspace_placement_trials_ms": placement,
        "ground_mass_end_of_last_window": {"t": stats[-1][2], "value": stats[-1][1]},
    }
    # whole-step traffic at the algorithmic minimum of this plan vs peak
    step_bytes = (last_bytes + high_bytes) / max(int_steps, 1)
    result["effective_frac"] = (step_bytes * int_steps / elapsed) / peak
    result["bytes_per_amp_step"] = step_bytes / N

    del ws
    torch.cuda.empty_cache()
    if args.copy_calib:
        a = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        result["copy_calib_bytes"] = {"read": a.numel() * 8, "write": a.numel() * 8}
        del a, b
    del psi
    torch.cuda.empty_cache()
    if not args.no_accuracy and args.dtype == "c64":
        result["accuracy"] = accuracy_checks(ctx, inst, W, h, opts)
        log(f"accuracy: {result['accuracy']}")
    if not args.no_legs:
        result["batched_and_served"] = compact_batch_and_serve(args)
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        result["cpu_baseline"] = cpu_baseline(ctx)
        log(f"cpu baseline: {result['cpu_baseline']}")
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--window", type=int, default=200, help="integration steps per bench step")
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c64")
    ap.add_argument("--method", choices=["pc4", "rk4"], default="pc4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the complex64 vs complex128 comparisons")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the compact batched and served runs")
    ap.add_argument("--leg-batch", type=int, default=24, help="solves of the compact batch")
    ap.add_argument("--leg-serve", type=int, default=24, help="requests of the compact serving run")
    ap.add_argument("--leg-qps", type=float, default=2.0)
    ap.add_argument("--placement-trials", type=int, default=6,
                    help="workspace allocations tried before the timed run (the fastest is kept)")
    ap.add_argument("--no-carry", action="store_true",
                    help="restart the multistep history in every bench step")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB copy (for scaling hardware byte counters)")
    ap.add_argument("--mode", choices=["single", "batch", "serve", "adaptive", "paths", "sector", "gap",
                                       "tsearch", "scaling"], default="single")
    ap.add_argument("--ts-sizes", default="10,12,14")
    ap.add_argument("--scaling-sizes", default="12,16,20,24,28,30")
    ap.add_argument("--scaling-oracle-max", type=int, default=20)
    ap.add_argument("--ts-instances", type=int, default=8)
    ap.add_argument("--ts-algorithms", default="x,xy")
    ap.add_argument("--ts-rel", type=float, default=0.05)
    ap.add_argument("--ts-batched", action="store_true",
                    help="solve each round of the T_s search as one batch (refused: see find_ts)")
    ap.add_argument("--n-gap", type=int, default=20)
    ap.add_argument("--gap-path", default="cbc")
    ap.add_argument("--gap-points", type=int, default=21)
    ap.add_argument("--n-sector", type=int, default=34, help="qubits of the sector mode")
    ap.add_argument("--w-sector", type=int, default=-1,
                    help="weight of the sector (default n/2, gap mode n/3; -2: full space)")
    ap.add_argument("--sector-paths", default="linear,cbc")
    ap.add_argument("--n-paths", type=int, default=26, help="qubits of the paths mode")
    ap.add_argument("--paths-kinds", default="linear,nonlinear,cbc")
    ap.add_argument("--paths-autotune", action="store_true",
                    help="time H psi under the autotuner's candidate plans first")
    ap.add_argument("--atol", type=float, default=1e-9)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--batch-n-lo", type=int, default=14)
    ap.add_argument("--batch-n-hi", type=int, default=22)
    ap.add_argument("--resident-max-n", type=int, default=0,
                    help="batch mode: solves up to this size run resident (one workgroup each)")
    ap.add_argument("--baseline-subset", type=int, default=16)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--qps", type=float, default=1.0)
    ap.add_argument("--n-max", type=int, default=28)
    ap.add_argument("--ticks", type=int, default=64)
    ap.add_argument("--hbm-budget", type=float, default=200.0, help="GB")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the engine runs on one GPU; multi-GPU sharding is not implemented, so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        return run_batch_mode(args)
    if args.mode == "serve":
        return run_serve_mode(args)
    if args.mode == "adaptive":
        return run_adaptive_mode(args)
    if args.mode == "paths":
        return run_paths_mode(args)
    if args.mode == "sector":
        return run_sector_mode(args)
    if args.mode == "gap":
        return run_gap_mode(args)
    if args.mode == "tsearch":
        return run_tsearch_mode(args)
    if args.mode == "scaling":
        return run_scaling_mode(args)

    return run_single_mode(args)


if __name__ == "__main__":
    main()
