"""GPU: the serving loop admits requests over time, batches them continuously,
and returns for every request exactly the state of solving it alone."""
import math

import numpy as np
import pytest

from paper_1311_3938_amd import instances as I

pytestmark = pytest.mark.gpu


def _requests(serve, k=6, T=1.5, n_lo=8, n_hi=15):
    reqs = []
    for i in range(k):
        inst = I.workload_serving_request(i, n_lo=n_lo, n_hi=n_hi)
        inst.path["T"] = T
        reqs.append(serve.Request(i, inst, arrival=0.02 * i))
    return reqs


def test_served_results_equal_alone():
    import torch
    from paper_1311_3938_amd import engine, serve
    reqs = _requests(serve)
    srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=2e9,
                       size_classes=((12, 4), (34, 4)), ticks=4, keep_states=True)
    res, wall = srv.run(reqs)
    srv.close()
    assert [r.rid for r in res] == [q.rid for q in reqs]
    ctx = engine.Context(0)
    for r, q in zip(res, reqs):
        assert r.finished >= r.admitted >= r.arrival - 1e-9
        ham = engine.Hamiltonian(ctx, q.inst)
        serve.choose_plan(ctx, ham, q.inst, torch.complex64)
        K, shift = serve.solve_plan(ctx, ham, q.T)
        assert r.steps == K
        N = 1 << q.n
        psi = torch.full((N,), 1.0 / math.sqrt(N), dtype=torch.complex64, device="cuda")
        engine.evolve(ctx, ham, psi, 0.0, q.T, method="pc4", n_steps=K, shift=shift)
        assert np.array_equal(psi.cpu().numpy(), r.extra["psi"])
        mass, _ = engine.ground_mass(ctx, ham, q.T, psi)
        assert mass == r.fidelity
        ham.free()
    ctx.close()


def test_budget_limits_admission():
    """With room for one request at a time, requests run one after another."""
    import torch
    from paper_1311_3938_amd import serve
    reqs = _requests(serve, k=3, T=0.5, n_lo=12, n_hi=12)
    for q in reqs:
        q.arrival = 0.0
    big = max(8 * (1 << q.n) * 8 for q in reqs)
    srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=big * 1.5,
                       size_classes=((34, 8),), ticks=4)
    res, wall = srv.run(reqs)
    srv.close()
    spans = sorted((r.admitted, r.finished) for r in res)
    for (a0, f0), (a1, f1) in zip(spans, spans[1:]):
        assert a1 >= f0 - 1e-3   # the next admission waits for memory


def test_two_classes_build_graphs_concurrently():
    """Both size classes step, retire and rebuild their graphs at the same time
    on two host threads while torch allocates and copies on a third; every
    served state still equals the state of solving the request alone."""
    import threading
    import torch
    from paper_1311_3938_amd import engine, serve
    reqs = _requests(serve, k=16, T=1.0, n_lo=8, n_hi=15)
    for q in reqs:
        q.arrival = 0.0
    stop = threading.Event()

    def churn():
        while not stop.is_set():
            x = torch.randn(1 << 16, device="cuda")
            x.cpu()

    th = threading.Thread(target=churn, daemon=True)
    th.start()
    try:
        srv = serve.Server(dtype=torch.complex64, hbm_budget_bytes=2e9,
                           size_classes=((11, 8), (34, 8)), ticks=2, graph=True, keep_states=True)
        res, wall = srv.run(reqs)
        srv.close()
    finally:
        stop.set()
        th.join()
    ctx = engine.Context(0)
    for r, q in zip(res, reqs):
        ham = engine.Hamiltonian(ctx, q.inst)
        serve.choose_plan(ctx, ham, q.inst, torch.complex64)
        K, shift = serve.solve_plan(ctx, ham, q.T)
        N = 1 << q.n
        psi = torch.full((N,), 1.0 / math.sqrt(N), dtype=torch.complex64, device="cuda")
        engine.evolve(ctx, ham, psi, 0.0, q.T, method="pc4", n_steps=K, shift=shift)
        assert np.array_equal(psi.cpu().numpy(), r.extra["psi"]), q.rid
        ham.free()
    ctx.close()
