"""GPU: the batch engine (aqc_batch_*) gives each solve exactly the result it
gets alone, and matches the oracle."""
import numpy as np
import pytest

from oracle import integrate
from paper_1311_3938_amd import instances as I
from tests._gpu import TOL, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


def _mix():
    """Solves of different size and plan: one pass (n <= 13 for complex64),
    register hypercube passes, tile high passes for straddling pairs."""
    out = []
    for i, n in enumerate([9, 12, 14, 16, 15, 17]):
        inst = I.workload_batch_member(i, n_lo=n, n_hi=n)
        K = 20 + 7 * i
        T = inst.path["T"]
        t0, t1 = 0.1 * T, 0.1 * T + K * 0.004
        out.append((inst, t0, t1, K, 5.0 + i))
    return out


DEFAULT_TILING = {"c64": (13, 13, 4), "c128": (12, 12, 3)}


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("graph,reg", [(True, "auto"), (False, "auto"), (True, "mixed")])
def test_batch_equals_alone_bitwise(eng, dt, graph, reg):
    """reg = "mixed": the 16-qubit solve runs wide register passes with stream
    groups in its last pass, the 17-qubit one narrow register passes and tile
    high passes, the 14-qubit one a single pass with stream groups only, so one
    tick launches every kind of level and both y^p buffering schemes."""
    engine, ctx = eng
    import torch
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    mix = _mix()
    hams = [engine.Hamiltonian(ctx, inst) for inst, *_ in mix]
    if reg == "mixed":
        opts = {14: 4, 16: 3 | 4, 17: 2}
        for j, (inst, *_r) in enumerate(mix):
            if inst.n in opts:
                hams[j].set_tiling(tdt, *DEFAULT_TILING[dt], opts[inst.n])
    psi0 = [I.random_state(inst.n, np.random.default_rng(50 + j)) for j, (inst, *_r) in enumerate(mix)]
    alone = []
    for j, (inst, t0, t1, K, sh) in enumerate(mix):
        p = to_dev(psi0[j], dt)
        engine.evolve(ctx, hams[j], p, t0, t1, method="pc4", n_steps=K, shift=sh)
        alone.append(to_host(p))
    b = engine.Batch(ctx, tdt, capacity=8, graph=graph)
    states = {}
    # admit half, run a few ticks, then admit the rest (continuous batching)
    for j in range(3):
        inst, t0, t1, K, sh = mix[j]
        states[b.admit(hams[j], to_dev(psi0[j], dt), t0, t1, K, sh)] = j
    b.step(5)
    for j in range(3, len(mix)):
        inst, t0, t1, K, sh = mix[j]
        states[b.admit(hams[j], to_dev(psi0[j], dt), t0, t1, K, sh)] = j
    done = {}
    while True:
        na = b.step(4)
        for slot in b.poll():
            psi, st = b.retire(slot)
            j = states[slot]
            assert st["steps"] == mix[j][3]
            done[j] = to_host(psi)
        if na == 0 and len(done) == len(mix):
            break
    for j in range(len(mix)):
        assert np.array_equal(done[j], alone[j]), (j, np.abs(done[j] - alone[j]).max())
    b.close()
    for hm in hams:
        hm.free()


def test_batch_matches_oracle(eng):
    engine, ctx = eng
    import torch
    rng = np.random.default_rng(3)
    insts = [I.workload_batch_member(i, n_lo=8, n_hi=10) for i in range(4)]
    b = engine.Batch(ctx, torch.complex128, capacity=4)
    slots = {}
    for j, inst in enumerate(insts):
        psi0 = I.random_state(inst.n, rng)
        hm = engine.Hamiltonian(ctx, inst)
        K = 30 + 5 * j
        slots[b.admit(hm, to_dev(psi0, "c128"), 0.0, K * 0.003, K, 2.0)] = (inst, psi0, K, hm)
    got = {}
    while b.step(16) > 0 or len(got) < len(insts):
        for s in b.poll():
            got[s] = to_host(b.retire(s)[0])
    for s, (inst, psi0, K, hm) in slots.items():
        ref = integrate.evolve(inst, psi0, 0.0, K * 0.003, K, "pc4", 2.0)
        assert np.linalg.norm(got[s] - ref) < TOL["c128"]
        hm.free()
    b.close()


def test_batch_short_solves_and_empty_steps(eng):
    """Solves of 1 to 5 steps (the first three are RK4 bootstrap steps only)
    share ticks with a longer one and finish inside a group of ticks; a step
    of an empty batch does nothing.  Every result against the oracle."""
    engine, ctx = eng
    import torch
    b = engine.Batch(ctx, torch.complex128, capacity=8)
    assert b.step(4) == 0 and b.poll() == []
    rng = np.random.default_rng(9)
    slots = {}
    for j, K in enumerate([1, 2, 3, 4, 5, 40]):
        inst = I.workload_batch_member(j, n_lo=8, n_hi=10)
        psi0 = I.random_state(inst.n, rng)
        hm = engine.Hamiltonian(ctx, inst)
        t1 = K * 0.003
        slots[b.admit(hm, to_dev(psi0, "c128"), 0.0, t1, K, 1.5)] = (inst, psi0, K, t1, hm)
    got = {}
    while b.step(16) > 0 or len(got) < len(slots):
        for s in b.poll():
            got[s] = to_host(b.retire(s)[0])
    for s, (inst, psi0, K, t1, hm) in slots.items():
        ref = integrate.evolve(inst, psi0, 0.0, t1, K, "pc4", 1.5)
        assert np.linalg.norm(got[s] - ref) < TOL["c128"], K
        hm.free()
    assert b.step(4) == 0 and b.info()["active"] == 0
    b.close()


def _resident_oracle(inst, psi0, t0, t1, K, sh):
    from oracle import sqh
    return integrate.evolve(inst, psi0, t0, t1, K, "pc4", sh, apply=sqh.apply_h_parallel)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_resident_solves_match_oracle(eng, dt):
    """Resident solves (one workgroup runs a whole solve in one launch) beside
    ticked ones in one batch: every result against the oracle; the ticked
    ones also bit for bit against solving alone.  Sizes 9-17: one tile (9,
    12), a tile high pass (14-16), and 17 qubits above the resident limit."""
    engine, ctx = eng
    import torch
    tdt = torch.complex64 if dt == "c64" else torch.complex128
    mix = _mix()
    b = engine.Batch(ctx, tdt, capacity=8, resident_max_n=16)
    slots = {}
    for j, (inst, t0, t1, K, sh) in enumerate(mix):
        psi0 = I.random_state(inst.n, np.random.default_rng(70 + j)).astype(np.complex64).astype(np.complex128)
        hm = engine.Hamiltonian(ctx, inst)
        slots[b.admit(hm, to_dev(psi0, dt), t0, t1, K, sh)] = (inst, psi0, t0, t1, K, sh, hm)
    got = {}
    while b.step(8) > 0 or len(got) < len(slots):
        for s in b.poll():
            got[s] = to_host(b.retire(s)[0])
    b.close()
    for s, (inst, psi0, t0, t1, K, sh, hm) in slots.items():
        ref = _resident_oracle(inst, psi0, t0, t1, K, sh)
        err = float(np.linalg.norm(got[s] - ref))
        print(f"resident batch {dt} n={inst.n} K={K}: |dpsi| = {err:.3e}", flush=True)
        assert err < TOL[dt], (inst.n, err)
        if inst.n > 16:
            p = to_dev(psi0, dt)
            engine.evolve(ctx, hm, p, t0, t1, method="pc4", n_steps=K, shift=sh)
            assert np.array_equal(to_host(p), got[s])
        hm.free()


def test_resident_launches_while_others_run(eng):
    """Solves admitted while an earlier resident launch is still running go
    into a launch of their own; short and long, one to five steps included;
    every result against the oracle (complex128)."""
    engine, ctx = eng
    import torch
    b = engine.Batch(ctx, torch.complex128, capacity=4, resident_max_n=12)
    rng = np.random.default_rng(11)
    todo = []
    for j, K in enumerate([400, 1, 2, 3, 5, 60, 17, 250]):
        inst = I.workload_batch_member(20 + j, n_lo=8, n_hi=12)
        todo.append((inst, I.random_state(inst.n, rng), K, 0.6 + 0.1 * j))
    slots, got, nxt = {}, {}, 0

    def admit():
        nonlocal nxt
        inst, psi0, K, sh = todo[nxt]
        hm = engine.Hamiltonian(ctx, inst)
        slots[b.admit(hm, to_dev(psi0, "c128"), 0.0, K * 0.002, K, sh)] = (nxt, hm)
        nxt += 1

    while nxt < 4:
        admit()
    while len(got) < len(todo):
        b.step(4)
        for s in b.poll():
            j, hm = slots.pop(s)
            got[j] = to_host(b.retire(s)[0])
            hm.free()
            if nxt < len(todo):
                admit()
    b.close()
    for j, (inst, psi0, K, sh) in enumerate(todo):
        ref = _resident_oracle(inst, psi0, 0.0, K * 0.002, K, sh)
        assert np.linalg.norm(got[j] - ref) < TOL["c128"], (j, K)
