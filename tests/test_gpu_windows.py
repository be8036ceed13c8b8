"""GPU: the large and batched workloads against the oracle, windowed.

* 24-qubit EC3 with an XX catalyst (20 clauses, 24 pairs, T = 50) and its
  22-qubit counterpart: from one checkpoint state at several points of the
  path, a window of fixed predictor-corrector steps (its RK4 bootstrap
  included) on the GPU in complex64 (compensated state, float64 reductions)
  and complex128, and on the oracle from the same vector.  The checkpoint is a
  seeded random state rounded to complex64 (so both precisions start from
  exactly the same numbers); the step size and the shift come from a bound
  on the spectrum computed from the term weights alone.  A whole run at this
  size would take the oracle hours; a window of 8-20 steps takes it a minute.
* a complex64 batch of mixed 14-16-qubit members (EC3 and SK, each with a
  catalyst), 100-200 steps each, every member against the oracle.

Bars: ||dpsi|| <= 1e-6 (complex64), <= 1e-10 (complex128)."""
import functools
import math

import numpy as np
import pytest

from oracle import integrate, sqh
from paper_1311_3938_amd import instances as I
from tests._gpu import TOL, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


def _catalyst(n):
    if n == 24:
        return I.workload_ec3_catalyst()           # the 24-qubit workload itself
    return I.workload_ec3_catalyst(n=n, m=round(20 * n / 24), n_pairs=n, T=50.0, seed=I.seed_for(1, n))


def _step_and_shift(inst, t):
    """h with h * (bound + |shift|) = 0.1, from sum |w| max|f| (no device)."""
    path = inst.path
    svals = np.linspace(0.0, 1.0, 201)
    fmax = []
    for sc in inst.scheds:
        p = dict(path, kind="linear", T=1.0)
        fmax.append(max(abs(sqh.schedule_value(sc, s, p)) for s in svals))
    bound = 0.0
    ident = 0.0
    f_t = [sqh.schedule_value(sc, t, path) for sc in inst.scheds]
    for x, z, w, sid in zip(inst.x, inst.z, inst.w, inst.sid):
        bound += abs(w) * fmax[sid]
        if not int(x) and not int(z):
            ident += w * f_t[sid]
    shift = round(ident, 3)
    return 0.1 / (bound + abs(shift)), shift


def _oracle(inst, psi0, t0, t1, W, shift):
    return integrate.evolve(inst, psi0, t0, t1, W, "pc4", shift, apply=sqh.apply_h_parallel)


@functools.lru_cache(maxsize=None)
def _window(n, frac, W):
    inst = _catalyst(n)
    t_c = frac * inst.path["T"]
    h, shift = _step_and_shift(inst, t_c)
    rng = np.random.default_rng(1000 * n + int(100 * frac))
    start = I.random_state(n, rng).astype(np.complex64).astype(np.complex128)
    print(f"oracle window n={n} t_c={t_c:g} W={W} h={h:.3e} shift={shift}", flush=True)
    ref = _oracle(inst, start, t_c, t_c + W * h, W, shift)
    return inst, start, t_c, h, shift, ref


@pytest.mark.slow
@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n,frac,W", [(22, 0.3, 20), (22, 0.8, 20), (24, 0.55, 8)])
def test_catalyst_window_matches_oracle(eng, n, frac, W, dt):
    engine, ctx = eng
    inst, start, t_c, h, shift, ref = _window(n, frac, W)
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(start, dt)
    engine.evolve(ctx, ham, psi, t_c, t_c + W * h, method="pc4", n_steps=W, shift=shift)
    got = to_host(psi)
    err = float(np.linalg.norm(got - ref))
    print(f"window n={n} t_c={t_c:g} {dt}: |dpsi| = {err:.3e}", flush=True)
    assert err < TOL[dt]
    ham.free()


@pytest.mark.slow
def test_c64_batch_of_mixed_members_matches_oracle(eng):
    engine, ctx = eng
    import torch
    b = engine.Batch(ctx, torch.complex64, capacity=6)
    slots = {}
    for j in range(6):
        inst = I.workload_batch_member(j, n_lo=14, n_hi=16)
        K = 100 + 20 * j
        h, shift = _step_and_shift(inst, 0.0)
        t1 = K * h
        start = I.plus_state(inst.n).astype(np.complex64).astype(np.complex128)
        hm = engine.Hamiltonian(ctx, inst)
        slots[b.admit(hm, to_dev(start, "c64"), 0.0, t1, K, shift)] = (inst, start, K, t1, shift, hm)
    got = {}
    while b.step(16) > 0 or len(got) < len(slots):
        for s in b.poll():
            got[s] = to_host(b.retire(s)[0])
    b.close()
    for s, (inst, start, K, t1, shift, hm) in slots.items():
        ref = _oracle(inst, start, 0.0, t1, K, shift)
        err = float(np.linalg.norm(got[s] - ref))
        print(f"batch member n={inst.n} {inst.meta['kind']} K={K}: |dpsi| = {err:.3e}", flush=True)
        assert err < TOL["c64"]
        hm.free()
