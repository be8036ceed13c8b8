"""GPU: the interpolation paths of Sec. IV.A through the C ABI against the
oracle: straight line, nonlinear (eq. (nlpath)) and clause-by-clause
(eq. (cbc)-(kpath)) between H^xy and an EC3 H_f, with a Dicke initial state
(eq. (initstate)).  The clause ramps are piecewise-linear schedules, one per
clause, so a 31-clause path uses all 32 schedule slots."""
import functools
import math

import numpy as np
import pytest

from oracle import integrate, sqh
from paper_1311_3938_amd import instances as I
from tests._gpu import TOL, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

KINDS = ("linear", "nonlinear", "cbc")
N_EV, M_EV, T_EV, W_EV = 10, 8, 2.0, 3     # evolution case: n, clauses, T, Dicke weight


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


def _bound(inst):
    """A crude bound on |H(s) - identity part| for the step size: the sum of
    |weight| times the largest schedule value on [0, 1]."""
    path = I.linear_path(1.0)
    fmax = [max(abs(sqh.schedule_value(s, x, path)) for x in np.linspace(0, 1, 201)) for s in inst.scheds]
    return sum(abs(w) * fmax[sid] for x, z, w, sid in zip(inst.x, inst.z, inst.w, inst.sid)
               if int(x) or int(z))


def _case(kind):
    inst = I.workload_ec3_paths(n=N_EV, m=M_EV, T=T_EV, kind=kind, seed=I.seed_for(5, 1))
    b = _bound(inst)
    K = int(math.ceil(T_EV * b / 0.15))      # pc4: h * rho <= 0.15 < 0.2155
    shift = 3.0 * M_EV                       # identity part of H^xy; H_f in [0, 4m]
    return inst, K, shift


@functools.lru_cache(maxsize=None)
def _oracle(kind, method, windows):
    inst, K, shift = _case(kind)
    psi0 = I.dicke_state(N_EV, W_EV)
    if method == "rk4":
        return integrate.evolve(inst, psi0, 0.0, T_EV, 200, "rk4")
    if not windows:
        return integrate.evolve(inst, psi0, 0.0, T_EV, K, "pc4", shift)
    m = M_EV
    y = psi0
    for k in range(m):
        y = integrate.evolve(inst, y, k * T_EV / m, (k + 1) * T_EV / m, -(-K // m), "pc4", shift)
    return y


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind", KINDS)
def test_paths_apply_n16(eng, kind, dt):
    """H(t) psi at 16 qubits (several tiles) at the clause joints s = k/m and
    between them."""
    engine, ctx = eng
    import torch
    n, m, T = 16, 13, 5.0
    inst = I.workload_ec3_paths(n=n, m=m, T=T, kind=kind, seed=I.seed_for(5, 2))
    ham = engine.Hamiltonian(ctx, inst)
    rng = np.random.default_rng(3)
    v = I.random_state(n, rng)
    dv = to_dev(v, dt)
    out = torch.empty_like(dv)
    tol = 1e-12 if dt == "c128" else 5e-6
    for s in (0.0, 1.0 / m, 0.37, 5.0 / m, (m - 1.0) / m, 0.97, 1.0):
        engine.apply(ctx, ham, s * T, dv, out)
        assert rel_err(to_host(out), sqh.apply_h(inst, s * T, v)) < tol, s
    ham.free()


# pc4 restarted per clause window only matters where the schedules have kinks
CASES = [(k, m, False) for k in KINDS for m in ("rk4", "pc4")] + [("cbc", "pc4", True)]


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind,method,windows", CASES)
def test_paths_evolve(eng, kind, method, windows, dt):
    """The whole path [0, T] from the Dicke state: RK4, pc4 across the clause
    kinks, and pc4 restarted at every kink (one call per window of T/m)."""
    engine, ctx = eng
    inst, K, shift = _case(kind)
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(I.dicke_state(N_EV, W_EV), dt)
    if method == "rk4":
        engine.evolve(ctx, ham, psi, 0.0, T_EV, method="rk4", n_steps=200)
    elif not windows:
        engine.evolve(ctx, ham, psi, 0.0, T_EV, method="pc4", n_steps=K, shift=shift)
    else:
        for k in range(M_EV):
            engine.evolve(ctx, ham, psi, k * T_EV / M_EV, (k + 1) * T_EV / M_EV, method="pc4",
                          n_steps=-(-K // M_EV), shift=shift)
    ref = _oracle(kind, method, windows)
    got = to_host(psi)
    assert np.linalg.norm(got - ref) < TOL[dt]
    wt = np.bitwise_count(np.arange(1 << N_EV, dtype=np.uint64))
    # the Hamming weight is conserved (up to rounding where two products cancel)
    assert np.linalg.norm(got[wt != W_EV]) < TOL[dt]
    e_gpu = engine.energy(ctx, ham, T_EV, psi)
    from oracle import observables
    assert abs(e_gpu - observables.energy(inst, T_EV, ref)) < {"c128": 1e-8, "c64": 1e-4}[dt]
    ham.free()


def test_cbc_all_schedule_slots(eng):
    """31 clauses: H^xy, H_f and 30 ramps fill the 32 schedule slots; a 33rd
    schedule is rejected."""
    engine, ctx = eng
    import torch
    from paper_1311_3938_amd import _lib as L
    n, m, T = 14, 31, 3.0
    clauses = I.ec3_random_clauses(n, m, np.random.default_rng(8))
    inst = I.clause_by_clause(n, clauses, I.linear_path(T))
    assert len(inst.scheds) == 32
    ham = engine.Hamiltonian(ctx, inst)
    v = I.random_state(n, np.random.default_rng(4))
    dv = to_dev(v, "c128")
    out = torch.empty_like(dv)
    for s in (0.0, 0.5 / m, 7.0 / m, 29.5 / m, 30.0 / m, 1.0):
        engine.apply(ctx, ham, s * T, dv, out)
        assert rel_err(to_host(out), sqh.apply_h(inst, s * T, v)) < 1e-12, s
    ham.free()
    bad = I.TermList(n)
    bad.add({1: "Z"}, 1.0, 32)
    with pytest.raises(L.AqcError):
        engine.Hamiltonian(ctx, bad.instance([I.SCHED_CONST] * 33, I.linear_path(T)))
