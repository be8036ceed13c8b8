"""GPU: the benchmark workloads at their own sizes.

* 12-qubit EC3 (10 clauses, linear path, T = 20, |+>^12, 2000 steps): the whole
  path against the oracle, RK4 and the paper-literal predictor-corrector.
* 24-qubit EC3 with XX catalyst (T = 50), adaptive steps: complex64 against
  complex128 on the same accepted grid (the oracle cannot hold this size for
  a full run; the adaptive rules themselves are checked against the oracle in
  test_gpu_evolve)."""
import functools

import numpy as np
import pytest

from oracle import integrate, observables
from paper_1311_3938_amd import instances as I
from tests._gpu import TOL, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


@functools.lru_cache(maxsize=None)
def _oracle_ec3(method, shift):
    inst = I.workload_ec3_linear()
    return integrate.evolve(inst, I.plus_state(12), 0.0, 20.0, 2000, method, shift)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("method,shift", [("rk4", 0.0), ("pc4", 20.0)])
def test_ec3_12_full_path(eng, dt, method, shift):
    engine, ctx = eng
    inst = I.workload_ec3_linear()
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(I.plus_state(12), dt)
    engine.evolve(ctx, ham, psi, 0.0, 20.0, method=method, n_steps=2000, shift=shift)
    ref = _oracle_ec3(method, shift)
    got = to_host(psi)
    assert np.linalg.norm(got - ref) < TOL[dt]
    f_gpu, e_min = engine.ground_mass(ctx, ham, 20.0, psi)
    f_ref, e_ref = observables.ground_mass(inst, 20.0, ref)
    assert e_min == e_ref
    assert abs(f_gpu - f_ref) < TOL[dt]
    ham.free()


def test_ec3_catalyst_24_adaptive_c64_vs_c128(eng):
    engine, ctx = eng
    import torch
    inst = I.workload_ec3_catalyst()          # n = 24, 20 clauses, 24 XX pairs, T = 50
    ham = engine.Hamiltonian(ctx, inst)
    T = inst.path["T"]
    t1 = 0.05 * T                             # a window at the start of the path
    lo, hi = ham.spectral_bounds(0.0, T)
    shift = 0.5 * (lo + hi)
    kw = dict(method="pc4", n_steps=0, atol=1e-9, h0=0.05, window=8, shift=shift,
              stab_limit=0.2155, record_cap=4096)
    p128 = torch.full((1 << 24,), 2.0 ** -12, dtype=torch.complex128, device="cuda")
    st128, segs = engine.evolve(ctx, ham, p128, 0.0, t1, **kw)
    assert st128["steps"] > 0 and abs(st128["t_reached"] - t1) < 1e-12
    p64 = torch.full((1 << 24,), 2.0 ** -12, dtype=torch.complex64, device="cuda")
    engine.evolve(ctx, ham, p64, 0.0, t1, method="pc4", replay=segs, shift=shift)
    dpsi = torch.linalg.vector_norm(p64.to(torch.complex128) - p128).item()
    assert dpsi < TOL["c64"]
    f64, _ = engine.ground_mass(ctx, ham, T, p64)
    f128, _ = engine.ground_mass(ctx, ham, T, p128)
    assert abs(f64 - f128) < TOL["c64"]
    ham.free()
