"""GPU: degenerate Hamiltonians, each at n = 1, 5 and 14 in complex128 and
complex64: no terms at all (H = 0: H psi is zero and evolution leaves the
state as it is) and identity terms only (H(t) = 2.5 s(t) 1: H psi is a
multiple of psi, evolution only turns the phase).  H psi against its closed
form; fixed-step pc4 and RK4 runs with the centred shift against the
oracle's, and against the closed form psi0 exp(-i 2.5 T / 2)."""
import numpy as np
import pytest

from oracle import integrate
from paper_1311_3938_amd import instances as I

from tests._gpu import TOL, to_dev, to_host

pytestmark = pytest.mark.gpu

T = 3.0


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 5, 14])
@pytest.mark.parametrize("kind", ["zero", "identity"])
def test_degenerate_hamiltonians(eng, kind, n, dt):
    engine, ctx = eng
    t = I.TermList(n)
    if kind == "identity":
        t.add({}, 2.5, 0)
    inst = t.instance([I.SCHED_S], I.linear_path(T))
    ham = engine.Hamiltonian(ctx, inst)
    psi0 = I.random_state(n, np.random.default_rng(100 + n))
    dpsi0 = to_dev(psi0, dt)
    psi0_r = to_host(dpsi0)                  # the values the device holds
    out = to_host(engine.apply(ctx, ham, 1.2, dpsi0))
    want = (2.5 * 1.2 / T if kind == "identity" else 0.0) * psi0_r
    assert np.max(np.abs(out - want)) <= (1e-6 if dt == "c64" else 1e-14)
    lo, hi = ham.spectral_bounds(0.0, T)
    shift = 0.5 * (lo + hi)
    closed = psi0_r * (np.exp(-1j * 2.5 * T / 2.0) if kind == "identity" else 1.0)
    for method, K in (("pc4", 40), ("rk4", 8)):   # h rho = 0.09 and 0.47
        psi = to_dev(psi0, dt)
        engine.evolve(ctx, ham, psi, 0.0, T, method=method, n_steps=K, shift="center")
        got = to_host(psi)
        ref = integrate.evolve(inst, psi0_r, 0.0, T, K, method, shift)
        assert np.linalg.norm(got - ref) < TOL[dt], (method, np.linalg.norm(got - ref))
        # the residual H - shift is a multiple of 1 that the integrator follows
        # to its own order; the phase of the shift is exact
        assert np.linalg.norm(got - closed) < 1e-3
    ham.free()
