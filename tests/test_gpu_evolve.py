"""GPU parity of aqc_evolve (through the C ABI) against the oracle's integrators."""
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
def _oracle_fixed(key, method, K, t0, t1, shift):
    inst, psi0 = _PROBLEMS[key]()
    return integrate.evolve(inst, psi0, t0, t1, K, method, shift)


def _ec3_12():
    # the 12-qubit exact-cover workload: 10 clauses, T = 20, |+>^12
    return I.workload_ec3_linear(), I.plus_state(12)


def _cat_15():
    inst = I.workload_ec3_catalyst(n=15, m=12, n_pairs=15, T=5.0, seed=21)
    return inst, I.random_state(15, np.random.default_rng(2))


_PROBLEMS = {"ec3_12": _ec3_12, "cat_15": _cat_15}


def _run(engine, ctx, key, dt, method, K, t0, t1, shift):
    inst, psi0 = _PROBLEMS[key]()
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(psi0, dt)
    # the guard only has to catch divergence: near its stability limit (h rho
    # = 0.2 here) the predictor-corrector itself grows the norm by ~1.5% over
    # 400 steps, exactly as the oracle does
    st, _ = engine.evolve(ctx, ham, psi, t0, t1, method=method, n_steps=K, shift=shift,
                          check_every=50, norm_tol=0.1)
    return inst, ham, psi, st


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("method", ["pc4", "rk4"])
def test_evolve_ec3_window_matches_oracle(eng, method, dt):
    """First fifth of the 12-qubit EC3 path at h = T/2000 (the workload's step)."""
    engine, ctx = eng
    K, t0, t1, shift = 400, 0.0, 4.0, 20.0
    inst, ham, psi, st = _run(engine, ctx, "ec3_12", dt, method, K, t0, t1, shift)
    ref = _oracle_fixed("ec3_12", method, K, t0, t1, shift)
    got = to_host(psi)
    err = np.linalg.norm(got - ref)
    assert err < TOL[dt], err
    f_gpu, _ = engine.ground_mass(ctx, ham, inst.path["T"], psi)
    f_ref, _ = observables.ground_mass(inst, inst.path["T"], ref)
    assert abs(f_gpu - f_ref) < TOL[dt]
    assert st["steps"] == K
    assert st["matvecs"] == (K - 3 + 13 if method == "pc4" else 4 * K)
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("method", ["pc4", "rk4"])
@pytest.mark.parametrize("plan", ["tile", "stream", "stream_only"])
def test_evolve_two_pass_catalyst_matches_oracle(eng, method, dt, plan, monkeypatch):
    """15 qubits: flips above the last tile run in a high-bit pass ("tile"), or
    as stream groups of the last pass beside a register pass ("stream"), or
    all as stream groups in a single pass ("stream_only"); the stream plans
    alternate two y^p buffers, which every RK4 stage and pc4 step exercises."""
    engine, ctx = eng
    if plan != "tile":
        monkeypatch.setenv("AQC_STREAM", "1")
    if plan == "stream_only":
        monkeypatch.setenv("AQC_REGPASS", "0")
    K, t0, t1, shift = 60, 1.0, 1.6, 6.0
    inst, ham, psi, st = _run(engine, ctx, "cat_15", dt, method, K, t0, t1, shift)
    npass = ham.info()["n_passes"][0 if dt == "c64" else 1]
    assert npass == 1 if plan == "stream_only" else npass >= 2
    ref = _oracle_fixed("cat_15", method, K, t0, t1, shift)
    err = np.linalg.norm(to_host(psi) - ref)
    assert err < TOL[dt], err
    ham.free()


def test_evolve_center_shift_and_guard(eng):
    engine, ctx = eng
    from paper_1311_3938_amd import _lib
    inst, psi0 = _ec3_12()
    ham = engine.Hamiltonian(ctx, inst)
    lo, hi = ham.spectral_bounds(0.0, inst.path["T"])
    # H(s) = (1-s) H^x + s H_f with H^x in [0, 12] and H_f in [0, 4m]
    assert lo <= 0.0 + 1e-12 and hi >= 12.0 - 1e-12
    psi = to_dev(psi0, "c128")
    st, _ = engine.evolve(ctx, ham, psi, 0.0, 1.0, method="pc4", n_steps=100, shift="center",
                          stab_limit=0.2155)
    # the centred shift uses the enclosure over the call's own interval
    lo1, hi1 = ham.spectral_bounds(0.0, 1.0)
    assert st["shift_used"] == pytest.approx(0.5 * (lo1 + hi1), rel=1e-15)
    assert st["rho"] == pytest.approx(0.5 * (hi1 - lo1), rel=1e-12)
    ref = integrate.evolve(inst, psi0, 0.0, 1.0, 100, "pc4", st["shift_used"])
    assert np.linalg.norm(to_host(psi) - ref) < TOL["c128"]
    with pytest.raises(_lib.AqcError) as ei:
        engine.evolve(ctx, ham, to_dev(psi0, "c128"), 0.0, 1.0, method="pc4", n_steps=5,
                      shift="center", stab_limit=0.2155)
    assert ei.value.status == _lib.AQC_EUNSTABLE
    ham.free()


def test_norm_guard_trips_on_divergence(eng):
    """pc4 without a shift far beyond its stability limit: the guard stops it."""
    engine, ctx = eng
    from paper_1311_3938_amd import _lib
    inst, psi0 = _ec3_12()
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(psi0, "c128")
    with pytest.raises(_lib.AqcError) as ei:
        engine.evolve(ctx, ham, psi, 0.0, 20.0, method="pc4", n_steps=500, shift=0.0,
                      check_every=10, norm_tol=1e-2)
    assert ei.value.status == _lib.AQC_EUNSTABLE
    assert np.isfinite(to_host(psi)).all()
    ham.free()


def _adaptive_problem():
    rng = np.random.default_rng(81)
    inst = I.random_terms(8, 24, rng, max_weight_ops=3, n_sched=3).instance(
        [I.SCHED_ONE_MINUS_S, I.poly_s([0.0, 1.0, -1.0]), I.trig_t(0.8, 2.0, 0.3)],
        I.sin2_path(2.0))
    return inst, I.random_state(8, rng)


def test_adaptive_matches_oracle_decisions(eng):
    engine, ctx = eng
    inst, psi0 = _adaptive_problem()
    kw = dict(atol=1e-9, h0=0.2, window=8)
    ref, segs_ref, cnt = integrate.evolve_adaptive(inst, psi0, 0.0, 2.0, **kw)
    assert cnt.rejected > 0
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(psi0, "c128")
    st, segs = engine.evolve(ctx, ham, psi, 0.0, 2.0, method="pc4", n_steps=0, record_cap=256,
                             **kw)
    assert st["n_segments"] == len(segs_ref)
    assert [s[2] for s in segs] == [s[2] for s in segs_ref]
    np.testing.assert_allclose(np.array(segs)[:, :2], np.array(segs_ref)[:, :2], rtol=0, atol=0)
    assert st["steps"] == cnt.steps and st["rejected"] == cnt.rejected
    assert np.linalg.norm(to_host(psi) - ref) < TOL["c128"]
    # complex64 replays the oracle's accepted grid
    psi64 = to_dev(psi0, "c64")
    engine.evolve(ctx, ham, psi64, 0.0, 2.0, method="pc4", replay=segs_ref)
    assert np.linalg.norm(to_host(psi64) - integrate.evolve_segments(inst, psi0, 0.0, 2.0,
                                                                      segs_ref)) < TOL["c64"]
    ham.free()


def test_deterministic_bitwise(eng):
    engine, ctx = eng
    inst, psi0 = _cat_15()
    ham = engine.Hamiltonian(ctx, inst)
    outs = []
    for _ in range(2):
        psi = to_dev(psi0, "c64")
        engine.evolve(ctx, ham, psi, 0.0, 0.5, method="pc4", n_steps=50, shift=6.0)
        outs.append(to_host(psi))
    assert np.array_equal(outs[0], outs[1])
    ham.free()


def test_adaptive_below_precision_floor_fails_fast(eng):
    """complex64 cannot meet atol = 1e-12 at 2^12 amplitudes (its rounding
    floor is far above): the controller stops with AQC_EUNSTABLE."""
    engine, ctx = eng
    from paper_1311_3938_amd import _lib
    inst, psi0 = _ec3_12()
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(psi0, "c64")
    with pytest.raises(_lib.AqcError) as ei:
        engine.evolve(ctx, ham, psi, 0.0, 1.0, method="pc4", n_steps=0, atol=1e-12, h0=0.01,
                      window=8, shift=20.0)
    assert ei.value.status == _lib.AQC_EUNSTABLE
    assert "precision floor" in str(ei.value)
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("key", ["ec3_12", "cat_15"])
def test_carry_chain_equals_one_call(eng, dt, key, monkeypatch):
    """Fixed-step pc4 in pieces with a carry performs exactly the steps of one
    call: the pieces split inside the RK4 bootstrap (after 2 steps), at its end
    (3, where the first evaluation of the multistep part is pending) and in the
    predictor-corrector part.  A chain's step is fixed by its first call, so a
    chain [2, 38] and a chain [2, 1, 7, 30] run on the same grid and must agree
    bit for bit; once the phase is applied both match a self-contained call
    (whose step (t1 - t0)/40 may differ from the chain's in the last bit).  The
    15-qubit plan uses stream groups, so the two alternating y^p buffers are
    carried too."""
    engine, ctx = eng
    import torch
    from paper_1311_3938_amd import _lib
    if key == "cat_15":
        monkeypatch.setenv("AQC_STREAM", "1")
    inst, psi0 = _PROBLEMS[key]()
    ham = engine.Hamiltonian(ctx, inst)
    K, t0, t1, shift = 40, 0.5, 0.5 + 40 * 0.004, 9.0
    h = (t1 - t0) / K
    kw = dict(method="pc4", shift=shift)
    ref = to_dev(psi0, dt)
    engine.evolve(ctx, ham, ref, t0, t1, n_steps=K, **kw)
    one = to_dev(psi0, dt)
    c1 = engine.new_carry()
    opts, _, _ = engine.evolve_opts(n_steps=K, **kw)
    ws1 = engine.workspace(ctx, engine.evolve_workspace_bytes(ham, engine.dtype_code(one), opts))
    for a, b, k in ((t0, t0 + 2 * h, 2), (t0 + 2 * h, t1, K - 2)):
        engine.evolve(ctx, ham, one, a, b, ws=ws1, carry=c1, n_steps=k, **kw)
    pieces = [2, 1, 7, K - 10]
    chain = to_dev(psi0, dt)
    ws2 = engine.workspace(ctx, ws1.numel())
    c2 = engine.new_carry()
    ta = t0
    for k in pieces:
        engine.evolve(ctx, ham, chain, ta, ta + k * h, ws=ws2, carry=c2, n_steps=k, **kw)
        ta += k * h
    assert c2.k == K and c1.k == K
    assert torch.equal(one, chain)
    phase = complex(c2.phase_re, c2.phase_im)
    got = to_host(chain) * phase
    assert np.linalg.norm(got - to_host(ref)) < (1e-12 if dt == "c128" else 1e-6)
    # a call that does not continue its chain is refused
    with pytest.raises(_lib.AqcError):
        engine.evolve(ctx, ham, chain, ta + h, ta + 2 * h, ws=ws2, carry=c2, n_steps=1, **kw)
    ham.free()


@pytest.mark.parametrize("t1", [0.01, 0.35])
def test_adaptive_interval_shorter_than_first_steps(eng, t1):
    """Adaptive runs over an interval shorter than the first step (t1 = 0.01,
    h0 = 0.2) or than the RK4 bootstrap (t1 = 0.35): the last step is cut to
    end at t1; the accepted grid and the state equal the oracle's."""
    engine, ctx = eng
    inst, psi0 = _adaptive_problem()
    kw = dict(atol=1e-9, h0=0.2, window=8)
    ref, segs_ref, cnt = integrate.evolve_adaptive(inst, psi0, 0.0, t1, **kw)
    ham = engine.Hamiltonian(ctx, inst)
    psi = to_dev(psi0, "c128")
    st, segs = engine.evolve(ctx, ham, psi, 0.0, t1, method="pc4", n_steps=0, record_cap=64, **kw)
    assert st["n_segments"] == len(segs_ref)
    assert [s[2] for s in segs] == [s[2] for s in segs_ref]
    np.testing.assert_allclose(np.array(segs)[:, :2], np.array(segs_ref)[:, :2], rtol=0, atol=0)
    assert st["steps"] == cnt.steps and st["rejected"] == cnt.rejected
    assert st["t_reached"] == t1
    assert np.linalg.norm(to_host(psi) - ref) < TOL["c128"]
    ham.free()
