"""Pins of the oracle's integrators (Sec. II.B) against closed forms, dense
propagation and convergence order."""
import math

import numpy as np
import pytest

from oracle import integrate, observables, sqh
from paper_1311_3938_amd import instances as I
from tests._dense import dense_h, magnus4_propagate


def _rabi(omega0, Omega, omega):
    """H = (w0/2) sz + (W/2)(cos wt sx + sin wt sy): a circularly driven spin."""
    t = I.TermList(1)
    t.add({1: "Z"}, omega0 / 2.0, 0)
    t.add({1: "X"}, 1.0, 1)
    t.add({1: "Y"}, 1.0, 2)
    return t.instance([I.SCHED_CONST, I.trig_t(Omega / 2.0, omega, 0.0),
                       I.trig_t(Omega / 2.0, omega, -math.pi / 2.0)], I.linear_path(1.0))


@pytest.mark.parametrize("method", ["rk4", "pc4"])
def test_rabi_closed_form(method):
    """P(|0> -> |1>) = W^2/(W^2+d^2) sin^2(sqrt(W^2+d^2) t/2), d = w0 - w.  Holds
    only with sigma^y = [[0,-i],[i,0]] and the bit convention of Sec. II.A."""
    w0, W, w, T = 1.0, 0.3, 0.8, 10.0
    inst = _rabi(w0, W, w)
    psi0 = np.array([1.0, 0.0], dtype=np.complex128)
    psi = integrate.evolve(inst, psi0, 0.0, T, 4000, method)
    d = w0 - w
    r = math.sqrt(W * W + d * d)
    p1 = W * W / (r * r) * math.sin(r * T / 2.0) ** 2
    assert abs(psi[1]) ** 2 == pytest.approx(p1, abs=1e-10)
    # the wrong rotation sense (d = w0 + w) would give a far smaller amplitude
    r_bad = math.sqrt(W * W + (w0 + w) ** 2)
    assert abs(W * W / r_bad ** 2 * math.sin(r_bad * T / 2) ** 2 - p1) > 1e-2


@pytest.mark.slow
def test_landau_zener_asymptotics():
    """H = (v t/2) sz + (D/2) sx on [-tau, tau]: P_stay -> exp(-pi D^2 / 2v).  A loose
    pin: the finite window leaves an oscillating error of a few 1e-3 at tau = 50;
    the step keeps h |lambda| <= 0.1 so that RK4's damping stays below 1e-6."""
    v, D, tau = 1.0, 0.5, 50.0
    t = I.TermList(1)
    t.add({1: "Z"}, v / 2.0, 0)
    t.add({1: "X"}, D / 2.0, 1)
    inst = t.instance([I.poly_s([0.0, 1.0]), I.SCHED_CONST], I.linear_path(1.0))
    psi = integrate.evolve(inst, np.array([1.0, 0.0], complex), -tau, tau, 25000, "rk4")
    assert abs(psi[0]) ** 2 == pytest.approx(math.exp(-math.pi * D * D / (2 * v)), abs=1e-2)


@pytest.mark.parametrize("path", [I.linear_path(4.0), I.sin2_path(4.0)])
@pytest.mark.parametrize("method", ["rk4", "pc4"])
def test_commuting_hamiltonian_exact_phases(path, method):
    """Diagonal H(t) = s(t) E(z): psi_T(z) = exp(-i E(z) int_0^T s dt) psi_0(z), and
    the integral is T/2 for both paths."""
    n = 6
    rng = np.random.default_rng(21)
    ft = I.sk_terms(n, *I.sk_couplings(n, rng))
    inst = ft.instance([I.SCHED_S], path)
    psi0 = I.random_state(n, rng)
    E = sqh.diagonal(I.sk_terms(n, *I.sk_couplings(n, np.random.default_rng(21))).instance(
        [I.SCHED_CONST], path), 0.0)
    exact = np.exp(-1j * E * path["T"] / 2.0) * psi0
    psi = integrate.evolve(inst, psi0, 0.0, path["T"], 1600, method, shift=float(E.mean()))
    # global error of a 4th-order method on exp(-i lam t): ~ T |lam|^5 h^4 / 120
    lam = float(np.max(np.abs(E - E.mean())))
    bound = 4.0 * path["T"] * lam ** 5 * (path["T"] / 1600) ** 4 / 120.0
    assert np.linalg.norm(psi - exact) < max(bound, 1e-12)


def test_transverse_field_product_state():
    """H(t) = sum_q m_q(t) sx_q: each qubit turns by exp(-i A_q sx), A_q = int m_q dt."""
    n = 5
    T = 3.0
    wts = [0.5, 1.0, -0.7, 0.3, 1.2]
    t = I.TermList(n)
    for q in range(n):
        t.add({q + 1: "X"}, wts[q], 0)
    inst = t.instance([I.SCHED_ONE_MINUS_S], I.linear_path(T))
    A = [w * T / 2.0 for w in wts]                      # int_0^T (1 - t/T) dt = T/2
    psi0 = np.zeros(1 << n, complex)
    psi0[0] = 1.0
    z = np.arange(1 << n)
    exact = np.ones(1 << n, complex)
    for q in range(n):
        bit = (z >> q) & 1
        exact *= np.where(bit == 0, math.cos(A[q]), -1j * math.sin(A[q]))
    lam = sum(abs(w) for w in wts)
    bound = 4.0 * T * lam ** 5 * (T / 600) ** 4 / 120.0
    for method in ("rk4", "pc4"):
        psi = integrate.evolve(inst, psi0, 0.0, T, 600, method)
        assert np.linalg.norm(psi - exact) < bound


def _random_td_instance(n, seed):
    rng = np.random.default_rng(seed)
    t = I.random_terms(n, 14, rng, max_weight_ops=3, n_sched=3)
    return t.instance([I.SCHED_ONE_MINUS_S, I.poly_s([0.0, 1.0, -1.0]), I.trig_t(0.8, 2.0, 0.3)],
                      I.sin2_path(2.0)), rng


@pytest.mark.parametrize("method", ["rk4", "pc4"])
def test_dense_magnus_propagation(method):
    """Oracle vs 4th-order Magnus propagation with dense matrix exponentials (n = 4)."""
    inst, rng = _random_td_instance(4, 31)
    psi0 = I.random_state(4, rng)
    ref = magnus4_propagate(inst, psi0, 0.0, 2.0, 800)
    got = integrate.evolve(inst, psi0, 0.0, 2.0, 800, method)
    assert np.linalg.norm(got - ref) < 1e-8


@pytest.mark.parametrize("method", ["rk4", "pc4"])
def test_fourth_order_convergence(method):
    """Halving h divides the global error by ~2^4 (a dropped or wrong weight in
    either Adams formula or in RK4 breaks this)."""
    inst, rng = _random_td_instance(3, 41)
    psi0 = I.random_state(3, rng)
    ref = magnus4_propagate(inst, psi0, 0.0, 2.0, 2000)
    errs = []
    for K in (100, 200, 400):
        errs.append(np.linalg.norm(integrate.evolve(inst, psi0, 0.0, 2.0, K, method) - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 11.0 < r1 < 22.0 and 11.0 < r2 < 22.0, errs


def test_norm_drift_small():
    """Both methods lose norm only through their principal root: per step
    |r(i h lam)| - 1 = O((h rho)^6) with rho the spectral radius of H (about
    (h rho)^6/144 for RK4, 0.39 (h rho)^6 for the PEC scheme)."""
    inst, rng = _random_td_instance(4, 51)
    psi0 = I.random_state(4, rng)
    rho = max(np.max(np.abs(np.linalg.eigvalsh(dense_h(inst, t)))) for t in np.linspace(0, 2, 9))
    K = 400
    bound = K * (2.0 / K * rho) ** 6
    for method in ("rk4", "pc4"):
        psi = integrate.evolve(inst, psi0, 0.0, 2.0, K, method)
        assert abs(observables.norm2(psi) - 1.0) < bound


def test_pc4_counts_one_evaluation_per_step():
    inst, rng = _random_td_instance(3, 61)
    c = integrate.Counter()
    integrate.evolve(inst, I.random_state(3, rng), 0.0, 1.0, 50, "pc4", counter=c)
    # 3 RK4 bootstrap steps (4 evaluations each), f_3, then one per step
    assert c.matvecs == 12 + 1 + (50 - 3)
    c = integrate.Counter()
    integrate.evolve(inst, I.random_state(3, rng), 0.0, 1.0, 50, "rk4", counter=c)
    assert c.matvecs == 200


def test_shift_only_changes_phase_in_the_limit():
    inst, rng = _random_td_instance(3, 71)
    psi0 = I.random_state(3, rng)
    a = integrate.evolve(inst, psi0, 0.0, 2.0, 800, "rk4", shift=0.0)
    b = integrate.evolve(inst, psi0, 0.0, 2.0, 800, "rk4", shift=3.0)
    assert np.linalg.norm(a - b) < 1e-9


def test_adaptive_meets_tolerance_and_replays_bitwise():
    inst, rng = _random_td_instance(4, 81)
    psi0 = I.random_state(4, rng)
    ref = magnus4_propagate(inst, psi0, 0.0, 2.0, 2000)
    psi, segs, cnt = integrate.evolve_adaptive(inst, psi0, 0.0, 2.0, atol=1e-9, h0=0.05)
    assert np.linalg.norm(psi - ref) < 1e-6
    assert sum(k for (_, _, k) in segs) == cnt.steps
    assert segs[0][0] == 0.0
    end = segs[-1][0] + segs[-1][1] * segs[-1][2]
    assert end == pytest.approx(2.0, abs=1e-12)
    rep = integrate.evolve_segments(inst, psi0, 0.0, 2.0, segs)
    assert np.array_equal(rep, psi)
    # too large a first step must be rejected and halved
    psi2, segs2, cnt2 = integrate.evolve_adaptive(inst, psi0, 0.0, 2.0, atol=1e-9, h0=0.5)
    assert cnt2.rejected > 0
    assert np.linalg.norm(psi2 - ref) < 1e-6


def test_planted_mistakes_are_caught(monkeypatch):
    """A wrong Adams weight must fail the convergence pin."""
    inst, rng = _random_td_instance(3, 41)
    psi0 = I.random_state(3, rng)
    ref = magnus4_propagate(inst, psi0, 0.0, 2.0, 2000)
    monkeypatch.setattr(integrate, "AM4", (9.0, 19.0, -5.0, 1.1))
    errs = [np.linalg.norm(integrate.evolve(inst, psi0, 0.0, 2.0, K, "pc4") - ref)
            for K in (100, 200)]
    assert not (11.0 < errs[0] / errs[1] < 22.0)
    monkeypatch.setattr(integrate, "AM4", (9.0, 19.0, -5.0, 1.0))
    monkeypatch.setattr(integrate, "AB4", (55.0, -59.0, 37.0, -8.0))
    errs = [np.linalg.norm(integrate.evolve(inst, psi0, 0.0, 2.0, K, "pc4") - ref)
            for K in (100, 200)]
    assert not (11.0 < errs[0] / errs[1] < 22.0)


def test_adaptive_refuses_unreachable_tolerance():
    """An atol below the rounding floor of the estimate is refused up front; an
    estimate that still cannot fall below atol (here: a floor declared finer
    than the float64 arithmetic really is) ends the run after a bounded number
    of halvings instead of halving forever."""
    inst, rng = _random_td_instance(3, 91)
    psi0 = I.random_state(3, rng)
    with pytest.raises(ValueError):
        integrate.evolve_adaptive(inst, psi0, 0.0, 2.0, atol=1e-30, h0=0.1)
    with pytest.raises(RuntimeError):
        integrate.evolve_adaptive(inst, psi0, 0.0, 2.0, atol=1e-30, h0=0.1, unit_roundoff=2.0 ** -120)
