"""Pins of the interpolation paths of Sec. IV.A: the clause-by-clause path
(eq. (cbc)-(kpath)), the nonlinear path (eq. (nlpath)), the piecewise-linear
schedule that expresses them, and the XYZ initial Hamiltonian (eq. (Hixyz))."""
import math

import numpy as np
import pytest

from oracle import sqh, integrate
from paper_1311_3938_amd import instances as I
from tests._dense import dense_h, dense_pauli


def _clause_energy(n, clauses):
    """sum_c (z_a + z_b + z_c - 1)^2 by counting bits (eq. (hci))."""
    z = np.arange(1 << n)
    e = np.zeros(1 << n)
    for c in clauses:
        e += (sum((z >> (q - 1)) & 1 for q in c) - 1) ** 2
    return e


def _hd_literal(n, clauses, s):
    """H_d(s) of eq. (kpath) written out window by window: s_k = m s - k + 1,
    the k-th window counts for 0 <= s_k < 1 (half open; the last window also
    at s_m = 1), H_k = the first k clauses, H_0 = H_m = 0."""
    m = len(clauses)
    H = [np.zeros(1 << n)] + [_clause_energy(n, clauses[:k]) for k in range(1, m)] + [np.zeros(1 << n)]
    out = np.zeros(1 << n)
    for k in range(1, m + 1):
        sk = m * s - k + 1
        if 0.0 <= sk < 1.0 or (k == m and sk == 1.0):
            out += (1.0 - sk) * H[k - 1] + sk * H[k]
    return out


def _xy_dense(n, clauses):
    """eq. (Hixy) from Kronecker products: 3m 1 - sum n_ij/2 (X_i X_j + Y_i Y_j)."""
    N = 1 << n
    H = 3.0 * len(clauses) * np.eye(N, dtype=complex)
    for c in clauses:
        for a in range(3):
            for b in range(a + 1, 3):
                i, j = c[a], c[b]
                for P in ("X", "Y"):
                    x, z = I.pauli_masks(n, {i: P, j: P})
                    H -= 0.5 * dense_pauli(n, x, z)
    return H


@pytest.mark.parametrize("n,m,seed", [(6, 4, 0), (7, 5, 1), (8, 7, 2)])
def test_clause_by_clause_matches_window_formula(n, m, seed):
    """The whole H(s) of eq. (cbc) assembled from the ramps equals (1-s) H^xy +
    s H_f + H_d(s) built window by window, at the joints s = k/m and between."""
    clauses = I.ec3_random_clauses(n, m, np.random.default_rng(seed))
    T = 3.0
    inst = I.clause_by_clause(n, clauses, I.linear_path(T))
    Hxy = _xy_dense(n, clauses)
    Ef = _clause_energy(n, clauses)
    ss = sorted(set([k / m for k in range(m + 1)] + list(np.random.default_rng(seed).uniform(0, 1, 9))))
    for s in ss:
        t = s * T
        want = (1 - s) * Hxy + np.diag(s * Ef + _hd_literal(n, clauses, s))
        assert np.max(np.abs(dense_h(inst, t) - want)) < 1e-12, s
        # the oracle's own diagonal and product agree with it
        assert np.max(np.abs(sqh.diagonal(inst, t) - np.real(np.diag(want)))) < 1e-12
        v = I.random_state(n, np.random.default_rng(7))
        assert np.linalg.norm(sqh.apply_h(inst, t, v) - want @ v) < 1e-11


def test_clause_by_clause_end_points():
    """H(0) = H^xy and H(1) = H_f: H_d vanishes at both ends (H_0 = H_m = 0)."""
    n, m = 7, 6
    clauses = I.ec3_random_clauses(n, m, np.random.default_rng(4))
    inst = I.clause_by_clause(n, clauses, I.linear_path(2.0))
    assert np.max(np.abs(dense_h(inst, 0.0) - _xy_dense(n, clauses))) < 1e-12
    assert np.max(np.abs(dense_h(inst, 2.0) - np.diag(_clause_energy(n, clauses)))) < 1e-12


def test_clause_ramp_values():
    """Clause c of m: 0, the secondary ramp s_c, 1, then 1 - s_m."""
    m = 5
    for c in range(1, m):
        r = I.clause_ramp(c, m)
        path = I.linear_path(1.0)
        for s in np.linspace(0, 1, 101):
            if s < (c - 1) / m:
                want = 0.0
            elif s < c / m:
                want = m * s - c + 1
            elif s < (m - 1) / m:
                want = 1.0
            else:
                want = 1.0 - (m * s - m + 1)
            assert sqh.schedule_value(r, s, path) == pytest.approx(want, abs=1e-12)
    with pytest.raises(ValueError):
        I.clause_ramp(m, m)


def test_pwl_schedule_edges():
    """Constant outside the knots; the later value holds at a repeated knot."""
    sch = I.pwl_s([(0.2, 1.0), (0.5, 3.0), (0.5, -1.0), (0.9, 0.0)])
    path = I.linear_path(1.0)
    for s, want in [(0.0, 1.0), (0.2, 1.0), (0.35, 2.0), (0.5, -1.0), (0.7, -0.5), (0.9, 0.0), (1.0, 0.0)]:
        assert sqh.schedule_value(sch, s, path) == pytest.approx(want, abs=1e-15)
    with pytest.raises(ValueError):
        I.pwl_s([(0.5, 0.0), (0.4, 1.0)])


@pytest.mark.parametrize("seed", [0, 3])
def test_nonlinear_path(seed):
    """eq. (nlpath): H(s) - (1-s) H^xy - s H_f = alpha s (1-s) H_{m-1}, with the
    removed clause one that keeps the clause graph connected."""
    n, m, alpha = 7, 6, 8.0
    clauses = I.ec3_random_clauses(n, m, np.random.default_rng(seed))
    inst = I.nonlinear_path(n, clauses, I.linear_path(1.0), alpha=alpha)
    k = inst.meta["removed"]
    reduced = clauses[:k] + clauses[k + 1:]
    assert I.clause_graph_components(n, reduced) == I.clause_graph_components(n, clauses)
    # every earlier clause would have split the graph
    for j in range(k):
        assert I.clause_graph_components(n, clauses[:j] + clauses[j + 1:]) > \
            I.clause_graph_components(n, clauses)
    Hxy = _xy_dense(n, clauses)
    for s in (0.0, 0.3, 0.5, 1.0):
        want = (1 - s) * Hxy + np.diag(s * _clause_energy(n, clauses)
                                       + alpha * s * (1 - s) * _clause_energy(n, reduced))
        assert np.max(np.abs(dense_h(inst, s) - want)) < 1e-12


def test_clause_graph_components():
    assert I.clause_graph_components(6, [(1, 2, 3), (4, 5, 6)]) == 2
    assert I.clause_graph_components(6, [(1, 2, 3), (3, 4, 5)]) == 2   # bit 6 alone
    assert I.clause_graph_components(5, [(1, 2, 3), (3, 4, 5)]) == 1
    # a chain: every clause holds bits no other clause has, so none can go
    with pytest.raises(ValueError):
        I.removable_clause(7, [(1, 2, 3), (3, 4, 5), (5, 6, 7)])
    # clause 0 alone holds bit 7; clause 1 lies on a cycle
    cl = [(1, 2, 7), (1, 2, 3), (3, 4, 5), (1, 5, 6), (2, 4, 6)]
    assert I.removable_clause(7, cl) == 1


@pytest.mark.parametrize("n", [4, 6])
def test_xyz_dicke_states_are_zero_energy_ground_states(n):
    """eq. (Hixyz) is a sum of n_ij (1 - SWAP_ij) >= 0, and every Dicke state
    (eq. (initstate)) is symmetric, so H^xyz annihilates it: the ground
    energy is 0 in every Hamming-weight sector."""
    clauses = I.ec3_random_clauses(n, n - 1, np.random.default_rng(n))
    inst = I.xyz_initial_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    H = dense_h(inst, 0.0)
    assert np.linalg.eigvalsh(H)[0] == pytest.approx(0.0, abs=1e-12)
    for w in range(n + 1):
        v = I.dicke_state(n, w)
        assert np.linalg.norm(H @ v) < 1e-12
        assert np.linalg.norm(sqh.apply_h(inst, 0.0, v)) < 1e-12
    # one clause is the three-spin Heisenberg ferromagnet 3 - sum of the three
    # SWAPs: 0 on total spin 3/2 (4 states), 3 on the two spin-1/2 doublets
    t = I.xyz_initial_terms(n, [clauses[0]]).instance([I.SCHED_CONST], I.linear_path(1.0))
    ev = np.round(np.linalg.eigvalsh(dense_h(t, 0.0)), 12)
    assert np.count_nonzero(ev == 0.0) == 4 << (n - 3)
    assert np.count_nonzero(ev == 3.0) == 4 << (n - 3)


def test_cbc_evolution_keeps_sectors_and_converges():
    """The clause-by-clause path commutes with Sigma^z (only diagonal terms are
    added), so a Dicke state stays in its sector.  Its ramps have kinks at
    s = k/m: RK4 with the kinks on the grid and pc4 restarted at every kink
    (one call per window) converge at 4th order (error / 16 per halving),
    while pc4 run across the kinks drops to 2nd order (error / 4), since its
    history then spans a jump of dH/dt."""
    n, m, T = 7, 5, 4.0
    clauses = I.ec3_random_clauses(n, m, np.random.default_rng(9))
    inst = I.clause_by_clause(n, clauses, I.linear_path(T))
    psi0 = I.dicke_state(n, 3)
    wt = np.bitwise_count(np.arange(1 << n, dtype=np.uint64))
    ref = integrate.evolve(inst, psi0, 0.0, T, 6400, "rk4")
    e_rk, e_win, e_pc = [], [], []
    for K in (400, 800):
        e_rk.append(np.linalg.norm(integrate.evolve(inst, psi0, 0.0, T, K, "rk4") - ref))
        y = psi0
        for k in range(m):
            y = integrate.evolve(inst, y, k * T / m, (k + 1) * T / m, K // m, "pc4", shift=7.5)
        assert np.max(np.abs(y[wt != 3])) == 0.0
        e_win.append(np.linalg.norm(y - ref))
        e_pc.append(np.linalg.norm(integrate.evolve(inst, psi0, 0.0, T, K, "pc4", shift=7.5) - ref))
    assert e_rk[0] / e_rk[1] > 12.0
    assert e_win[0] / e_win[1] > 12.0
    assert 3.0 < e_pc[0] / e_pc[1] < 6.0
