"""Pins of the problem Hamiltonians (Sec. II.C, Sec. III.A) and their invariants."""
import math

import numpy as np
import pytest

from oracle import sqh, observables, integrate
from paper_1311_3938_amd import instances as I


def _clause_penalty(n, clauses):
    """sum_c (z_a + z_b + z_c - 1)^2 by direct bit counting (eq. (hci))."""
    z = np.arange(1 << n)
    e = np.zeros(1 << n, dtype=np.int64)
    for c in clauses:
        s = sum((z >> (q - 1)) & 1 for q in c)
        e += (s - 1) ** 2
    return e


@pytest.mark.parametrize("n,m,seed", [(5, 4, 0), (7, 6, 1), (9, 8, 2), (12, 10, 3)])
def test_ec3_expansion_equals_clause_count(n, m, seed):
    """eq. (final_ham) (the expanded Pauli form) equals the clause penalty exactly."""
    clauses = I.ec3_random_clauses(n, m, np.random.default_rng(seed))
    assert len(set(clauses)) == m and all(len(set(c)) == 3 for c in clauses)
    inst = I.ec3_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    d = sqh.diagonal(inst, 0.0)
    ref = _clause_penalty(n, clauses)
    assert np.array_equal(d, ref.astype(np.float64))
    # integer energies in [0, 4m]; the all-ones string violates every clause by 2
    assert d.min() >= 0 and d.max() <= 4 * m
    assert d[(1 << n) - 1] == 4 * m


def test_energy_bound_by_success_probability():
    """Sec. III.B: with a gapped integer spectrum and E_1 = 0, E >= Omega (1 - P_1)."""
    rng = np.random.default_rng(11)
    n = 8
    for _ in range(200):
        clauses = I.ec3_random_clauses(n, 6, rng)
        d = _clause_penalty(n, clauses)
        if d.min() == 0 and np.count_nonzero(d == 0) == 1:
            break
    inst = I.ec3_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    w = int(np.argmin(d))
    for _ in range(20):
        psi = I.random_state(n, rng)
        p1 = abs(psi[w]) ** 2
        assert observables.energy(inst, 0.0, psi) >= (1.0 - p1) - 1e-12
        mass, emin = observables.ground_mass(inst, 0.0, psi)
        assert emin == 0.0 and mass == pytest.approx(p1, abs=1e-15)


def test_hamming_weight_sectors_conserved_under_xy_path():
    """H^xy and H_f commute with Sigma^z (eq. (Sigmaz)): a state inside the
    weight-2 and weight-4 sectors never leaks out of them, and each sector keeps
    its mass up to the method's own (tiny) norm drift."""
    n = 7
    rng = np.random.default_rng(5)
    clauses = I.ec3_random_clauses(n, 5, rng)
    inst = I.interpolated(n, I.xy_initial_terms(n, clauses), I.ec3_terms(n, clauses),
                          I.linear_path(3.0))
    wt = np.bitwise_count(np.arange(1 << n, dtype=np.uint64))
    psi0 = I.random_state(n, rng)
    psi0[(wt != 2) & (wt != 4)] = 0.0
    psi0 /= np.linalg.norm(psi0)
    psi = integrate.evolve(inst, psi0, 0.0, 3.0, 300, "pc4", shift=10.0)
    assert np.max(np.abs(psi[(wt != 2) & (wt != 4)])) == 0.0
    for k in (2, 4):
        sel = wt == k
        m0 = np.sum(np.abs(psi0[sel]) ** 2)
        # drift bound K (h rho)^6 with the spectrum of H(s) inside [0, 20], shift 10
        assert np.sum(np.abs(psi[sel]) ** 2) == pytest.approx(m0, rel=300 * (0.01 * 10.0) ** 6)


def test_dicke_state_normalised():
    """eq. (initstate): C(n, w)^{-1/2} sum over weight-w basis states has norm 1."""
    for n, w in [(5, 2), (8, 3), (10, 5)]:
        v = I.dicke_state(n, w)
        assert observables.norm2(v) == pytest.approx(1.0, abs=1e-14)
        assert np.count_nonzero(v) == math.comb(n, w)


def test_sk_and_catalyst_shapes():
    inst = I.workload_sk_sin2(n=10, T=5.0, seed=1)
    # transverse field (identity + n X) + SK (n(n-1)/2 ZZ + n Z)
    assert inst.n_terms == 1 + 10 + 45 + 10
    inst2 = I.workload_ec3_catalyst(n=9, m=6, n_pairs=9, T=5.0, seed=2)
    xs = [int(x) for x in inst2.x if bin(int(x)).count("1") == 2]
    assert len(xs) == 9 and len(set(xs)) == 9
