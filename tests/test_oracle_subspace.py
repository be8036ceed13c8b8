"""Pins of the Hamming-weight sector oracle (Sec. III.A.2-3): the basis order
is the combinatorial number system, H^xy in the one-excitation sector is the
clause graph's hopping matrix, Dicke states are the zero-energy ground states
of H^xyz, and sector evolution equals the exact propagator of the sector
matrix."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import subspace, sqh
from paper_1311_3938_amd import instances as I
from tests._dense import dense_h


def _colex_rank(z):
    """sum over the set bits p_0 < p_1 < ... of C(p_k, k + 1)."""
    r, k, p = 0, 0, 0
    while z:
        if z & 1:
            r += math.comb(p, k + 1)
            k += 1
        z >>= 1
        p += 1
    return r


@pytest.mark.parametrize("n,w", [(1, 0), (1, 1), (5, 2), (8, 3), (10, 5), (12, 0), (12, 12), (13, 6)])
def test_basis_is_the_combinatorial_number_system(n, w):
    b = subspace.basis(n, w)
    assert len(b) == math.comb(n, w) == subspace.dim(n, w)
    assert all(bin(int(z)).count("1") == w for z in b)
    assert [_colex_rank(int(z)) for z in b] == list(range(len(b)))


def test_restrict_expand_round_trip():
    n, w = 9, 4
    rng = np.random.default_rng(1)
    v = rng.normal(size=subspace.dim(n, w)) + 1j * rng.normal(size=subspace.dim(n, w))
    full = subspace.expand(v, n, w)
    assert np.count_nonzero(full) == len(v)
    assert np.array_equal(subspace.restrict(full, n, w), v)
    d = subspace.dicke(n, w)
    assert np.allclose(subspace.expand(d, n, w), I.dicke_state(n, w), atol=1e-15)


def test_xy_one_excitation_sector_is_the_hopping_matrix():
    """In the weight-1 sector (basis |q> = bit q-1 set, q = 1..n) eq. (Hixy)
    acts as 3m 1 - A with A_ij = n_ij, the clause graph's weighted adjacency."""
    n = 8
    clauses = I.ec3_random_clauses(n, 6, np.random.default_rng(2))
    inst = I.xy_initial_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    A = np.zeros((n, n))
    for (i, j), c in I.clause_pair_counts(clauses).items():
        A[i - 1, j - 1] = A[j - 1, i - 1] = c
    want = 3 * len(clauses) * np.eye(n) - A
    M = np.array([subspace.apply_h(inst, 0.0, e, 1) for e in np.eye(n, dtype=complex)]).T
    assert np.max(np.abs(M - want)) < 1e-13


@pytest.mark.parametrize("n", [5, 8])
def test_dicke_is_zero_energy_in_every_sector(n):
    clauses = I.ec3_random_clauses(n, n - 2, np.random.default_rng(n))
    inst = I.xyz_initial_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    for w in range(n + 1):
        assert np.linalg.norm(subspace.apply_h(inst, 0.0, subspace.dicke(n, w), w)) < 1e-12


def test_sector_evolution_equals_exact_propagator():
    """Time-independent H^xy + H_f: the sector evolution (pc4, fine steps)
    matches expm(-i H_w t) of the dense sector block to 1e-9."""
    n, w, T = 8, 3, 1.5
    clauses = I.ec3_random_clauses(n, 6, np.random.default_rng(3))
    t = I.xy_initial_terms(n, clauses)
    t.extend(I.ec3_terms(n, clauses))
    inst = t.instance([I.SCHED_CONST], I.linear_path(T))
    b = subspace.basis(n, w)
    Hw = dense_h(inst, 0.0)[np.ix_(b, b)]
    psi0 = subspace.dicke(n, w)
    want = expm(-1j * T * Hw) @ psi0
    got = subspace.evolve(inst, psi0, w, 0.0, T, 3000, "pc4", shift=float(np.mean(np.real(np.diag(Hw)))))
    assert np.linalg.norm(got - want) < 1e-9


def test_one_state_sectors_only_pick_up_a_phase():
    """w = 0 and w = n hold one state each: psi(T) = exp(-i int E dt) psi(0)."""
    n, T = 6, 2.0
    clauses = I.ec3_random_clauses(n, 4, np.random.default_rng(4))
    inst = I.workload_ec3_paths(n=n, m=4, T=T, kind="cbc", seed=7)
    for w in (0, n):
        z = 0 if w == 0 else (1 << n) - 1
        # E(t) of the single state, integrated with Simpson's rule on a fine grid
        ts = np.linspace(0.0, T, 4001)
        E = np.array([sqh.diagonal(inst, t)[z] for t in ts])
        phi = (ts[1] - ts[0]) / 3 * (E[0] + E[-1] + 4 * E[1:-1:2].sum() + 2 * E[2:-1:2].sum())
        got = subspace.evolve(inst, np.ones(1, dtype=complex), w, 0.0, T, 3200, "rk4")
        assert abs(got[0] - np.exp(-1j * phi)) < 5e-8   # RK4 at h E <= 0.025


def test_non_conserving_hamiltonian_is_refused():
    inst = I.transverse_terms(4).instance([I.SCHED_CONST], I.linear_path(1.0))
    with pytest.raises(ValueError):
        subspace.apply_h(inst, 0.0, subspace.dicke(4, 2), 2)
