"""Pins of the oracle's Pauli-string product against textbook dense matrices."""
import json
import os

import numpy as np
import pytest

from oracle import sqh, observables
from paper_1311_3938_amd import instances as I
from tests._dense import dense_pauli, dense_h

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_pauli_string_matches_kron(n):
    rng = np.random.default_rng(100 + n)
    N = 1 << n
    for _ in range(60):
        x = int(rng.integers(0, N))
        z = int(rng.integers(0, N))
        psi = rng.normal(size=N) + 1j * rng.normal(size=N)
        got = sqh.apply_pauli(psi, n, x, z)
        want = dense_pauli(n, x, z) @ psi
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_time_dependent_h_matches_dense():
    rng = np.random.default_rng(7)
    n = 4
    t = I.random_terms(n, 25, rng, n_sched=3)
    inst = t.instance([I.poly_s([0.3, -1.0, 2.0]), I.trig_t(0.7, 1.3, 0.2), I.SCHED_CONST],
                      I.sin2_path(3.0))
    psi = I.random_state(n, rng)
    for tt in (0.0, 0.37, 1.9, 3.0):
        H = dense_h(inst, tt)
        np.testing.assert_allclose(sqh.apply_h(inst, tt, psi), H @ psi, atol=1e-12)
        # Hermitian: real weights times Pauli strings
        np.testing.assert_allclose(H, H.conj().T, atol=1e-14)
        np.testing.assert_allclose(sqh.diagonal(inst, tt), _diag_terms_only(inst, tt),
                                   atol=1e-12)


def _diag_terms_only(inst, t):
    """Diagonal of the x = 0 terms' dense matrix (diagonal() ignores flips)."""
    n = inst.n
    sub = I.TermList(n)
    for l in range(len(inst.w)):
        if int(inst.x[l]) == 0:
            sub.add_masks(0, inst.z[l], inst.w[l], inst.sid[l])
    d = sub.instance(inst.scheds, inst.path)
    return np.real(np.diag(dense_h(d, t)))


def test_bit_order_worked_example():
    """Fig. ec3: z = 1098 has the bitstring z_13..z_1 = 0010001001010 and up-bits
    2, 4, 7, 11; the three clauses printed in Fig. 1098N13 are all satisfied."""
    g = json.load(open(os.path.join(GOLDEN, "ec3_fig_1098.json")))
    z = g["solution"]
    assert int(g["bitstring_msb_first"], 2) == z
    up = [q for q in range(1, g["n"] + 1) if (z >> (q - 1)) & 1]
    assert up == g["upbits"]
    inst = I.ec3_terms(g["n"], [tuple(c) for c in g["clauses"]]).instance(
        [I.SCHED_CONST], I.linear_path(1.0))
    d = sqh.diagonal(inst, 0.0)
    assert d[z] == 0.0
    assert d.min() == 0.0
    # sigma^z_q on |z> gives (-1)^{z_q}: a single Z term reads the same bits
    for q in range(1, g["n"] + 1):
        zt = I.TermList(g["n"])
        zt.add({q: "Z"}, 1.0, 0)
        dq = sqh.diagonal(zt.instance([I.SCHED_CONST], I.linear_path(1.0)), 0.0)
        assert dq[z] == (-1.0 if q in g["upbits"] else 1.0)


def test_plus_state_is_zero_energy_ground_state_of_hx():
    """|+>^n is the ground state of H^x = sum (n_i/2)(1 - sigma^x_i) with energy 0."""
    n = 6
    w = [1.0, 2.0, 3.0, 1.0, 2.0, 1.0]
    inst = I.transverse_terms(n, w).instance([I.SCHED_CONST], I.linear_path(1.0))
    psi = I.plus_state(n)
    np.testing.assert_allclose(sqh.apply_h(inst, 0.0, psi), 0.0, atol=1e-14)
    rng = np.random.default_rng(3)
    for _ in range(5):
        v = I.random_state(n, rng)
        assert observables.energy(inst, 0.0, v) >= -1e-12


def test_schedules_closed_forms():
    p = I.linear_path(4.0)
    assert sqh.schedule_value(I.SCHED_ONE_MINUS_S, 1.0, p) == pytest.approx(0.75)
    assert sqh.schedule_value(I.SCHED_S, 1.0, p) == pytest.approx(0.25)
    assert sqh.schedule_value(I.SCHED_S_ONE_MINUS_S, 2.0, p) == pytest.approx(0.25)
    q = I.sin2_path(2.0)
    assert sqh.path_s(q, 1.0) == pytest.approx(0.5)
    assert sqh.path_s(q, 2.0) == pytest.approx(1.0)
    w = I.poly_s([1.0], 0.25, 0.5)
    assert sqh.schedule_value(w, 1.0, p) == 1.0      # s = 0.25: inside, closed low end
    assert sqh.schedule_value(w, 2.0, p) == 0.0      # s = 0.5: outside, open high end
    wc = I.poly_s([1.0], 0.25, 0.5, hi_closed=True)
    assert sqh.schedule_value(wc, 2.0, p) == 1.0


def test_row_wise_product_matches_full_product():
    rng = np.random.default_rng(9)
    n = 6
    inst = I.random_terms(n, 30, rng, n_sched=2).instance(
        [I.SCHED_S, I.trig_t(1.0, 0.7)], I.linear_path(2.0))
    psi = I.random_state(n, rng)
    full = sqh.apply_h(inst, 0.8, psi, shift=0.3)
    rows = rng.choice(1 << n, 20, replace=False)
    got = sqh.apply_h_rows(inst, 0.8, lambda idx: psi[idx], rows, shift=0.3)
    np.testing.assert_allclose(got, full[rows], atol=1e-13)
    np.testing.assert_allclose(sqh.diagonal_rows(inst, 0.8, rows), sqh.diagonal(inst, 0.8)[rows],
                               atol=1e-13)


@pytest.mark.parametrize("n,seed", [(9, 1), (12, 2)])
def test_parallel_product_is_the_plain_product(n, seed):
    """apply_h_parallel (row blocks of apply_h_rows on threads) gives exactly
    apply_h's values, and so does an evolution that uses it."""
    from oracle import integrate
    rng = np.random.default_rng(seed)
    inst = I.random_terms(n, 3 * n, rng, n_sched=2).instance(
        [I.SCHED_ONE_MINUS_S, I.SCHED_S], I.linear_path(3.0))
    psi = I.random_state(n, rng)
    a = sqh.apply_h(inst, 1.3, psi, shift=0.7)
    b = sqh.apply_h_parallel(inst, 1.3, psi, shift=0.7, threads=4, block=1 << (n - 3))
    assert np.array_equal(a, b)
    y0 = integrate.evolve(inst, psi, 0.2, 0.5, 9, "pc4", 0.4)
    y1 = integrate.evolve(inst, psi, 0.2, 0.5, 9, "pc4", 0.4,
                          apply=lambda *a_: sqh.apply_h_parallel(*a_, threads=3, block=1 << (n - 2)))
    assert np.array_equal(y0, y1)
