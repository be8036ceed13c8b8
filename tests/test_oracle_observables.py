"""Pins of the oracle's reductions (Sec. II.A normalisation, Sec. III.B):
overlap, state fidelity, basis mass and energy against values fixed by the
mathematics, not by the oracle's own formulas.

* overlap: <e_a|psi> = psi_a and <psi|e_a> = conj(psi_a) fix which argument is
  conjugated; a hand-computed two-amplitude case fixes the sum.
* state fidelity: |<phi|psi>|^2 of two one-qubit states a relative phase theta
  apart is cos^2(theta / 2); a complex state against itself gives 1; a basis
  target gives |psi_w|^2.
* basis mass: repeated indices count once.
* energy: on a basis state |z> an exact-cover Hamiltonian gives the number of
  violated-clause units sum_c (b_a + b_b + b_c - 1)^2, counted directly from
  the clauses; on an eigenvector of the dense matrix (numpy.kron, an
  independent construction) it gives the eigenvalue; a product state under the
  unit transverse field has the closed form n (1 - sin 2a) / 2.

Each pin is written as a check that takes the function under test, so that
the planted mistakes below (a conjugate on the wrong side, a missing
conjugate, a factor of two, a squared modulus dropped) are shown to fail it."""
import math

import numpy as np
import pytest

from oracle import observables as O
from paper_1311_3938_amd import instances as I

from _dense import dense_h

RNG = np.random.default_rng(20251)


def _cstate(n, rng=RNG):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


# ---- overlap ---------------------------------------------------------------

def _overlap_pins_hold(overlap):
    psi = _cstate(3)
    for a in range(8):
        e = np.zeros(8, dtype=complex)
        e[a] = 1.0
        if abs(overlap(e, psi) - psi[a]) > 1e-15:
            return False
        if abs(overlap(psi, e) - np.conj(psi[a])) > 1e-15:
            return False
    # by hand: phi = (1, i)/sqrt2, psi = (1, 1)/sqrt2 -> (1 - i)/2
    phi = np.array([1.0, 1j]) / math.sqrt(2)
    ps = np.array([1.0, 1.0]) / math.sqrt(2)
    if abs(overlap(phi, ps) - (1 - 1j) / 2) > 1e-15:
        return False
    # antilinear in the first argument, linear in the second
    c = 0.3 - 1.7j
    phi, psi = _cstate(4), _cstate(4)
    if abs(overlap(c * phi, psi) - np.conj(c) * overlap(phi, psi)) > 1e-14:
        return False
    if abs(overlap(phi, c * psi) - c * overlap(phi, psi)) > 1e-14:
        return False
    return True


def test_overlap_pinned():
    assert _overlap_pins_hold(O.overlap)


@pytest.mark.parametrize("wrong", [
    lambda phi, psi: complex(np.sum(phi * np.conj(psi))),   # conjugate on the wrong side
    lambda phi, psi: complex(np.sum(phi * psi)),            # no conjugate
    lambda phi, psi: complex(np.sum(np.conj(phi) * psi)) * 2,
])
def test_overlap_pins_catch_planted_mistakes(wrong):
    assert not _overlap_pins_hold(wrong)


# ---- state fidelity and basis mass -----------------------------------------

def _fidelity_pins_hold(fid):
    for theta in np.linspace(0.0, 2 * math.pi, 13):
        phi = np.array([1.0, 1.0]) / math.sqrt(2)
        psi = np.array([1.0, np.exp(1j * theta)]) / math.sqrt(2)
        if abs(fid(phi, psi) - math.cos(theta / 2) ** 2) > 1e-14:
            return False
    # a complex state against itself: fidelity one
    phi = np.array([1.0, 1j]) / math.sqrt(2)
    if abs(fid(phi, phi) - 1.0) > 1e-15:
        return False
    psi = _cstate(4)
    for w in (0, 5, 15):
        e = np.zeros(16, dtype=complex)
        e[w] = 1.0
        if abs(fid(e, psi) - abs(psi[w]) ** 2) > 1e-15:
            return False
    # a global phase on either state does not change it
    phi = _cstate(4)
    if abs(fid(np.exp(0.7j) * phi, np.exp(-2.1j) * psi) - fid(phi, psi)) > 1e-14:
        return False
    return True


def test_state_fidelity_pinned():
    assert _fidelity_pins_hold(O.state_fidelity)


@pytest.mark.parametrize("wrong", [
    lambda phi, psi: abs(np.sum(np.conj(phi) * psi)),              # modulus, not its square
    lambda phi, psi: float(np.real(np.sum(np.conj(phi) * psi)) ** 2),  # real part only
    lambda phi, psi: abs(np.sum(phi * psi)) ** 2,                   # no conjugate
])
def test_fidelity_pins_catch_planted_mistakes(wrong):
    assert not _fidelity_pins_hold(wrong)


def test_basis_mass_counts_each_state_once():
    psi = _cstate(5)
    by_loop = sum(abs(psi[z]) ** 2 for z in (3, 5, 17))
    assert O.basis_mass(psi, [3, 5, 3, 17, 5]) == pytest.approx(by_loop, abs=1e-16)
    assert O.basis_mass(psi, []) == 0.0
    assert O.basis_mass(psi, range(32)) == pytest.approx(1.0, abs=1e-14)


# ---- energy ----------------------------------------------------------------

def _clause_energy(z, clauses):
    """sum_c (b_a + b_b + b_c - 1)^2 with b_q bit q-1 of z (eq. (final_ham))."""
    return sum((sum((z >> (q - 1)) & 1 for q in c) - 1) ** 2 for c in clauses)


def _energy_pins_hold(energy):
    # basis states of an exact-cover problem: the clause count, exactly
    n = 7
    clauses = I.ec3_random_clauses(n, 6, np.random.default_rng(5))
    hf = I.ec3_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    for z in (0, 1, 37, 90, 127):
        e = np.zeros(1 << n, dtype=complex)
        e[z] = 1.0
        if energy(hf, 0.0, e) != float(_clause_energy(z, clauses)):
            return False
    # eigenvectors of the dense matrix of a mixed X/Y/Z Hamiltonian
    inst = I.random_terms(5, 14, np.random.default_rng(8)).instance([I.SCHED_CONST], I.linear_path(1.0))
    vals, vecs = np.linalg.eigh(dense_h(inst, 0.0))
    for k in (0, 7, 31):
        if abs(energy(inst, 0.0, vecs[:, k]) - vals[k]) > 1e-12 * max(1.0, abs(vals[k])):
            return False
    # a complex state: <psi|H|psi> from the dense matrix
    psi = _cstate(5)
    ref = float(np.real(np.conj(psi) @ dense_h(inst, 0.0) @ psi))
    if abs(energy(inst, 0.0, psi) - ref) > 1e-12:
        return False
    # product state cos a |0> + sin a |1> per qubit under sum (1 - sigma^x)/2
    n, a = 6, 0.37
    tf = I.transverse_terms(n).instance([I.SCHED_CONST], I.linear_path(1.0))
    q = np.array([math.cos(a), math.sin(a)], dtype=complex)
    prod = q
    for _ in range(n - 1):
        prod = np.kron(q, prod)
    if abs(energy(tf, 0.0, prod) - n * (1 - math.sin(2 * a)) / 2) > 1e-13:
        return False
    return True


def test_energy_pinned():
    assert _energy_pins_hold(O.energy)


def _energy_no_conj(ham, t, psi):
    from oracle.sqh import apply_h
    return float(np.real(np.sum(psi * apply_h(ham, t, psi))))


def _energy_twice(ham, t, psi):
    return 2.0 * O.energy(ham, t, psi)


def _energy_imag(ham, t, psi):
    from oracle.sqh import apply_h
    v = np.vdot(psi, apply_h(ham, t, psi))
    return float(abs(v))


@pytest.mark.parametrize("wrong", [_energy_no_conj, _energy_twice, _energy_imag])
def test_energy_pins_catch_planted_mistakes(wrong):
    assert not _energy_pins_hold(wrong)
