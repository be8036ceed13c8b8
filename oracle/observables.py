"""Oracle: reductions over a state vector (Sec. II.A normalisation, Sec. III.B).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

  * norm^2            sum_z |alpha_z|^2 (eq. (expansion))
  * overlap           <phi|psi> = sum_z conj(phi_z) psi_z
  * state fidelity    |<phi|psi>|^2, i.e. P_1(T) = |<psi(T)|w>|^2 for |phi> = |w>
  * basis mass        sum over a list of basis states of |psi_z|^2
  * ground mass       mass on the ground set of a diagonal Hamiltonian: the basis
                      states whose energy is within rel_tol*max(1,|E_min|) of the
                      minimum; for a unique solution this is P_1(T)
  * energy            <psi|H(t)|psi> (real for Hermitian H), the quantity E(T)
                      of Sec. III.B
"""
from __future__ import annotations

import numpy as np

from .sqh import apply_h, diagonal


def norm2(psi):
    return float(np.sum(np.abs(np.asarray(psi, dtype=np.complex128)) ** 2))


def overlap(phi, psi):
    return complex(np.sum(np.conj(np.asarray(phi, dtype=np.complex128)) *
                          np.asarray(psi, dtype=np.complex128)))


def state_fidelity(phi, psi):
    return abs(overlap(phi, psi)) ** 2


def basis_mass(psi, indices):
    psi = np.asarray(psi, dtype=np.complex128)
    idx = np.unique(np.asarray(indices, dtype=np.int64))
    return float(np.sum(np.abs(psi[idx]) ** 2))


def ground_set(ham, t, rel_tol=1e-9):
    """(E_min, indices) of the basis states with E(z) <= E_min + rel_tol*max(1, |E_min|),
    E(z) being the diagonal of H(t)."""
    d = diagonal(ham, t)
    e_min = float(d.min())
    sel = np.nonzero(d <= e_min + rel_tol * max(1.0, abs(e_min)))[0]
    return e_min, sel


def ground_mass(ham, t, psi, rel_tol=1e-9):
    e_min, sel = ground_set(ham, t, rel_tol)
    return basis_mass(psi, sel), e_min


def energy(ham, t, psi):
    psi = np.asarray(psi, dtype=np.complex128)
    return float(np.real(np.vdot(psi, apply_h(ham, t, psi))))
