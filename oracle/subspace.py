"""Oracle: states and evolution restricted to one Hamming weight (Sec. III.A.2-3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

H^xyz (eq. (Hixyz)), H^xy (eq. (Hixy)) and a diagonal H_f all commute with
Sigma^z (eq. (Sigmaz)), so the number of 1-bits of the basis states is
conserved and only the C(n, w) states of weight w need to be kept, starting
for instance from their balanced superposition (eq. (initstate)).

Basis of the weight-w sector: every z with popcount(z) = w, in increasing
order of the integer z.  A sector state psi_s holds psi_s[r] = psi[basis[r]];
``expand`` puts it back into the 2^n space with zeros elsewhere.  The sector's
product and evolution are the full-space ones of ``sqh`` and ``integrate`` on
the expanded state, restricted again; that is exact because H maps the sector
into itself (checked on every product).
"""
from __future__ import annotations

import math

import numpy as np

from . import integrate, observables, sqh


def basis(n, w):
    """The weight-w basis states in increasing order (int64)."""
    z = np.arange(1 << n, dtype=np.uint64)
    return np.flatnonzero(np.bitwise_count(z) == w).astype(np.int64)


def dim(n, w):
    return math.comb(n, w)


def restrict(psi, n, w):
    return np.asarray(psi, dtype=np.complex128)[basis(n, w)]


def expand(psi_s, n, w):
    out = np.zeros(1 << n, dtype=np.complex128)
    out[basis(n, w)] = psi_s
    return out


def dicke(n, w):
    """eq. (initstate) in the sector: every amplitude C(n, w)^{-1/2}."""
    c = dim(n, w)
    return np.full(c, 1.0 / math.sqrt(c), dtype=np.complex128)


def _outside(v, n, w):
    z = np.arange(1 << n, dtype=np.uint64)
    return np.asarray(v)[np.bitwise_count(z) != w]


def apply_h(ham, t, psi_s, w, shift=0.0):
    """(H(t) - shift) psi in the sector; raises if H leaks out of it."""
    full = sqh.apply_h(ham, t, expand(psi_s, ham.n, w), shift)
    leak = _outside(full, ham.n, w)
    if leak.size and np.max(np.abs(leak)) > 1e-12 * max(1.0, np.max(np.abs(full))):
        raise ValueError("the Hamiltonian does not conserve the Hamming weight")
    return full[basis(ham.n, w)]


def evolve(ham, psi_s, w, t0, t1, n_steps, method="pc4", shift=0.0):
    """Fixed-step evolution of a sector state (integrate.evolve on the expanded state)."""
    y = integrate.evolve(ham, expand(psi_s, ham.n, w), t0, t1, n_steps, method, shift)
    return y[basis(ham.n, w)]


def energy(ham, t, psi_s, w):
    return observables.energy(ham, t, expand(psi_s, ham.n, w))


def ground_mass(ham, t, psi_s, w, rel_tol=1e-9):
    """Mass on the lowest-energy states of the sector under the diagonal of H(t):
    the sector's E_min and the states within rel_tol * max(1, |E_min|) of it."""
    d = sqh.diagonal(ham, t)[basis(ham.n, w)]
    e_min = float(np.min(d))
    sel = d <= e_min + rel_tol * max(1.0, abs(e_min))
    return float(np.sum(np.abs(np.asarray(psi_s)[sel]) ** 2)), e_min
