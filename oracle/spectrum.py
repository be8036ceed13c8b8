"""Oracle: the lowest eigenvalues of H(t) and the gap above the ground state
(Sec. IV.B: the lower spectrum along each path and the gap between the two
lowest levels, which the paper computes with ARPACK).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

  * ``lowest_dense``    the k smallest eigenvalues of the dense H(t) built from
                        the matrix-free product on the unit vectors (small n);
  * ``lowest``          the k smallest eigenvalues through ARPACK (scipy's
                        eigsh on a LinearOperator wrapping sqh.apply_h), the
                        same route as the paper's; optionally restricted to a
                        Hamming-weight sector (``subspace.apply_h``);
  * ``gap``             E_1 - E_0.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigsh

from . import sqh, subspace


def _matvec(ham, t, weight):
    if weight is None:
        return (1 << ham.n), (lambda v: sqh.apply_h(ham, t, np.asarray(v, dtype=np.complex128).ravel()))
    dim = subspace.dim(ham.n, weight)
    return dim, (lambda v: subspace.apply_h(ham, t, np.asarray(v, dtype=np.complex128).ravel(), weight))


def lowest_dense(ham, t, k=2, weight=None):
    dim, mv = _matvec(ham, t, weight)
    H = np.array([mv(e) for e in np.eye(dim, dtype=np.complex128)]).T
    return np.linalg.eigvalsh(0.5 * (H + H.conj().T))[:k]


def lowest(ham, t, k=2, weight=None, tol=1e-12, seed=0, dense_max=1024):
    """Dense up to dense_max states (exact with degenerate levels, e.g. a
    diagonal H_f with several solutions, where a single Krylov sequence sees
    one copy of each level), ARPACK above."""
    dim, mv = _matvec(ham, t, weight)
    if dim <= dense_max:
        return lowest_dense(ham, t, k, weight)
    op = LinearOperator((dim, dim), matvec=mv, dtype=np.complex128)
    v0 = np.random.default_rng(seed).normal(size=dim) + 0j
    vals = eigsh(op, k=k, which="SA", tol=tol, v0=v0, return_eigenvectors=False)
    return np.sort(np.real(vals))


def gap(ham, t, weight=None):
    e = lowest(ham, t, 2, weight)
    return float(e[1] - e[0])
