"""Oracle: the SQH Hamiltonian and its matrix-free product, written from Sec. II.A.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (Sec. II.A):
  * basis state |z> = |z_n> x ... x |z_1>, z = sum_i z_i 2^(i-1): qubit i is bit i-1
    of the integer index (eq. (ztensor));
  * |0> and |1> are the sigma^z eigenvectors with eigenvalues +1 and -1;
  * sigma^y = [[0, -i], [i, 0]] (the standard matrix; the paper names it only).

A Hamiltonian is H(t) = sum_terms m_l(t) * P_l with P_l a product of single-qubit
Pauli matrices (eq. (SQH-Hamiltonian)) and m_l(t) = w_l * f_{sid_l}(s(t)) a real
time-dependent coefficient (end of Sec. II.A).  The term's Pauli letters are read
from two masks: bit q-1 set in ``x`` only -> sigma^x on qubit q, in ``z`` only ->
sigma^z, in both -> sigma^y.

The product H|psi> follows the paper's recipe literally: every term acts on every
basis state |z> as a succession of single-qubit operations sigma^alpha |z_q>, which
maps |z> to a phase times another basis state; the results are summed.
"""
from __future__ import annotations

import math

import numpy as np

_ONE = np.uint64(1)


# ---------------------------------------------------------------------------
# Path and schedules (eq. (aqc), eq. (nlpath), time-dependent m_l(t))
# ---------------------------------------------------------------------------

def path_s(path, t):
    """Interpolation parameter s(t).  'linear': s = t/T (eq. (aqc));
    'sin2': s = sin^2(pi t / 2T) (a smooth nonlinear speed profile)."""
    T = path["T"]
    if path["kind"] == "linear":
        return t / T
    if path["kind"] == "sin2":
        return math.sin(math.pi * t / (2.0 * T)) ** 2
    raise ValueError(f"unknown path {path['kind']!r}")


def schedule_value(sched, t, path):
    """Scalar f(t) that multiplies a term's weight."""
    kind = sched["kind"]
    if kind == "const":
        return 1.0
    if kind == "poly_s":
        s = path_s(path, t)
        lo, hi = sched["s_lo"], sched["s_hi"]
        inside = (s >= lo) and ((s <= hi) if sched.get("hi_closed", False) else (s < hi))
        if not inside:
            return 0.0
        val = 0.0
        for d, c in enumerate(sched["coef"]):
            val += c * s ** d
        return val
    if kind == "trig_t":
        return sched["amp"] * math.cos(sched["omega"] * t + sched["phase"])
    if kind == "pwl_s":
        # linear interpolation in s between knots (s_i, v_i), constant outside;
        # the ramps of the clause-by-clause path, eq. (kpath)
        s = path_s(path, t)
        knots = sched["knots"]
        if s < knots[0][0]:
            return float(knots[0][1])
        for (a, va), (b, vb) in zip(knots[:-1], knots[1:]):
            if a <= s < b:
                return va + (vb - va) * (s - a) / (b - a)
        return float(knots[-1][1])
    raise ValueError(f"unknown schedule {kind!r}")


def coefficients(ham, t):
    """m_l(t) = w_l * f_{sid_l}(t) for every term (float64 array)."""
    f = [schedule_value(s, t, ham.path) for s in ham.scheds]
    return np.array([ham.w[l] * f[ham.sid[l]] for l in range(len(ham.w))], dtype=np.float64)


# ---------------------------------------------------------------------------
# One Pauli string on all basis states
# ---------------------------------------------------------------------------

def pauli_letters(n, x, z):
    """[(qubit, 'X'|'Y'|'Z'), ...] of the string encoded by the masks (x, z)."""
    out = []
    for q in range(1, n + 1):
        b = 1 << (q - 1)
        xb = bool(int(x) & b)
        zb = bool(int(z) & b)
        if xb and zb:
            out.append((q, "Y"))
        elif xb:
            out.append((q, "X"))
        elif zb:
            out.append((q, "Z"))
    return out


def pauli_on_basis(n, letters):
    """Image of every basis state under the string: P|z> = phase(z) |image(z)>.

    Each single-qubit factor acts on bit q-1 of z:
      sigma^x |0> = |1>,    sigma^x |1> = |0>
      sigma^y |0> = i|1>,   sigma^y |1> = -i|0>
      sigma^z |0> = |0>,    sigma^z |1> = -|1>
    Returns (image, phase) as arrays over z = 0 .. 2^n - 1.
    """
    N = 1 << n
    z = np.arange(N, dtype=np.uint64)
    image = z.copy()
    phase = np.ones(N, dtype=np.complex128)
    for q, a in letters:
        bit = np.uint64(q - 1)
        zq = (z >> bit) & _ONE            # the qubit's value in the *input* state
        if a == "X":
            image ^= (_ONE << bit)
        elif a == "Y":
            image ^= (_ONE << bit)
            phase *= np.where(zq == 0, 1j, -1j)
        elif a == "Z":
            phase *= np.where(zq == 0, 1.0, -1.0)
        else:
            raise ValueError(a)
    return image, phase


def apply_pauli(psi, n, x, z, coef=1.0):
    """coef * P|psi> with P the string (x, z):  sum_z psi_z coef phase(z) |image(z)>."""
    image, phase = pauli_on_basis(n, pauli_letters(n, x, z))
    out = np.zeros_like(psi, dtype=np.complex128)
    # image is a permutation of the basis, so a plain scatter is exact
    out[image.astype(np.int64)] = coef * phase * psi
    return out


def apply_h(ham, t, psi, shift=0.0):
    """(H(t) - shift) |psi>, H(t) = sum_l m_l(t) P_l (eq. (SQH-Hamiltonian))."""
    m = coefficients(ham, t)
    out = np.zeros(psi.shape, dtype=np.complex128)
    for l in range(len(m)):
        if m[l] == 0.0:
            continue
        out += apply_pauli(psi, ham.n, ham.x[l], ham.z[l], m[l])
    if shift != 0.0:
        out -= shift * psi
    return out


def diagonal(ham, t):
    """Diagonal of H(t) over all basis states: sum over the terms without a flip
    (x = 0) of m_l(t) times their sign on |z>."""
    N = 1 << ham.n
    m = coefficients(ham, t)
    d = np.zeros(N, dtype=np.float64)
    for l in range(len(m)):
        if int(ham.x[l]) != 0 or m[l] == 0.0:
            continue
        _, phase = pauli_on_basis(ham.n, pauli_letters(ham.n, 0, ham.z[l]))
        d += m[l] * phase.real
    return d


def is_diagonal_term(ham, l):
    return int(ham.x[l]) == 0


def apply_h_rows(ham, t, values_at, rows, shift=0.0):
    """Selected entries of (H(t) - shift)|psi> without forming the whole vector.

    ``values_at(idx)`` returns psi at the basis states ``idx`` (int64 array);
    ``rows`` are the output indices y.  Every term maps |z> to phase(z)|z ^ x>
    (the per-qubit rule of ``pauli_on_basis``), so entry y of P|psi> is
    phase(y ^ x) psi[y ^ x]."""
    rows = np.asarray(rows, dtype=np.uint64)
    m = coefficients(ham, t)
    out = np.zeros(rows.shape, dtype=np.complex128)
    for l in range(len(m)):
        if m[l] == 0.0:
            continue
        x = np.uint64(int(ham.x[l]))
        src = rows ^ x
        letters = pauli_letters(ham.n, ham.x[l], ham.z[l])
        if any(a == "Y" for _, a in letters):
            phase = np.ones(rows.shape, dtype=np.complex128)
            for q, a in letters:
                bit = np.uint64(q - 1)
                zq = (src >> bit) & _ONE
                if a == "Y":
                    phase *= np.where(zq == 0, 1j, -1j)
                elif a == "Z":
                    phase *= np.where(zq == 0, 1.0, -1.0)
            out += m[l] * phase * values_at(src.astype(np.int64))
        elif any(a == "Z" for _, a in letters):
            # X and Z letters only: the phase is a real sign
            sign = np.ones(rows.shape, dtype=np.float64)
            for q, a in letters:
                if a == "Z":
                    sign *= np.where(((src >> np.uint64(q - 1)) & _ONE) == 0, 1.0, -1.0)
            out += (m[l] * sign) * values_at(src.astype(np.int64))
        else:
            # X letters only: phase 1
            out += m[l] * values_at(src.astype(np.int64))
    if shift != 0.0:
        out -= shift * values_at(rows.astype(np.int64))
    return out


def apply_h_parallel(ham, t, psi, shift=0.0, threads=None, block=1 << 18):
    """(H(t) - shift)|psi> for large states: the rows are split into blocks and
    each block is ``apply_h_rows`` (the same per-term, per-qubit rule, terms
    summed in the same order), computed on host threads.  Every entry is the
    same value as in ``apply_h`` (the product m_l * phase * psi, summed term by
    term in the same order; a real sign multiplies as a real number), so the
    results agree; only the rows are shared out."""
    from concurrent.futures import ThreadPoolExecutor
    import os

    psi = np.asarray(psi, dtype=np.complex128)
    N = psi.shape[0]
    if threads is None:
        threads = max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
    out = np.empty(N, dtype=np.complex128)

    def values_at(idx):
        return psi[idx]

    def work(r0):
        rows = np.arange(r0, min(N, r0 + block), dtype=np.uint64)
        out[r0:r0 + rows.shape[0]] = apply_h_rows(ham, t, values_at, rows, shift)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, range(0, N, block)))
    return out


def diagonal_rows(ham, t, rows):
    """Entries of the diagonal of H(t) at the basis states ``rows``."""
    rows = np.asarray(rows, dtype=np.uint64)
    m = coefficients(ham, t)
    d = np.zeros(rows.shape, dtype=np.float64)
    for l in range(len(m)):
        if int(ham.x[l]) != 0 or m[l] == 0.0:
            continue
        sign = np.ones(rows.shape)
        for q, a in pauli_letters(ham.n, 0, ham.z[l]):
            sign *= np.where(((rows >> np.uint64(q - 1)) & _ONE) == 0, 1.0, -1.0)
        d += m[l] * sign
    return d
