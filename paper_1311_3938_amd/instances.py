"""Seeded synthetic problem instances: the inputs shared by the library and the oracle.

This module only *describes* Hamiltonians and initial states as plain arrays; it
contains no part of the time-stepping method.  A Hamiltonian is a list of
Pauli-string terms in the compact qubit ("SQH") form of Sec. II.A,
eq. (SQH-Hamiltonian): each term is a real weight times a product of single-qubit
Pauli matrices, with a path-dependent scalar schedule that multiplies the weight
(time-dependent coefficients, end of Sec. II.A).

Encoding of one term (used by both sides):
  * ``x`` bit q-1 set  <=> qubit q carries sigma^x or sigma^y,
  * ``z`` bit q-1 set  <=> qubit q carries sigma^z or sigma^y,
  so sigma^y on qubit q sets the bit in both masks.  Qubit q is bit q-1 of the
  basis index (Sec. II.A, eq. (ztensor)).
  * ``w`` real weight, ``sid`` index of the schedule that multiplies it.

Schedules (functions of the path parameter s(t) or of t):
  * ``{"kind": "const"}``                                  f = 1
  * ``{"kind": "poly_s", "coef": [c0, c1, ...],
       "s_lo": a, "s_hi": b, "hi_closed": bool}``          f = sum_d c_d s^d on
    a <= s < b (or s <= b when ``hi_closed``), 0 outside
  * ``{"kind": "trig_t", "amp": A, "omega": w, "phase": p}``  f = A cos(w t + p)
Paths: ``{"kind": "linear", "T": T}`` gives s = t/T (eq. (aqc));
``{"kind": "sin2", "T": T}`` gives s = sin^2(pi t / 2T).

Random numbers: every generator takes a ``numpy.random.Generator``; the benchmark
workloads seed it as ``default_rng(10_000 * config + instance)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

INF = float("inf")

SCHED_CONST = {"kind": "const"}


def poly_s(coef, s_lo=-INF, s_hi=INF, hi_closed=False):
    return {"kind": "poly_s", "coef": [float(c) for c in coef], "s_lo": float(s_lo),
            "s_hi": float(s_hi), "hi_closed": bool(hi_closed)}


def pwl_s(knots):
    """Piecewise-linear schedule in s through up to 4 knots (s_i, v_i), s_i
    nondecreasing; v_0 below the first knot, the last value from the last on."""
    knots = [(float(a), float(v)) for a, v in knots]
    if not 1 <= len(knots) <= 4 or any(b[0] < a[0] for a, b in zip(knots, knots[1:])):
        raise ValueError("pwl_s: 1..4 knots with nondecreasing s")
    return {"kind": "pwl_s", "knots": knots}


def trig_t(amp, omega, phase=0.0):
    return {"kind": "trig_t", "amp": float(amp), "omega": float(omega), "phase": float(phase)}


# The three schedules of the interpolated path H(s) = (1-s) H_i + s H_f + s(1-s) H_c
# (eq. (aqc) and eq. (nlpath)).
SCHED_ONE_MINUS_S = poly_s([1.0, -1.0])
SCHED_S = poly_s([0.0, 1.0])
SCHED_S_ONE_MINUS_S = poly_s([0.0, 1.0, -1.0])


def linear_path(T):
    return {"kind": "linear", "T": float(T)}


def sin2_path(T):
    return {"kind": "sin2", "T": float(T)}


@dataclass
class Instance:
    """A time-dependent Hamiltonian in term form plus the data it was drawn from."""

    n: int
    x: np.ndarray
    z: np.ndarray
    w: np.ndarray
    sid: np.ndarray
    scheds: list
    path: dict
    meta: dict = field(default_factory=dict)

    @property
    def n_terms(self):
        return int(self.w.shape[0])


def pauli_masks(n, ops):
    """Masks of one Pauli string given as ``{qubit (1-based): 'X'|'Y'|'Z'}``."""
    x = 0
    z = 0
    for q, a in ops.items():
        if not 1 <= q <= n:
            raise ValueError(f"qubit {q} outside 1..{n}")
        b = 1 << (q - 1)
        a = a.upper()
        if a == "X":
            x |= b
        elif a == "Z":
            z |= b
        elif a == "Y":
            x |= b
            z |= b
        elif a != "I":
            raise ValueError(f"unknown Pauli {a!r}")
    return x, z


class TermList:
    """Accumulates (x, z, weight, schedule) terms."""

    def __init__(self, n):
        self.n = n
        self.x, self.z, self.w, self.sid = [], [], [], []

    def add(self, ops, w, sid):
        x, z = pauli_masks(self.n, ops)
        self.x.append(x)
        self.z.append(z)
        self.w.append(float(w))
        self.sid.append(int(sid))

    def add_masks(self, x, z, w, sid):
        self.x.append(int(x))
        self.z.append(int(z))
        self.w.append(float(w))
        self.sid.append(int(sid))

    def extend(self, other: "TermList", sid=None):
        for x, z, w, s in zip(other.x, other.z, other.w, other.sid):
            self.add_masks(x, z, w, s if sid is None else sid)

    def instance(self, scheds, path, meta=None):
        return Instance(
            n=self.n,
            x=np.array(self.x, dtype=np.uint64),
            z=np.array(self.z, dtype=np.uint64),
            w=np.array(self.w, dtype=np.float64),
            sid=np.array(self.sid, dtype=np.int32),
            scheds=list(scheds),
            path=dict(path),
            meta=dict(meta or {}),
        )


# ---------------------------------------------------------------------------
# Problem Hamiltonians
# ---------------------------------------------------------------------------

def ec3_random_clauses(n, m, rng):
    """m different clauses, each over 3 different bits drawn uniformly (eq. (1clause)).

    Clauses are sorted triples of 1-based qubit labels; a duplicate clause is
    redrawn, so all m are different (Sec. II.C requires distinct clauses).
    """
    if n < 3:
        raise ValueError("EC3 needs n >= 3")
    max_m = n * (n - 1) * (n - 2) // 6
    if m > max_m:
        raise ValueError("more clauses than distinct triples")
    seen = set()
    out = []
    while len(out) < m:
        c = tuple(sorted(int(q) + 1 for q in rng.choice(n, 3, replace=False)))
        if c in seen:
            continue
        seen.add(c)
        out.append(c)
    return out


def _clause_ok_mask(n, clause, z):
    """Assignments (int array z) in which exactly one bit of the clause is 1."""
    a, b, c = (int(q) - 1 for q in clause)
    return (((z >> a) & 1) + ((z >> b) & 1) + ((z >> c) & 1)) == 1


def usa_hard_instance(n, rng, m_max=None, max_restarts=1000):
    """A random hard EC3 instance with a unique satisfying assignment, by the
    recipe of Sec. II.D: from the pool of all clauses, a random first clause
    starts a graph; clauses that touch the graph and share no pair of bits
    with it (so n_ij is 0 or 1) are added at random; once every bit is in the
    graph, a clause that would leave no solution is discarded, and the
    instance is done when exactly one solution is left.  The search restarts
    when the pool is empty or m_max clauses are reached.  Returns (clauses,
    solution).  Solutions are counted over all 2^n assignments (n <= 26);
    below n = 7 such instances are rare, and the search gives up with an error."""
    if not 3 <= n <= 26:
        raise ValueError("usa_hard_instance: 3 <= n <= 26")
    m_max = n if m_max is None else int(m_max)
    triples = [tuple(int(q) + 1 for q in t) for t in
               np.array([(a, b, c) for a in range(n) for b in range(a + 1, n) for c in range(b + 1, n)])]
    z = np.arange(1 << n, dtype=np.int64)
    for _ in range(max_restarts):
        pool = list(triples)
        first = pool.pop(int(rng.integers(len(pool))))
        clauses = [first]
        covered = set(first)
        edges = {(first[0], first[1]), (first[0], first[2]), (first[1], first[2])}
        ok = _clause_ok_mask(n, first, z)
        while pool and len(clauses) < m_max:
            # drop clauses that share a pair of bits with the graph
            pool = [c for c in pool if not ({(c[0], c[1]), (c[0], c[2]), (c[1], c[2])} & edges)]
            touching = [i for i, c in enumerate(pool) if covered & set(c)]
            if not touching:
                break
            c = pool.pop(touching[int(rng.integers(len(touching)))])
            new_ok = ok & _clause_ok_mask(n, c, z)
            if len(covered | set(c)) == n and not new_ok.any():
                continue                       # would leave no solution: discard
            clauses.append(c)
            covered |= set(c)
            edges |= {(c[0], c[1]), (c[0], c[2]), (c[1], c[2])}
            ok = new_ok
            if len(covered) == n and int(ok.sum()) == 1:
                return clauses, int(np.flatnonzero(ok)[0])
    raise RuntimeError("usa_hard_instance: no instance found")


def ec3_terms(n, clauses, omega=1.0):
    """Final Hamiltonian of EC3 in the expanded form of eq. (final_ham).

    H_f = Omega m 1 - Omega sum_i (n_i/2) sigma^z_i + Omega sum_{i<j} (n_ij/2) sigma^z_i sigma^z_j,
    n_i = number of clauses containing bit i, n_ij = number containing both i and j.
    """
    ni = {}
    nij = {}
    for c in clauses:
        for a in c:
            ni[a] = ni.get(a, 0) + 1
        for i in range(3):
            for j in range(i + 1, 3):
                p = (min(c[i], c[j]), max(c[i], c[j]))
                nij[p] = nij.get(p, 0) + 1
    t = TermList(n)
    t.add({}, omega * len(clauses), 0)
    for i in sorted(ni):
        t.add({i: "Z"}, -omega * ni[i] / 2.0, 0)
    for (i, j) in sorted(nij):
        t.add({i: "Z", j: "Z"}, omega * nij[(i, j)] / 2.0, 0)
    return t


def sk_couplings(n, rng):
    """Sherrington-Kirkpatrick couplings: J_ij ~ N(0, 1/n), h_i ~ N(0, 0.1) (variances)."""
    J = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            J[i, j] = rng.normal(0.0, math.sqrt(1.0 / n))
    h = rng.normal(0.0, math.sqrt(0.1), size=n)
    return J, h


def sk_terms(n, J, h):
    """H_f = sum_{i<j} J_ij sigma^z_i sigma^z_j + sum_i h_i sigma^z_i."""
    t = TermList(n)
    for i in range(n):
        for j in range(i + 1, n):
            t.add({i + 1: "Z", j + 1: "Z"}, J[i, j], 0)
    for i in range(n):
        t.add({i + 1: "Z"}, h[i], 0)
    return t


def transverse_terms(n, weights=None, omega=1.0):
    """H^x = Omega sum_i (w_i/2)(1 - sigma^x_i) (eq. (Hix)); unit weights by default."""
    if weights is None:
        weights = [1.0] * n
    t = TermList(n)
    t.add({}, omega * sum(weights) / 2.0, 0)
    for i in range(n):
        t.add({i + 1: "X"}, -omega * weights[i] / 2.0, 0)
    return t


def xx_catalyst(n, n_pairs, rng):
    """sum over distinct random pairs of g sigma^x_i sigma^x_j with g ~ N(0, 1)."""
    max_pairs = n * (n - 1) // 2
    n_pairs = min(n_pairs, max_pairs)
    seen = set()
    pairs = []
    while len(pairs) < n_pairs:
        i, j = sorted(int(q) + 1 for q in rng.choice(n, 2, replace=False))
        if (i, j) in seen:
            continue
        seen.add((i, j))
        pairs.append((i, j))
    g = rng.normal(0.0, 1.0, size=len(pairs))
    t = TermList(n)
    for (i, j), gij in zip(pairs, g):
        t.add({i: "X", j: "X"}, gij, 0)
    return t, pairs, g


def xy_initial_terms(n, clauses, omega=1.0):
    """H^xy = 3 m Omega 1 - Omega sum_{i<j} (n_ij/2)(sigma^x_i sigma^x_j + sigma^y_i sigma^y_j)
    (eq. (Hixy))."""
    nij = clause_pair_counts(clauses)
    t = TermList(n)
    t.add({}, 3.0 * len(clauses) * omega, 0)
    for (i, j) in sorted(nij):
        t.add({i: "X", j: "X"}, -omega * nij[(i, j)] / 2.0, 0)
        t.add({i: "Y", j: "Y"}, -omega * nij[(i, j)] / 2.0, 0)
    return t


def xyz_initial_terms(n, clauses, omega=1.0):
    """H^xyz = Omega sum_{i<j} (n_ij/2)(1 - sigma_i . sigma_j), the Heisenberg
    ferromagnet on the clause graph (eq. (Hixyz))."""
    nij = clause_pair_counts(clauses)
    t = TermList(n)
    t.add({}, omega * sum(nij.values()) / 2.0, 0)
    for (i, j) in sorted(nij):
        for a in "XYZ":
            t.add({i: a, j: a}, -omega * nij[(i, j)] / 2.0, 0)
    return t


def clause_pair_counts(clauses):
    """n_ij: the number of clauses that contain both bits i < j."""
    nij = {}
    for c in clauses:
        for a in range(3):
            for b in range(a + 1, 3):
                p = (min(c[a], c[b]), max(c[a], c[b]))
                nij[p] = nij.get(p, 0) + 1
    return nij


def tfim_terms(n, omega=1.0):
    """Transverse-field Ising chain of eq. (ising) split into its two schedule parts:
    returns (-Omega sum sigma^x, -Omega sum sigma^z_i sigma^z_{i+1}) with periodic boundary."""
    tx = TermList(n)
    tz = TermList(n)
    for i in range(1, n + 1):
        tx.add({i: "X"}, -omega, 0)
    for i in range(1, n + 1):
        j = i % n + 1
        if n == 1:
            continue  # sigma^z_1 sigma^z_1 is the identity: no bond
        tz.add({i: "Z", j: "Z"}, -omega, 0)
    return tx, tz


def interpolated(n, h_i: TermList, h_f: TermList, path, h_c: TermList | None = None, meta=None):
    """H(s) = (1 - s) H_i + s H_f [+ s (1 - s) H_c]: eq. (aqc), eq. (nlpath)."""
    t = TermList(n)
    t.extend(h_i, sid=0)
    t.extend(h_f, sid=1)
    scheds = [SCHED_ONE_MINUS_S, SCHED_S]
    if h_c is not None:
        t.extend(h_c, sid=2)
        scheds.append(SCHED_S_ONE_MINUS_S)
    return t.instance(scheds, path, meta)


def clause_ramp(c, m):
    """The weight of clause c (1-based) of m in H_d(s) of eq. (kpath), as a
    function of s: 0 until s = (c-1)/m, rising to 1 at c/m (the secondary
    interpolation s_c = m s - c + 1 that switches it on), 1 until (m-1)/m, then
    falling to 0 at s = 1 (the last window's (1 - s_m) H_{m-1}, since H_m = 0).
    Windows are half open, so at a joint s = k/m only one window counts; the
    ramp is continuous there.  Clause m never enters H_d."""
    if not 1 <= c < m:
        raise ValueError("clause_ramp: 1 <= c < m")
    return pwl_s([((c - 1) / m, 0.0), (c / m, 1.0), ((m - 1) / m, 1.0), (1.0, 0.0)])


def clause_by_clause(n, clauses, path, h_i=None, omega=1.0, meta=None):
    """H(s) = (1 - s) H_i + s H_f + H_d(s), eq. (cbc)-(kpath): the clauses are
    switched on one after the other in stored order; H_i defaults to H^xy."""
    m = len(clauses)
    if m + 1 > 32:
        raise ValueError("clause_by_clause: at most 31 clauses (one schedule each)")
    t = TermList(n)
    t.extend(h_i if h_i is not None else xy_initial_terms(n, clauses, omega), sid=0)
    t.extend(ec3_terms(n, clauses, omega), sid=1)
    scheds = [SCHED_ONE_MINUS_S, SCHED_S]
    for c in range(1, m):
        t.extend(ec3_terms(n, [clauses[c - 1]], omega), sid=len(scheds))
        scheds.append(clause_ramp(c, m))
    return t.instance(scheds, path, meta)


def clause_graph_components(n, clauses):
    """Connected components of the graph on bits 1..n whose edges join bits
    that share a clause."""
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for c in clauses:
        for q in c[1:]:
            ra, rb = find(c[0]), find(q)
            if ra != rb:
                parent[ra] = rb
    return len({find(q) for q in range(1, n + 1)})


def removable_clause(n, clauses):
    """Index of the first clause (stored order) whose removal leaves the clause
    graph as connected as before (Sec. IV.A.1 removes only such clauses)."""
    base = clause_graph_components(n, clauses)
    for k in range(len(clauses)):
        if clause_graph_components(n, clauses[:k] + clauses[k + 1:]) == base:
            return k
    raise ValueError("no clause can be removed without splitting the clause graph")


def nonlinear_path(n, clauses, path, alpha=8.0, removed=None, h_i=None, omega=1.0, meta=None):
    """H(s) = (1 - s) H_i + s H_f + alpha s (1 - s) H_{m-1}, eq. (nlpath), with
    H_{m-1} = H_f without one clause (removable_clause by default); H_i
    defaults to H^xy."""
    k = removable_clause(n, clauses) if removed is None else int(removed)
    reduced = clauses[:k] + clauses[k + 1:]
    t = TermList(n)
    t.extend(h_i if h_i is not None else xy_initial_terms(n, clauses, omega), sid=0)
    t.extend(ec3_terms(n, clauses, omega), sid=1)
    t.extend(ec3_terms(n, reduced, omega), sid=2)
    meta = dict(meta or {})
    meta["removed"] = k
    return t.instance([SCHED_ONE_MINUS_S, SCHED_S, poly_s([0.0, alpha, -alpha])], path, meta)


def random_terms(n, k, rng, max_weight_ops=None, n_sched=1):
    """k random Pauli strings with N(0,1) weights and random schedule ids (test input)."""
    t = TermList(n)
    for _ in range(k):
        ops = {}
        nops = int(rng.integers(0, n + 1)) if max_weight_ops is None else int(
            rng.integers(0, min(n, max_weight_ops) + 1))
        qs = rng.choice(n, nops, replace=False) if nops else []
        for q in qs:
            ops[int(q) + 1] = "XYZ"[int(rng.integers(0, 3))]
        t.add(ops, rng.normal(), int(rng.integers(0, n_sched)))
    return t


# ---------------------------------------------------------------------------
# Initial states
# ---------------------------------------------------------------------------

def plus_state(n, dtype=np.complex128):
    """|+>^n = 2^{-n/2} sum_z |z>, the ground state of H^x (Sec. III.A.1)."""
    N = 1 << n
    return np.full(N, 1.0 / math.sqrt(N), dtype=dtype)


def random_state(n, rng, dtype=np.complex128):
    N = 1 << n
    v = rng.normal(size=N) + 1j * rng.normal(size=N)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


def dicke_state(n, weight, dtype=np.complex128):
    """Balanced superposition of all basis states of Hamming weight `weight` (eq. (initstate))."""
    N = 1 << n
    idx = np.arange(N, dtype=np.uint64)
    sel = np.bitwise_count(idx) == weight
    v = np.zeros(N, dtype=dtype)
    v[sel] = 1.0 / math.sqrt(math.comb(n, weight))
    return v


# ---------------------------------------------------------------------------
# Benchmark workloads (sizes and distributions of the paper's AQC runs)
# ---------------------------------------------------------------------------

def seed_for(config, instance=0):
    return 10_000 * config + instance


def workload_ec3_linear(n=12, m=10, T=20.0, seed=seed_for(0)):
    """n-bit random EC3 with m clauses, H_i = sum (1 - sigma^x)/2, linear path, s = t/T."""
    rng = np.random.default_rng(seed)
    clauses = ec3_random_clauses(n, m, rng)
    inst = interpolated(n, transverse_terms(n), ec3_terms(n, clauses), linear_path(T),
                        meta={"kind": "ec3", "clauses": clauses, "T": T, "seed": seed})
    return inst


def workload_ec3_catalyst(n=24, m=20, n_pairs=24, T=50.0, seed=seed_for(1)):
    """EC3 with an XX catalyst: H(s) = (1-s) H_i + s H_f + s(1-s) H_c."""
    rng = np.random.default_rng(seed)
    clauses = ec3_random_clauses(n, m, rng)
    cat, pairs, g = xx_catalyst(n, n_pairs, rng)
    inst = interpolated(n, transverse_terms(n), ec3_terms(n, clauses), linear_path(T), h_c=cat,
                        meta={"kind": "ec3+xx", "clauses": clauses, "pairs": pairs,
                              "g": g.tolist(), "T": T, "seed": seed})
    return inst


def workload_sk_sin2(n=30, T=30.0, seed=seed_for(2)):
    """Sherrington-Kirkpatrick H_f, transverse field H_i, s(t) = sin^2(pi t / 2T)."""
    rng = np.random.default_rng(seed)
    J, h = sk_couplings(n, rng)
    inst = interpolated(n, transverse_terms(n), sk_terms(n, J, h), sin2_path(T),
                        meta={"kind": "sk", "T": T, "seed": seed})
    return inst


def workload_ec3_paths(n=13, m=10, T=20.0, kind="cbc", seed=seed_for(5)):
    """The paths of Sec. IV.A between H^xy and an EC3 H_f: "linear" (eq. (aqc)),
    "nonlinear" (eq. (nlpath), alpha = 8) or "cbc" (eq. (cbc)-(kpath)); s = t/T.
    The same seed gives the same clauses for every kind."""
    rng = np.random.default_rng(seed)
    clauses = ec3_random_clauses(n, m, rng)
    meta = {"kind": "ec3-" + kind, "clauses": clauses, "T": T, "seed": seed}
    path = linear_path(T)
    if kind == "linear":
        return interpolated(n, xy_initial_terms(n, clauses), ec3_terms(n, clauses), path, meta=meta)
    if kind == "nonlinear":
        return nonlinear_path(n, clauses, path, meta=meta)
    if kind == "cbc":
        return clause_by_clause(n, clauses, path, meta=meta)
    raise ValueError(kind)


def workload_usa(n, i, algorithm="xy", T=1.0, config=6):
    """Hard instance i of size n (usa_hard_instance) with the straight-line
    path from the initial Hamiltonian of one algorithm of Sec. III.A: "x"
    (eq. (Hix), weights n_i/2), "xyz" (eq. (Hixyz)) or "xy" (eq. (Hixy)).
    meta holds the clauses, the solution and its Hamming weight."""
    rng = np.random.default_rng(seed_for(config, 1000 * n + i))
    clauses, sol = usa_hard_instance(n, rng)
    if algorithm == "x":
        ni = [sum(q in c for c in clauses) for q in range(1, n + 1)]
        hi = transverse_terms(n, weights=ni)
    elif algorithm == "xyz":
        hi = xyz_initial_terms(n, clauses)
    elif algorithm == "xy":
        hi = xy_initial_terms(n, clauses)
    else:
        raise ValueError(algorithm)
    return interpolated(n, hi, ec3_terms(n, clauses), linear_path(T),
                        meta={"kind": "usa-" + algorithm, "clauses": clauses, "solution": sol,
                              "weight": bin(sol).count("1"), "n": n, "i": i})


def workload_batch_member(i, n_lo=14, n_hi=22, config=3):
    """One member of the mixed batch: n uniform in [n_lo, n_hi], EC3 (m = round(0.8 n))
    or SK, n random XX catalyst pairs, T uniform in [10, 100], linear path."""
    rng = np.random.default_rng(seed_for(config, i))
    n = int(rng.integers(n_lo, n_hi + 1))
    T = float(rng.uniform(10.0, 100.0))
    if i % 2 == 0:
        clauses = ec3_random_clauses(n, int(round(0.8 * n)), rng)
        hf = ec3_terms(n, clauses)
        kind = "ec3"
    else:
        J, h = sk_couplings(n, rng)
        hf = sk_terms(n, J, h)
        kind = "sk"
    cat, _, _ = xx_catalyst(n, n, rng)
    return interpolated(n, transverse_terms(n), hf, linear_path(T), h_c=cat,
                        meta={"kind": kind, "T": T, "seed": seed_for(config, i)})


def workload_serving_request(i, n_lo=12, n_hi=28, config=4):
    """One serving request: n in [n_lo, n_hi] with P(n) ~ 2^{-(n - n_lo)/2}, EC3 or SK,
    linear or catalysed path, T uniform in [10, 100]."""
    rng = np.random.default_rng(seed_for(config, i))
    ns = np.arange(n_lo, n_hi + 1)
    p = 2.0 ** (-(ns - n_lo) / 2.0)
    n = int(rng.choice(ns, p=p / p.sum()))
    T = float(rng.uniform(10.0, 100.0))
    if rng.random() < 0.5:
        clauses = ec3_random_clauses(n, int(round(0.8 * n)), rng)
        hf = ec3_terms(n, clauses)
        kind = "ec3"
    else:
        J, h = sk_couplings(n, rng)
        hf = sk_terms(n, J, h)
        kind = "sk"
    cat = None
    if rng.random() < 0.5:
        cat, _, _ = xx_catalyst(n, n, rng)
    return interpolated(n, transverse_terms(n), hf, linear_path(T), h_c=cat,
                        meta={"kind": kind, "T": T, "seed": seed_for(config, i),
                              "catalyst": cat is not None})
