"""Pins of the hard-instance generator (Sec. II.D) and of the T_s bracket
logic (Sec. III.B): a unique satisfying assignment, n_ij in {0, 1}, one
connected clause graph; the search brackets and bisects a known crossing."""
import math

import numpy as np
import pytest

from oracle import sqh
from paper_1311_3938_amd import instances as I


@pytest.mark.parametrize("n,seed", [(7, 0), (8, 1), (11, 2), (14, 3)])
def test_usa_instance_has_one_solution(n, seed):
    clauses, sol = I.usa_hard_instance(n, np.random.default_rng(seed))
    assert len(set(clauses)) == len(clauses) <= n
    assert all(len(set(c)) == 3 and all(1 <= q <= n for q in c) for c in clauses)
    # the oracle's H_f: exactly one zero-energy state, the returned solution
    inst = I.ec3_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    d = sqh.diagonal(inst, 0.0)
    assert np.count_nonzero(d == 0.0) == 1 and d[sol] == 0.0
    # clauses share bits but no pair of bits, and connect every bit
    assert set(I.clause_pair_counts(clauses).values()) == {1}
    assert I.clause_graph_components(n, clauses) == 1


def test_usa_workloads_share_the_instance():
    a = I.workload_usa(9, 2, "x")
    b = I.workload_usa(9, 2, "xy")
    assert a.meta["clauses"] == b.meta["clauses"] and a.meta["solution"] == b.meta["solution"]
    assert a.meta["weight"] == bin(a.meta["solution"]).count("1")


def test_ts_bracket_logic():
    """E(T) = exp(-T / 3): the crossing is at T = 3 ln 2."""
    from paper_1311_3938_amd.tsearch import Search
    s = Search()
    while True:
        T = s.next_T(1.0, 0.01)
        if T is None:
            break
        s.record(T, math.exp(-T / 3.0))
    assert s.T_lo < 3 * math.log(2) <= s.T_hi and s.T_hi / s.T_lo <= 1.01
    assert s.T_s == pytest.approx(3 * math.log(2), rel=0.01)
    # a start above the crossing halves down first
    s = Search()
    for _ in range(40):
        T = s.next_T(50.0, 0.05)
        if T is None:
            break
        s.record(T, math.exp(-T / 3.0))
    assert s.T_lo < 3 * math.log(2) <= s.T_hi
