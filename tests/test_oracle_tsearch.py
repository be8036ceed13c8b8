"""Pins of the oracle's T_s search (Sec. III.B: E(T_s) = 1/2, located by
doubling or halving to a bracket and bisecting in log T).

* E(T) = exp(-T/3) crosses 1/2 at T = 3 ln 2 exactly; the search must bracket
  that value to the relative width asked, from below (doubling) and from above
  (halving), and the bracket must stay a true bracket at every step.
* a step function E(T) = 1 for T < c, 0 otherwise has its crossing at c.
* the runtimes tried are the ones the procedure fixes: T0, 2 T0, 4 T0, ...
  until the first E <= 1/2, then geometric midpoints.
* doubling past T_max gives up with no T_s.
* a planted mistake (bisecting toward the wrong end) fails the first pin.

The library's own search (paper_1311_3938_amd.tsearch, host logic) is
checked here against the oracle on the same functions: same runtimes tried,
same T_s."""
import math

import pytest

from oracle import tsearch as OT

CROSS = 3.0 * math.log(2.0)


def _exp_energy(T):
    return math.exp(-T / 3.0)


@pytest.mark.parametrize("T0", [0.05, 1.0, 2.0, 50.0, 1000.0])
@pytest.mark.parametrize("rel", [0.2, 0.01, 1e-6])
def test_brackets_the_known_crossing(T0, rel):
    tried, lo, hi, ts = OT.successful_runtime(_exp_energy, T0, rel)
    assert lo < CROSS <= hi and hi / lo <= 1.0 + rel
    assert abs(math.log(ts / CROSS)) <= math.log(1.0 + rel)
    # every evaluation is the function itself, in order
    assert all(e == _exp_energy(T) for T, e in tried)


def test_runtimes_tried_follow_the_procedure():
    tried, lo, hi, ts = OT.successful_runtime(_exp_energy, 0.25, 0.1)
    Ts = [T for T, _ in tried]
    # doubling from 0.25: 0.25, 0.5, 1, 2, 4 (E(4) = 0.26 <= 1/2)
    assert Ts[:5] == [0.25, 0.5, 1.0, 2.0, 4.0]
    a, b = 2.0, 4.0
    for T in Ts[5:]:
        assert T == math.sqrt(a * b)
        if _exp_energy(T) > 0.5:
            a = T
        else:
            b = T
    assert (a, b) == (lo, hi) and b / a <= 1.1


def test_halving_from_a_long_runtime():
    tried, lo, hi, ts = OT.successful_runtime(_exp_energy, 64.0, 0.05)
    Ts = [T for T, _ in tried]
    assert Ts[:6] == [64.0, 32.0, 16.0, 8.0, 4.0, 2.0]
    assert lo < CROSS <= hi


@pytest.mark.parametrize("c", [0.7, 3.3, 17.0])
def test_step_function(c):
    tried, lo, hi, ts = OT.successful_runtime(lambda T: 1.0 if T < c else 0.0, 1.0, 1e-3)
    assert lo < c <= hi and hi / lo <= 1.001


def test_gives_up_past_t_max():
    tried, lo, hi, ts = OT.successful_runtime(lambda T: 1.0, 1.0, 0.1, T_max=100.0)
    assert [T for T, _ in tried] == [1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0]
    assert hi == math.inf and math.isnan(ts)


def test_planted_wrong_bisection_is_caught():
    def wrong(energy_of, T0, rel):
        lo, hi = 0.0, math.inf
        T = T0
        while energy_of(T) > 0.5:
            lo, T = T, 2 * T
        hi = T
        lo = lo or hi / 2
        while hi / lo > 1 + rel:
            T = math.sqrt(lo * hi)
            if energy_of(T) > 0.5:
                hi = T      # wrong end
            else:
                lo = T
        return lo, hi

    lo, hi = wrong(_exp_energy, 1.0, 0.01)
    assert not (lo < CROSS <= hi)


@pytest.mark.parametrize("T0,rel", [(0.25, 0.1), (64.0, 0.05), (2.0, 1e-3)])
def test_library_search_matches_oracle(T0, rel):
    from paper_1311_3938_amd.tsearch import Search
    tried, lo, hi, ts = OT.successful_runtime(_exp_energy, T0, rel)
    s = Search()
    while True:
        T = s.next_T(T0, rel)
        if T is None:
            break
        s.record(T, _exp_energy(T))
    assert s.evals == tried
    assert (s.T_lo, s.T_hi) == (lo, hi) and s.T_s == ts
