"""Oracle: the successful runtime T_s of Sec. III.B, by bracketing and bisection.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. III.B judges a runtime T by the final energy E(T) = <psi(T)|H_f|psi(T)>:
with a zero ground energy and every excited level at least 1, E(T) <= 1/2
means at least half of the population is in the ground state.  T_s is the
runtime at which E(T) falls to 1/2.  The paper does not say how the crossing is
located; this module takes the reading that the library documents:

  1. evaluate E at a first runtime T0;
  2. if E(T0) > 1/2, double T until E(T) <= 1/2 (give up above T_max);
     otherwise halve T until E(T) > 1/2;
  3. bisect the bracket [T_lo, T_hi] in log T (next runtime sqrt(T_lo T_hi))
     until T_hi / T_lo <= 1 + rel;
  4. report T_s = sqrt(T_lo T_hi).

It is written as plain loops, separately from the library's search, so that
the runtimes tried by the two can be compared one by one.  E(T) here is the
oracle's own evolution (``integrate.evolve``) followed by ``observables.energy``.
"""
from __future__ import annotations

import copy
import math

from . import integrate, observables


def on_runtime(inst, T):
    """The same instance on the path of duration T (only path["T"] changes)."""
    out = copy.copy(inst)
    out.path = dict(inst.path)
    out.path["T"] = float(T)
    return out


def successful_runtime(energy_of, T0, rel, T_max=math.inf):
    """Locate E(T) = 1/2 for a function energy_of(T) that decreases through 1/2.

    Returns (tried, T_lo, T_hi, T_s): tried is the list of (T, E(T)) in the
    order evaluated; E(T_lo) > 1/2 >= E(T_hi).  T_hi is inf (and T_s nan) when
    doubling passes T_max before E falls to 1/2."""
    tried = []

    def ev(T):
        e = float(energy_of(T))
        tried.append((T, e))
        return e

    T_lo, T_hi = 0.0, math.inf
    if ev(T0) > 0.5:
        T_lo = T0
        while True:
            T = 2.0 * T_lo
            if T > T_max:
                return tried, T_lo, math.inf, math.nan
            if ev(T) > 0.5:
                T_lo = T
            else:
                T_hi = T
                break
    else:
        T_hi = T0
        while True:
            T = 0.5 * T_hi
            if ev(T) > 0.5:
                T_lo = T
                break
            T_hi = T
    while T_hi / T_lo > 1.0 + rel:
        T = math.sqrt(T_lo * T_hi)
        if ev(T) > 0.5:
            T_lo = T
        else:
            T_hi = T
    return tried, T_lo, T_hi, math.sqrt(T_lo * T_hi)


def final_energy(inst, psi0, T, n_steps, method="pc4", shift=0.0):
    """E(T): evolve psi0 over [0, T] on the path of duration T with n_steps fixed
    steps, then <psi(T)|H(T)|psi(T)> (H(T) = H_f at the end of the path)."""
    it = on_runtime(inst, T)
    y = integrate.evolve(it, psi0, 0.0, T, n_steps, method, shift)
    return observables.energy(it, T, y)


def search_instance(inst, psi0, steps_and_shift, T0, rel, T_max=math.inf, method="pc4"):
    """T_s of one instance; steps_and_shift(T) -> (n_steps, shift) of the solve
    at runtime T."""
    def energy_of(T):
        K, shift = steps_and_shift(T)
        return final_energy(inst, psi0, T, K, method, shift)

    return successful_runtime(energy_of, T0, rel, T_max)
