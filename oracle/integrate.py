"""Oracle: time stepping of i d|psi>/dt = H(t)|psi> (eq. (schroedinger), hbar = 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. II.B integrates the N coupled ODEs with a fourth-order predictor-corrector
that needs a single evaluation of H|psi> per step.  The paper does not write the
scheme out; the reading used here (and by the library) is:

  * ``pc4``: 4-step Adams-Bashforth predictor, 3-step Adams-Moulton corrector, in
    "PEC" mode: the one evaluation per step is made at the predicted point and is
    kept as the history value f_{k+1}.  On a uniform grid t_k = t_s + k h:
        y^p_{k+1} = y_k + h/24 (55 f_k - 59 f_{k-1} + 37 f_{k-2} - 9 f_{k-3})
        f_{k+1}   = f(t_{k+1}, y^p_{k+1})
        y_{k+1}   = y_k + h/24 (9 f_{k+1} + 19 f_k - 5 f_{k-1} + f_{k-2})
    with f(t, y) = -i (H(t) - c) y.  The first three steps of every segment are
    classical RK4 steps, which also supply f_0 .. f_3.
  * ``rk4``: the classical 4-stage Runge-Kutta method (also the bootstrap).
  * a constant spectral shift c may be subtracted from H; the exact solution only
    changes by the global phase exp(-i c (t1 - t0)), which is multiplied back in
    at the end.  Both methods are exact for c but their discretisation error is
    not shift-invariant, so the shift is an explicit input.
  * adaptive stepping (the paper is silent): Milne's device estimates the
    corrector's local error as (19/270) ||y_{k+1} - y^p_{k+1}||_2.  Steps are
    taken in windows of W steps; after each window the largest estimate decides:
    above ``atol`` the window is undone and the segment restarts from the
    window's first state with h/2; below atol/64 (after at least two windows at
    this h) the next segment starts with 2h.  An atol below the rounding floor
    of the estimate is refused (the estimate of a tiny step is pure rounding,
    or exactly zero, and the controller would creep along at that step).  The step is never halved below
    max(hmin, 1e-12 (t1 - t0)) and at most 60 windows in a row are undone: an
    estimate that stays above atol ends the run with an error.  Every restart re-runs the RK4
    bootstrap, since the multistep history needs equal spacing.  The last
    segment is shortened to end exactly at t1.
"""
from __future__ import annotations

import math

import numpy as np

from .sqh import apply_h

# Adams-Bashforth (4-step) and Adams-Moulton (3-step) weights, in units of h/24
AB4 = (55.0, -59.0, 37.0, -9.0)
AM4 = (9.0, 19.0, -5.0, 1.0)
MILNE = 19.0 / 270.0


def rhs(ham, t, y, shift=0.0, apply=apply_h):
    """f(t, y) = -i (H(t) - shift) y.  ``apply`` computes (H(t) - shift) y:
    sqh.apply_h, or sqh.apply_h_parallel (identical values) for large states."""
    return -1j * apply(ham, t, y, shift)


def rk4_step(ham, t, y, h, shift=0.0, k1=None, apply=apply_h):
    if k1 is None:
        k1 = rhs(ham, t, y, shift, apply)
    k2 = rhs(ham, t + 0.5 * h, y + (0.5 * h) * k1, shift, apply)
    k3 = rhs(ham, t + 0.5 * h, y + (0.5 * h) * k2, shift, apply)
    k4 = rhs(ham, t + h, y + h * k3, shift, apply)
    return y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


class Counter:
    def __init__(self):
        self.matvecs = 0
        self.steps = 0
        self.rejected = 0


class Segment:
    """A run of equal steps of size h on the grid t_k = t_s + k*h (computed, not
    accumulated).  A ``pc4`` segment takes RK4 steps for k = 0, 1, 2, keeping
    f_k = f(t_k, y_k) (RK4's first stage), evaluates f_3 once, and then takes
    predictor-corrector steps."""

    def __init__(self, ham, y, t_s, h, method="pc4", shift=0.0, counter=None, apply=apply_h):
        if method not in ("pc4", "rk4"):
            raise ValueError(method)
        self.ham, self.t_s, self.h, self.method, self.shift = ham, t_s, h, method, shift
        self.apply = apply
        self.cnt = counter if counter is not None else Counter()
        self.k = 0
        self.y = np.array(y, dtype=np.complex128, copy=True)
        self.f = []          # f_{k-3} .. f_k once the bootstrap is done

    def t(self, k):
        return self.t_s + k * self.h

    def state(self):
        return (self.k, self.y, list(self.f))

    def restore(self, st):
        self.k, self.y, self.f = st[0], st[1], list(st[2])

    def advance(self, nsteps, errs=None):
        """Take nsteps steps; append each predictor-corrector step's Milne
        estimate to ``errs`` when given."""
        ham, h, sh, cnt, ap = self.ham, self.h, self.shift, self.cnt, self.apply
        for _ in range(nsteps):
            k = self.k
            tk = self.t(k)
            y = self.y
            if self.method == "rk4":
                y = rk4_step(ham, tk, y, h, sh, apply=ap)
                cnt.matvecs += 4
            elif k < 3:
                fk = rhs(ham, tk, y, sh, ap)
                self.f.append(fk)
                y = rk4_step(ham, tk, y, h, sh, k1=fk, apply=ap)   # RK4's first stage is f_k
                cnt.matvecs += 4
            else:
                if k == 3:
                    self.f.append(rhs(ham, tk, y, sh, ap))   # f_3 closes the bootstrap
                    cnt.matvecs += 1
                fk, fk1, fk2, fk3 = self.f[-1], self.f[-2], self.f[-3], self.f[-4]
                yp = y + (h / 24.0) * (AB4[0] * fk + AB4[1] * fk1 + AB4[2] * fk2 + AB4[3] * fk3)
                fp = rhs(ham, self.t(k + 1), yp, sh, ap)     # the single evaluation
                yc = y + (h / 24.0) * (AM4[0] * fp + AM4[1] * fk + AM4[2] * fk1 + AM4[3] * fk2)
                if errs is not None:
                    errs.append(MILNE * float(np.linalg.norm(yc - yp)))
                y = yc
                self.f = self.f[-3:] + [fp]
                cnt.matvecs += 1
            self.y = y
            self.k = k + 1
            cnt.steps += 1
        return self.y


def run_segment(ham, y0, t_s, h, K, method="pc4", shift=0.0, counter=None, errs=None, apply=apply_h):
    """K steps of size h from (t_s, y0)."""
    return Segment(ham, y0, t_s, h, method, shift, counter, apply).advance(K, errs)


def evolve(ham, psi0, t0, t1, n_steps, method="pc4", shift=0.0, counter=None, apply=apply_h):
    """Fixed-step solution psi(t1) from psi(t0) = psi0 with h = (t1 - t0)/n_steps."""
    h = (t1 - t0) / n_steps
    y = run_segment(ham, psi0, t0, h, n_steps, method, shift, counter, apply=apply)
    return np.exp(-1j * shift * (t1 - t0)) * y


def evolve_segments(ham, psi0, t0, t1, segments, shift=0.0, counter=None):
    """Replay a list of (t_start, h, n_steps) pc4 segments (each with its own
    RK4 bootstrap), then restore the shift's phase."""
    y = np.array(psi0, dtype=np.complex128, copy=True)
    for (ts, h, K) in segments:
        y = run_segment(ham, y, ts, h, K, "pc4", shift, counter)
    return np.exp(-1j * shift * (t1 - t0)) * y


def evolve_adaptive(ham, psi0, t0, t1, atol, h0, hmin=0.0, hmax=math.inf, window=8,
                    shift=0.0, max_steps=10_000_000, unit_roundoff=2.0 ** -53):
    """Adaptive pc4 as described in the module docstring.

    ``unit_roundoff`` is that of the arithmetic the estimate is formed in: the
    estimate cannot resolve errors below floor = 4 (19/270) u ||psi0||, so an
    atol below the floor is refused, and the step only grows when the estimate
    is below max(atol/64, 8 floor).

    Returns (psi(t1), segments, counter); ``segments`` is the accepted
    (t_start, h, n_steps) list that ``evolve_segments`` replays.
    """
    floor = 4.0 * MILNE * unit_roundoff * float(np.linalg.norm(psi0))
    if atol < floor:
        raise ValueError(f"atol {atol:g} below the precision floor {floor:g} of the estimate")
    grow_below = max(atol / 64.0, 8.0 * floor)
    cnt = Counter()
    segments = []
    h = min(h0, hmax)
    seg = Segment(ham, psi0, t0, h, "pc4", shift, cnt)
    windows_at_h = 0
    # the step is not halved below this floor, and at most 60 windows in a row
    # are undone: an estimate that never falls below atol ends the run
    h_floor = max(hmin, 1e-12 * (t1 - t0))
    rejections_in_row = 0
    while True:
        t_now = seg.t(seg.k)
        left = t1 - t_now
        if left <= 0.0:
            break
        final = left <= window * seg.h * (1.0 + 1e-12)
        nsteps = window
        if final:
            # last stretch: an integer number of equal steps that ends at t1
            nsteps = max(1, int(math.ceil(left / seg.h - 1e-9)))
            hf = left / nsteps
            if hf != seg.h:
                if seg.k > 0:
                    segments.append((seg.t_s, seg.h, seg.k))
                seg = Segment(ham, seg.y, t_now, hf, "pc4", shift, cnt)
                windows_at_h = 0
        before = seg.state()
        errs = []
        seg.advance(nsteps, errs)
        emax = max(errs) if errs else 0.0
        if emax > atol:
            rejections_in_row += 1
            if seg.h / 2.0 < h_floor or rejections_in_row > 60:
                raise RuntimeError("adaptive step: error estimate stays above atol")
            # undo the window, restart from its first state with half the step
            cnt.rejected += nsteps
            cnt.steps -= nsteps
            seg.restore(before)
            if seg.k > 0:
                segments.append((seg.t_s, seg.h, seg.k))
            seg = Segment(ham, seg.y, seg.t(seg.k), seg.h / 2.0, "pc4", shift, cnt)
            windows_at_h = 0
            continue
        rejections_in_row = 0
        windows_at_h += 1
        if final:
            segments.append((seg.t_s, seg.h, seg.k))
            break
        if cnt.steps > max_steps:
            raise RuntimeError("adaptive step limit reached")
        if emax < grow_below and windows_at_h >= 2 and 2.0 * seg.h <= hmax:
            segments.append((seg.t_s, seg.h, seg.k))
            seg = Segment(ham, seg.y, seg.t(seg.k), 2.0 * seg.h, "pc4", shift, cnt)
            windows_at_h = 0
    return np.exp(-1j * shift * (t1 - t0)) * seg.y, segments, cnt
