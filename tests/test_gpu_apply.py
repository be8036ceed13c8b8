"""GPU parity of H(t)|psi> (aqc_apply through the C ABI) against the oracle."""
import math

import numpy as np
import pytest

from oracle import sqh, observables
from paper_1311_3938_amd import instances as I
from tests._gpu import to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu

# float32 products: a sum of ~n terms of relative error 2^-24 each
APPLY_TOL = {"c64": 5e-6, "c128": 1e-12}


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


def _cases():
    rng = np.random.default_rng(1234)
    out = []
    out.append(("sk_diag_only", I.sk_terms(9, *I.sk_couplings(9, rng)).instance(
        [I.SCHED_S], I.sin2_path(2.0))))
    tx, tz = I.tfim_terms(11)
    t = I.TermList(11)
    t.extend(tx, sid=0)
    t.extend(tz, sid=1)
    out.append(("tfim", t.instance([I.SCHED_ONE_MINUS_S, I.SCHED_S], I.linear_path(3.0))))
    out.append(("random_mixed", I.random_terms(10, 60, rng, n_sched=3).instance(
        [I.SCHED_ONE_MINUS_S, I.trig_t(0.9, 1.7, 0.1), I.poly_s([0.2, 1.0, -1.3])],
        I.linear_path(2.0))))
    cl = I.ec3_random_clauses(10, 8, rng)
    out.append(("xy_path", I.interpolated(10, I.xy_initial_terms(10, cl), I.ec3_terms(10, cl),
                                          I.linear_path(5.0))))
    out.append(("ec3_catalyst_16", I.workload_ec3_catalyst(n=16, m=13, n_pairs=16, T=5.0, seed=7)))
    out.append(("sk_sin2_18", I.workload_sk_sin2(n=18, T=5.0, seed=8)))
    out.append(("random_high_17", I.random_terms(17, 50, rng, max_weight_ops=3, n_sched=2).instance(
        [I.SCHED_S, I.trig_t(1.0, 0.5)], I.linear_path(2.0))))
    out.append(("one_qubit", _one_qubit()))
    out.append(("two_qubit", I.random_terms(2, 12, rng, n_sched=1).instance(
        [I.SCHED_CONST], I.linear_path(1.0))))
    return out


def _one_qubit():
    t = I.TermList(1)
    t.add({1: "Z"}, 0.7, 0)
    t.add({1: "X"}, 1.0, 1)
    t.add({1: "Y"}, 1.0, 2)
    t.add({}, 0.25, 0)
    return t.instance([I.SCHED_CONST, I.trig_t(0.4, 0.8), I.trig_t(0.4, 0.8, -math.pi / 2)],
                      I.linear_path(1.0))


CASES = _cases()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("name,inst", CASES, ids=[c[0] for c in CASES])
def test_apply_matches_oracle(eng, name, inst, dt):
    engine, ctx = eng
    ham = engine.Hamiltonian(ctx, inst)
    rng = np.random.default_rng(5)
    psi = I.random_state(inst.n, rng)
    T = inst.path["T"]
    for t in (0.31 * T, 0.77 * T):
        want = sqh.apply_h(inst, t, psi)
        got = to_host(engine.apply(ctx, ham, t, to_dev(psi, dt)))
        assert rel_err(got, want) < APPLY_TOL[dt], (name, dt, t)
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("exact", [True, False], ids=["quarter_weights", "normal_weights"])
def test_apply_many_low_bit_diagonal_schedules(eng, dt, exact):
    """Ten schedules, each with Z pairs and triples inside the last tile's low
    bits (one diagonal table per schedule, the first four read unrolled and
    the rest in a loop), beside single and straddling Z terms and flips;
    weights that are multiples of 1/4 (as in exact-cover clauses) and normal
    ones."""
    engine, ctx = eng
    rng = np.random.default_rng(77 if exact else 78)
    n, ns = 16, 10
    t = I.TermList(n)
    for sid in range(ns):
        for _ in range(4):
            k = int(rng.integers(2, 4))
            qs = rng.choice(10, k, replace=False)
            w = float(rng.integers(-8, 9)) / 4.0 if exact else float(rng.normal())
            t.add({int(q) + 1: "Z" for q in qs}, w, sid)
        t.add({int(rng.integers(0, n)) + 1: "Z", int(rng.integers(12, n)) + 1: "Z"}, 0.5, sid)
    for q in range(n):
        t.add({q + 1: "X"}, 0.3 + 0.01 * q, ns)
    scheds = [I.poly_s([0.1 * (j + 1), 1.0 - 0.15 * j]) for j in range(ns)] + [I.SCHED_ONE_MINUS_S]
    inst = t.instance(scheds, I.linear_path(2.0))
    ham = engine.Hamiltonian(ctx, inst)
    psi = I.random_state(n, np.random.default_rng(6))
    for tt in (0.4, 1.3):
        want = sqh.apply_h(inst, tt, psi)
        got = to_host(engine.apply(ctx, ham, tt, to_dev(psi, dt)))
        assert rel_err(got, want) < APPLY_TOL[dt], (dt, exact, tt)
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_apply_with_small_tiles_many_passes(eng, dt, monkeypatch):
    """Force tiny tiles so that flip patterns spread over many high passes."""
    engine, ctx = eng
    key = "C64" if dt == "c64" else "C128"
    monkeypatch.setenv(f"AQC_TBF_{key}", "5")
    monkeypatch.setenv(f"AQC_TBH_{key}", "6")
    monkeypatch.setenv(f"AQC_LH_{key}", "2")
    rng = np.random.default_rng(77)
    inst = I.random_terms(12, 80, rng, max_weight_ops=3, n_sched=2).instance(
        [I.SCHED_S, I.SCHED_ONE_MINUS_S], I.linear_path(1.0))
    ham = engine.Hamiltonian(ctx, inst)
    psi = I.random_state(12, rng)
    want = sqh.apply_h(inst, 0.4, psi)
    got = to_host(engine.apply(ctx, ham, 0.4, to_dev(psi, dt)))
    assert ham.info()["n_passes"][0 if dt == "c64" else 1] > 3
    assert rel_err(got, want) < APPLY_TOL[dt]
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_reductions_match_oracle(eng, dt):
    engine, ctx = eng
    rng = np.random.default_rng(11)
    inst = I.workload_ec3_catalyst(n=15, m=12, n_pairs=15, T=4.0, seed=3)
    ham = engine.Hamiltonian(ctx, inst)
    psi = I.random_state(15, rng)
    phi = I.random_state(15, rng)
    dpsi, dphi = to_dev(psi, dt), to_dev(phi, dt)
    psi_r = to_host(dpsi)     # the values the device holds (rounded for c64)
    phi_r = to_host(dphi)
    tol = 1e-12
    assert engine.norm2(ctx, dpsi) == pytest.approx(observables.norm2(psi_r), abs=tol)
    ov = engine.overlap(ctx, dphi, dpsi)
    want = observables.overlap(phi_r, psi_r)
    assert abs(ov - want) < tol
    assert engine.fidelity_state(ctx, dpsi, dphi) == pytest.approx(abs(want) ** 2, abs=tol)
    idx = [0, 5, 5, 77, (1 << 15) - 1]
    assert engine.fidelity_basis(ctx, dpsi, idx) == pytest.approx(
        observables.basis_mass(psi_r, idx), abs=tol)
    for t in (4.0, 1.3):
        m, emin = engine.ground_mass(ctx, ham, t, dpsi)
        m_want, e_want = observables.ground_mass(inst, t, psi_r)
        assert emin == pytest.approx(e_want, abs=1e-12)
        assert m == pytest.approx(m_want, abs=tol)
        e = engine.energy(ctx, ham, t, dpsi)
        e_ref = observables.energy(inst, t, psi_r)
        assert abs(e - e_ref) < (1e-11 if dt == "c128" else 1e-5 * max(1.0, abs(e_ref)))
    ham.free()


def test_errors_are_reported(eng):
    engine, ctx = eng
    from paper_1311_3938_amd import _lib
    inst = I.workload_ec3_linear(n=6, m=4, T=2.0, seed=1)
    ham = engine.Hamiltonian(ctx, inst)
    import torch
    psi = to_dev(I.plus_state(6), "c64")
    with pytest.raises(_lib.AqcError) as ei:
        engine.apply(ctx, ham, 0.0, psi, out=psi)
    assert ei.value.status == _lib.AQC_EINVAL
    bad = I.TermList(3)
    bad.add_masks(1 << 5, 0, 1.0, 0)
    with pytest.raises(_lib.AqcError):
        engine.Hamiltonian(ctx, bad.instance([I.SCHED_CONST], I.linear_path(1.0)))
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("regpass,n", [("1", 20), ("0", 20), ("2", 20), ("3", 20), ("3", 17),
                                       ("3", 16)])
def test_apply_register_hypercube_pass(eng, dt, regpass, n, monkeypatch):
    """Single-qubit flips above the last tile run in register hypercube passes:
    narrow (one wave per hypercube), wide (the waves of a workgroup span three
    more bits and trade vertices through LDS), or, switched off, in tile
    passes; pairs and Y/Z mixes that straddle the tile stay in tile passes.
    n = 16 and 17 are the smallest states with wide passes (one and two
    workgroups per pass)."""
    engine, ctx = eng
    monkeypatch.setenv("AQC_REGPASS", regpass)
    rng = np.random.default_rng(2020 + n)
    t = I.TermList(n)
    for q in range(1, n + 1):
        t.add({q: "X"}, rng.normal(), 0)
        t.add({q: "Z"}, rng.normal(), 1)
    for _ in range(12):
        i, j = sorted(int(v) + 1 for v in rng.choice(n, 2, replace=False))
        t.add({i: "X", j: "X"}, rng.normal(), 2)
        t.add({i: "Y", j: "Z"}, rng.normal(), 0)
    inst = t.instance([I.SCHED_ONE_MINUS_S, I.SCHED_S, I.SCHED_S_ONE_MINUS_S], I.linear_path(1.0))
    ham = engine.Hamiltonian(ctx, inst)
    psi = I.random_state(n, rng)
    want = sqh.apply_h(inst, 0.37, psi)
    got = to_host(engine.apply(ctx, ham, 0.37, to_dev(psi, dt)))
    assert rel_err(got, want) < APPLY_TOL[dt]
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("regpass,n", [("1", 20), ("0", 20), ("0", 14), ("3", 17)])
def test_apply_stream_groups(eng, dt, regpass, n, monkeypatch):
    """Flip patterns above the last tile applied by the last pass itself, which
    reads the partner amplitudes from the source vector: pairs straddling the
    tile, pairs and triples above it, and Y/Z mixes whose coefficient depends
    on the basis state; with register passes on, the single-qubit flips stay
    in them."""
    engine, ctx = eng
    monkeypatch.setenv("AQC_STREAM", "1")
    monkeypatch.setenv("AQC_REGPASS", regpass)
    rng = np.random.default_rng(3030 + n)
    t = I.TermList(n)
    for q in range(1, n + 1):
        t.add({q: "X"}, rng.normal(), 0)
        t.add({q: "Z"}, rng.normal(), 1)
    for _ in range(10):
        i, j, k = sorted(int(v) + 1 for v in rng.choice(n, 3, replace=False))
        t.add({i: "X", j: "X"}, rng.normal(), 2)
        t.add({i: "Y", k: "Z"}, rng.normal(), 0)
        t.add({j: "X", k: "Y"}, rng.normal(), 1)
        t.add({i: "X", j: "Y", k: "X"}, rng.normal(), 2)
    inst = t.instance([I.SCHED_ONE_MINUS_S, I.SCHED_S, I.SCHED_S_ONE_MINUS_S], I.linear_path(1.0))
    ham = engine.Hamiltonian(ctx, inst)
    psi = I.random_state(n, rng)
    want = sqh.apply_h(inst, 0.61, psi)
    got = to_host(engine.apply(ctx, ham, 0.61, to_dev(psi, dt)))
    assert rel_err(got, want) < APPLY_TOL[dt]
    if regpass == "0":
        assert ham.info()["n_passes"][0 if dt == "c64" else 1] == 1
    ham.free()


def test_freed_tables_are_not_reused_under_queued_launches(eng):
    """Table buffers of a freed Hamiltonian go to a pool and are handed out
    again only once every stream the library launches on has passed the
    release.  Products queued on one stream keep reading their tables while a
    Hamiltonian of the same size is built (and uploaded) on another stream
    right after the free; all of them must match the oracle.  The next
    Hamiltonian built after the queue has drained may reuse the buffers, and
    after aqc_trim new ones are allocated; both give the same product."""
    import dataclasses
    import torch
    engine, _ = eng
    from paper_1311_3938_amd import _lib
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ca, cb = engine.Context(0, stream=sa), engine.Context(0, stream=sb)
    inst = I.workload_sk_sin2(n=20, T=5.0, seed=21)
    inst2 = dataclasses.replace(inst, w=inst.w * 2.0)
    rng = np.random.default_rng(3)
    psi = I.random_state(20, rng)
    t = 1.1
    want = sqh.apply_h(inst, t, psi)
    x = to_dev(psi, "c128")
    outs = [torch.empty_like(x) for _ in range(40)]
    torch.cuda.synchronize()
    ham = engine.Hamiltonian(ca, inst)
    need = _lib.lib().aqc_apply_workspace_bytes(ham.handle, _lib.C128)
    ws = engine.workspace(ca, need)
    for o in outs:
        engine.apply(ca, ham, t, x, out=o, ws=ws)
    ham.free()                               # the products above are still queued on sa
    ham2 = engine.Hamiltonian(cb, inst2)     # built and uploaded on sb meanwhile
    sa.synchronize()
    for o in outs:
        assert rel_err(to_host(o), want) < APPLY_TOL["c128"]
    ws2 = engine.workspace(cb, need)
    out2 = engine.apply(cb, ham2, t, x, ws=ws2)
    sb.synchronize()                         # results are read on the default stream
    assert rel_err(to_host(out2), 2.0 * want) < APPLY_TOL["c128"]
    ham2.free()
    for rebuild in ("reused", "after trim"):
        if rebuild == "after trim":
            engine.trim(0)
        h = engine.Hamiltonian(ca, inst)
        out = engine.apply(ca, h, t, x, ws=ws)
        sa.synchronize()
        assert rel_err(to_host(out), want) < APPLY_TOL["c128"], rebuild
        h.free()
    sa.synchronize()
    sb.synchronize()
    ca.close()
    cb.close()
