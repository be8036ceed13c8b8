"""Drive the host code of the library, built against the CPU stand-in of the
HIP runtime (fake_hip.cpp) with AddressSanitizer, through the Python front
end: Hamiltonian compilation for every workload family, tilings, H|psi>,
fixed, chained and adaptive evolution, reductions, sectors, Lanczos, the host
eigensolver and the batch engine with retire / re-admit and graphs, then the
batched energies and whole batched rounds of the T_s search.  Prints "host paths done" and exits 0
when every path ran and no handle is left alive.

Usage: python drive.py <path of the instrumented libaqc.so>"""
import ctypes as C
import os
import sys
import types

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import numpy as np
import torch

from paper_1311_3938_amd import _lib as L

L.LIB_PATH = sys.argv[1]
from paper_1311_3938_amd import engine, instances as I, tsearch  # noqa: E402
from paper_1311_3938_amd._lib import check, lib  # noqa: E402


class CpuCtx(engine.Context):
    """A context whose "device" tensors are host tensors (the stand-in
    runtime's device memory is host memory)."""

    def __init__(self):
        self.device = torch.device("cpu")
        self.stream = types.SimpleNamespace(cuda_stream=0)
        h = C.c_void_p()
        check(lib().aqc_create(0, C.c_void_p(0), C.byref(h)))
        self._h = h


def expect(f, *errors):
    """Run f; library errors with one of the given statuses are expected
    outcomes of kernels that compute nothing (no convergence and the like)."""
    try:
        return f()
    except L.AqcError as e:
        if e.status not in errors:
            raise


def status_of(f):
    try:
        f()
    except L.AqcError as e:
        return e.status
    return L.AQC_OK


def host_error_paths(ctx):
    """Error returns the header documents that need a context: sizes,
    alignment, aliasing, workspace, batch slots."""
    lib_ = lib()
    ham = engine.Hamiltonian(ctx, I.workload_sk_sin2(n=10))
    N = 1 << 10
    a = torch.zeros(N + 2, dtype=torch.complex128)
    b = torch.zeros(N, dtype=torch.complex128)
    ws = torch.zeros(1 << 22, dtype=torch.uint8)
    P = C.c_void_p
    ap, bp, wp = P(a.data_ptr()), P(b.data_ptr()), P(ws.data_ptr())
    mis = P(a.data_ptr() + 8)                      # 8-byte offset: not 16-byte aligned
    need = lib_.aqc_apply_workspace_bytes(ham.handle, L.C128)
    assert status_of(lambda: check(lib_.aqc_apply(ctx.handle, ham.handle, 0.1, ap, ap, L.C128, wp, need))) \
        == L.AQC_EINVAL                            # in == out
    assert status_of(lambda: check(lib_.aqc_apply(ctx.handle, ham.handle, 0.1, mis, bp, L.C128, wp, need))) \
        == L.AQC_EINVAL                            # alignment
    assert status_of(lambda: check(lib_.aqc_apply(ctx.handle, ham.handle, 0.1, ap, bp, 7, wp, need))) \
        == L.AQC_ENOTSUP                           # dtype
    if need:
        assert status_of(lambda: check(lib_.aqc_apply(ctx.handle, ham.handle, 0.1, ap, bp, L.C128, wp,
                                                      need - 16))) == L.AQC_ENOMEM
    opts, _, _ = engine.evolve_opts(method="pc4", n_steps=10, shift=0.5)
    st = L.EvolveStats()
    wneed = lib_.aqc_evolve_workspace_bytes(ham.handle, L.C128, C.byref(opts))
    assert status_of(lambda: check(lib_.aqc_evolve(ctx.handle, ham.handle, ap, L.C128, 0.0, 1.0, C.byref(opts),
                                                   wp, wneed - 16, C.byref(st)))) == L.AQC_ENOMEM
    assert status_of(lambda: check(lib_.aqc_evolve(ctx.handle, ham.handle, ap, L.C128, 1.0, 0.0, C.byref(opts),
                                                   wp, wneed, C.byref(st)))) == L.AQC_EINVAL   # t1 < t0
    bad = engine.evolve_opts(method="pc4", n_steps=0, atol=0.0)[0]
    assert status_of(lambda: check(lib_.aqc_evolve(ctx.handle, ham.handle, ap, L.C128, 0.0, 1.0, C.byref(bad),
                                                   wp, ws.numel(), C.byref(st)))) == L.AQC_EINVAL
    assert status_of(lambda: ham.set_tiling(torch.complex128, 40, 12, 3, 1)) != L.AQC_OK
    # Lanczos: a basis larger than the space, too many levels, a basis too small for them
    tiny = engine.Hamiltonian(ctx, I.random_terms(2, 6, np.random.default_rng(2)).instance(
        [I.SCHED_CONST], I.linear_path(1.0)))
    assert status_of(lambda: engine.lowest_eigs(ctx, tiny, 0.0, k=2, max_basis=8)) == L.AQC_EINVAL
    assert status_of(lambda: engine.lowest_eigs(ctx, ham, 0.0, k=9, max_basis=24)) == L.AQC_EINVAL
    assert status_of(lambda: engine.lowest_eigs(ctx, ham, 0.0, k=3, max_basis=4)) == L.AQC_EINVAL
    tiny.free()
    # a batch of one slot: a second admission is refused, an unfinished solve
    # cannot retire, a short workspace is refused
    bt = engine.Batch(ctx, torch.complex64, capacity=1, graph=True)
    p1 = torch.zeros(N, dtype=torch.complex64)
    p2 = torch.zeros(N, dtype=torch.complex64)
    short = torch.zeros(16, dtype=torch.uint8)
    sl = C.c_int()
    assert status_of(lambda: check(lib_.aqc_batch_admit(bt._h, ham.handle, P(p1.data_ptr()), P(short.data_ptr()),
                                                        short.numel(), 0.0, 1.0, 20, 0.0, C.byref(sl)))) \
        == L.AQC_ENOMEM
    slot = bt.admit(ham, p1, 0.0, 1.0, 20, 0.0)
    assert status_of(lambda: bt.admit(ham, p2, 0.0, 1.0, 20, 0.0)) == L.AQC_EBUSY
    assert status_of(lambda: check(lib_.aqc_batch_retire(bt._h, slot, None))) == L.AQC_EBUSY
    assert status_of(lambda: check(lib_.aqc_batch_retire(bt._h, 5, None))) == L.AQC_EINVAL
    while bt.step(8):
        pass
    assert bt.poll() == [slot]
    bt.retire(slot)
    bt.close()
    ham.free()


def context_outlived_by_batch():
    """A batch and its context destroyed in either order (finalizers of a
    reference cycle run in no fixed order): the context's memory stays until
    its last batch is gone, a batch whose context was destroyed refuses work,
    and destroying that context again is refused."""
    for first in ("ctx", "batch"):
        c2 = CpuCtx()
        b = engine.Batch(c2, torch.complex64, capacity=2)
        ham = engine.Hamiltonian(c2, I.workload_batch_member(0, 10, 10))
        psi = torch.zeros(1 << ham.n, dtype=torch.complex64)
        psi[0] = 1
        b.admit(ham, psi, 0.0, 1.0, 6, 0.1)
        b.step(2)
        if first == "ctx":
            raw = c2.handle.value
            c2.close()
            assert status_of(lambda: b.step(1)) == L.AQC_EINVAL
            assert status_of(lambda: b.poll()) == L.AQC_EINVAL
            assert status_of(lambda: b.admit(ham, psi.clone(), 0.0, 1.0, 4, 0.0)) == L.AQC_EINVAL
            assert lib().aqc_destroy(C.c_void_p(raw)) == L.AQC_EINVAL
            b.close()
        else:
            b.close()
            c2.close()
        ham.free()


def failed_builds_release_tables(ctx):
    """A sector whose build fails at any of its device allocations returns an
    error and leaves no device buffer behind (the partly built Hamiltonian
    releases its tables), and the build then succeeds."""
    engine.trim(0)
    ham = engine.Hamiltonian(ctx, I.workload_usa(8, 0, "xy"))
    engine.trim(0)
    base = lib().fake_hip_live()
    lib().fake_hip_fail_malloc_after.argtypes = [C.c_long]
    failed = 0
    for k in range(64):
        lib().fake_hip_fail_malloc_after(k)
        try:
            sec = engine.Sector(ctx, ham, 3)
        except L.AqcError as e:
            lib().fake_hip_fail_malloc_after(-1)
            assert e.status == L.AQC_EDEVICE, (k, e)
            failed += 1
            engine.trim(0)
            live = lib().fake_hip_live() - base
            assert live == 0, f"failed sector build ({k} allocations) left {live} handles"
            continue
        lib().fake_hip_fail_malloc_after(-1)
        sec.free()
        break
    else:
        raise AssertionError("the sector build never succeeded")
    # the rank, hop, term and mask tables, and the stored diagonal
    assert failed >= 5, failed
    ham.free()
    engine.trim(0)
    # a context whose buffers cannot all be allocated
    base = lib().fake_hip_live()
    for k in range(2):
        lib().fake_hip_fail_malloc_after(k)
        out = C.c_void_p()
        status = lib().aqc_create(0, None, C.byref(out))
        lib().fake_hip_fail_malloc_after(-1)
        assert status == L.AQC_EDEVICE and not out.value, (k, status)
        live = lib().fake_hip_live() - base
        assert live == 0, f"failed context creation ({k} allocations) left {live} handles"


def plan_choice(ctx):
    """The default plan keeps register passes for the single-qubit flips above
    the last tile unless a layout without them needs fewer passes: the 24-qubit
    SK workload (single flips only: two register passes or two tile high
    passes, a tie) keeps them; the 24-qubit catalyst workload, whose pair
    flips straddle the tile, needs 4 passes without them instead of 5."""
    sk = engine.Hamiltonian(ctx, I.workload_sk_sin2(n=24))
    assert sk.info()["n_passes"][0] == 3, sk.info()
    sk.free()
    cat = engine.Hamiltonian(ctx, I.workload_ec3_catalyst())
    assert cat.info()["n_passes"][0] == 4, cat.info()
    cat.set_tiling(torch.complex64, 13, 13, 4, 3)        # wide register passes asked for
    assert cat.info()["n_passes"][0] == 5, cat.info()
    cat.free()


def main():
    lib().fake_hip_live.restype = C.c_long
    base = lib().fake_hip_live()
    ctx = CpuCtx()
    plan_choice(ctx)
    insts = [I.workload_sk_sin2(n=12), I.workload_ec3_catalyst(n=14, m=12, n_pairs=10),
             I.workload_ec3_paths(n=13, kind="cbc"), I.workload_ec3_paths(n=13, kind="nonlinear"),
             I.workload_usa(10, 0, "xy"), I.workload_usa(10, 1, "xyz")]
    for inst in insts:
        for dt in (torch.complex64, torch.complex128):
            ham = engine.Hamiltonian(ctx, inst)
            N = 1 << inst.n
            psi = torch.zeros(N, dtype=dt)
            psi[0] = 1
            engine.apply(ctx, ham, 0.3, psi, torch.empty_like(psi))
            ham.spectral_bounds(0.0, inst.path["T"])
            engine.evolve(ctx, ham, psi, 0.0, 1.0, method="pc4", n_steps=10, shift="center")
            engine.evolve(ctx, ham, psi, 0.0, 1.0, method="rk4", n_steps=5)
            expect(lambda: engine.evolve(ctx, ham, psi, 0.0, 1.0, method="pc4", n_steps=0, atol=1e-6,
                                         h0=0.01, window=4, hmin=1e-3, record_cap=16), L.AQC_EUNSTABLE)
            carry, ws = engine.new_carry(), engine.workspace(ctx, 1 << 25)
            for k in range(3):
                engine.evolve(ctx, ham, psi, 0.1 * k, 0.1 * (k + 1), ws=ws, carry=carry, method="pc4",
                              n_steps=5, shift=0.5)
            engine.energy(ctx, ham, 1.0, psi)
            engine.energy_noalloc(ctx, ham, 1.0, psi)
            engine.ground_mass(ctx, ham, 1.0, psi)
            engine.norm2(ctx, psi)
            engine.overlap(ctx, psi, psi)
            engine.fidelity_basis(ctx, psi, [0, 1, 3])
            engine.fidelity_state(ctx, psi, psi.clone())
            for bad in (lambda: engine.fidelity_state(ctx, psi, psi[:-1].clone()),
                        lambda: engine.fidelity_basis(ctx, psi[:-1].clone(), [0])):
                try:
                    bad()
                except ValueError:
                    pass
                else:
                    raise AssertionError("a state of the wrong size was accepted")
            for til in ((12, 12, 4, 3), (11, 12, 3, 2), (13, 13, 4, 4), (10, 11, 3, 0), (12, 13, 5, 7)):
                ham.set_tiling(dt, *til)
                engine.apply(ctx, ham, 0.3, psi, torch.empty_like(psi))
            expect(lambda: engine.lowest_eigs(ctx, ham, 0.5, k=2, dtype=dt, max_basis=12, max_matvecs=60),
                   L.AQC_EUNSTABLE)
            keeps = all(bin(int(x)).count("1") in (0, 2) for x in inst.x)
            for w in ((1, inst.n // 2, inst.n - 1) if keeps else ()):
                sec = engine.Sector(ctx, ham, w)
                sec.dicke(dt)
                sp = torch.zeros(sec.dim, dtype=dt)
                sp[0] = 1
                sec.expand(sp)
                # the wrappers check sizes the C calls do not take
                for bad in (lambda: sec.expand(torch.zeros(sec.dim + 1, dtype=dt)),
                            lambda: engine.energy(ctx, sec, 1.0, torch.zeros(sec.dim - 1, dtype=dt)),
                            lambda: engine.ground_mass(ctx, ham, 1.0, sp)):
                    try:
                        bad()
                    except ValueError:
                        pass
                    else:
                        raise AssertionError("a state of the wrong size was accepted")
                engine.apply(ctx, sec, 0.4, sp, torch.empty_like(sp))
                engine.evolve(ctx, sec, sp, 0.0, 1.0, method="pc4", n_steps=8, shift="center")
                engine.energy(ctx, sec, 1.0, sp)
                engine.energy_noalloc(ctx, sec, 1.0, sp)
                engine.ground_mass(ctx, sec, 1.0, sp)
                expect(lambda: engine.lowest_eigs(ctx, sec, 0.5, k=2, dtype=dt, max_basis=10, max_matvecs=40),
                       L.AQC_EUNSTABLE)
                sec.free()
            ham.free()
    # sector limits and refusals, decided on the host
    full_xy = I.TermList(34)
    for i in range(1, 35):
        for j in range(i + 1, 35):
            full_xy.add({i: "X", j: "X"}, -0.5, 0)
            full_xy.add({i: "Y", j: "Y"}, -0.5, 0)
    big = engine.Hamiltonian(ctx, full_xy.instance([I.SCHED_S], I.linear_path(1.0)))
    sk = engine.Hamiltonian(ctx, I.workload_sk_sin2(n=8))
    small = engine.Hamiltonian(ctx, I.workload_usa(8, 0, "xy"))
    one = engine.Sector(ctx, small, 3)
    for ham_, w, status in ((big, 17, L.AQC_ENOTSUP),      # 1122 pair terms > 1024
                            (big, 35, L.AQC_EINVAL), (small, -1, L.AQC_EINVAL),
                            (sk, 4, L.AQC_EINVAL),         # transverse field changes the weight
                            (one, 1, L.AQC_EINVAL)):       # already a sector
        try:
            engine.Sector(ctx, ham_, w)
        except L.AqcError as e:
            assert e.status == status, (w, e)
        else:
            raise AssertionError(f"sector of weight {w} was not refused")
    for h in (one, small, sk, big):
        h.free()
    host_error_paths(ctx)
    failed_builds_release_tables(ctx)
    # the allocation-free energy refuses what its fixed scratch cannot hold
    # and plans that are not built yet
    for n, status in ((23, L.AQC_ENOMEM), (27, L.AQC_EINVAL)):
        h = engine.Hamiltonian(ctx, I.workload_sk_sin2(n=n))
        expect(lambda: engine.energy_noalloc(ctx, h, 1.0, torch.empty(1 << n, dtype=torch.complex64)), status)
        h.free()
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 17, 48):
        a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        a = a + a.conj().T
        w, _ = engine.hermitian_eigh(a)
        assert np.max(np.abs(np.sort(w) - np.linalg.eigvalsh(a))) < 1e-10 * max(1.0, np.abs(w).max())
    # a batch smaller than its queue: solves retire and new ones are admitted
    for graph in (True, False):
        b = engine.Batch(ctx, torch.complex64, capacity=6, graph=graph)
        hams = [engine.Hamiltonian(ctx, I.workload_batch_member(k, 10, 14)) for k in range(10)]
        nxt = 0

        def admit():
            nonlocal nxt
            psi = torch.zeros(1 << hams[nxt].n, dtype=torch.complex64)
            psi[0] = 1
            b.admit(hams[nxt], psi, 0.0, 1.0, 5 + 3 * nxt, 0.3)
            nxt += 1

        while nxt < 6:
            admit()
        while b.info()["active"] or nxt < 10:
            b.step(5)
            for s in b.poll():
                b.retire(s)
                if nxt < 10:
                    admit()
        b.close()
        for h in hams:
            h.free()
    # resident solves (one workgroup each) beside ticked ones, with solves
    # retired and re-admitted between steps
    for dt in (torch.complex64, torch.complex128):
        b = engine.Batch(ctx, dt, capacity=6, resident_max_n=12)
        hams = [engine.Hamiltonian(ctx, I.workload_batch_member(k, 10, 14)) for k in range(9)]
        states = []
        for k in range(6):
            psi = torch.zeros(1 << hams[k].n, dtype=dt)
            psi[0] = 1
            states.append(psi)
            b.admit(hams[k], psi, 0.0, 1.0, 4 + 2 * k, 0.2)
        nxt = 6
        while b.info()["active"] or nxt < 9:
            b.step(6)
            for slot in b.poll():
                b.retire(slot)
                if nxt < 9:
                    psi = torch.zeros(1 << hams[nxt].n, dtype=dt)
                    psi[0] = 1
                    b.admit(hams[nxt], psi, 0.0, 1.0, 7, 0.1)
                    nxt += 1
        b.close()
        for h in hams:
            h.free()
    expect(lambda: engine.Batch(ctx, torch.complex64, capacity=2, resident_max_n=21), L.AQC_EINVAL)
    for alg, n in (("x", 7), ("xy", 8), ("xy", 10)):
        insts = [I.workload_usa(n, k, alg) for k in range(3)]
        tsearch.energies(ctx, insts, [1.0, 2.0, 3.0], [I.plus_state(n)] * 3)
    # whole batched searches: every round creates and closes a batch and its
    # Hamiltonians (the stand-in's energies are 1, so T doubles up to T_max)
    insts = [I.workload_usa(8, k, "xy") for k in range(4)]
    S = tsearch.search_rounds(ctx, insts, [I.plus_state(8)] * 4, tsearch.energies, T_max=64.0,
                              plan=lambda ham, T: (int(8 + T), 0.5))
    assert all(len(s.evals) == 7 for s in S)
    # a table buffer released while a batch lives (its release is marked on
    # the batch's streams), reused once the batch and its streams are gone
    b = engine.Batch(ctx, torch.complex64, capacity=2)
    h = engine.Hamiltonian(ctx, I.workload_batch_member(0, 10, 14))
    h.free()
    b.close()
    h = engine.Hamiltonian(ctx, I.workload_batch_member(0, 10, 14))
    h.free()
    context_outlived_by_batch()
    ctx.close()
    # released table buffers are kept for reuse until trimmed
    assert lib().aqc_trim(64) == L.AQC_EINVAL
    engine.trim(0)
    live = lib().fake_hip_live() - base
    assert live == 0, f"{live} runtime handles left alive"
    print("host paths done", flush=True)


if __name__ == "__main__":
    main()
