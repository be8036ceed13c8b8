"""Checks at the benchmark's full size (n = 30, 2^30 amplitudes, complex64, the
three-pass plan the benchmark times) and above it (n = 32, 33; sectors at
n = 34): sampled outputs against the oracle's row-wise product, and closed
forms that hold at any size."""
import math

import numpy as np
import pytest

from oracle import sqh
from paper_1311_3938_amd import instances as I

pytestmark = pytest.mark.gpu

N_FULL = 30


@pytest.fixture(scope="module")
def eng():
    import torch
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx, torch
    ctx.close()
    torch.cuda.empty_cache()


def _rows(rng, n, k=300):
    r = rng.integers(0, 1 << n, size=k, dtype=np.int64)
    return np.unique(np.concatenate([r, [0, (1 << n) - 1, 1 << (n - 1), (1 << 13) - 1]]))


def test_apply_sampled_rows_full_size(eng):
    engine, ctx, torch = eng
    inst = I.workload_sk_sin2(n=N_FULL, T=30.0, seed=I.seed_for(2))
    ham = engine.Hamiltonian(ctx, inst)
    g = torch.Generator(device="cuda").manual_seed(3)
    psi = torch.randn(1 << N_FULL, dtype=torch.complex64, device="cuda", generator=g)
    out = engine.apply(ctx, ham, 11.0, psi)
    assert ham.info()["n_passes"][0] >= 3  # the benchmark's multi-pass plan
    rows = _rows(np.random.default_rng(4), N_FULL)

    def values_at(idx):
        t = torch.from_numpy(np.ascontiguousarray(idx)).to("cuda")
        return psi.index_select(0, t).cpu().to(torch.complex128).numpy()

    want = sqh.apply_h_rows(inst, 11.0, values_at, rows)
    got = out.index_select(0, torch.from_numpy(rows).to("cuda")).cpu().to(torch.complex128).numpy()
    scale = np.abs(want).max()
    assert np.max(np.abs(got - want)) / scale < 5e-6
    del out, psi
    ham.free()
    torch.cuda.empty_cache()


def test_transverse_field_only_full_size_closed_form(eng):
    """H(t) = (1 - s) sum (1 - sx_q)/2 from |0...0>: each qubit turns by
    exp(-i A sx) with A = -(1/2) int (1 - s) dt; identity terms give a phase."""
    engine, ctx, torch = eng
    n, T, t1, K = N_FULL, 30.0, 0.3, 60
    inst = I.interpolated(n, I.transverse_terms(n), I.TermList(n), I.linear_path(T))
    ham = engine.Hamiltonian(ctx, inst)
    psi = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    psi[0] = 1.0
    st, _ = engine.evolve(ctx, ham, psi, 0.0, t1, method="pc4", n_steps=K, shift=n / 2.0)
    assert ham.info()["n_passes"][0] >= 3  # the benchmark's multi-pass plan
    F = t1 - t1 * t1 / (2 * T)                    # int_0^t1 (1 - t/T) dt
    A = -0.5 * F
    ph = np.exp(-1j * (n / 2.0) * F)
    rows = _rows(np.random.default_rng(5), n)
    pop = np.array([bin(int(r)).count("1") for r in rows])
    exact = ph * np.cos(A) ** (n - pop) * (-1j * np.sin(A)) ** pop
    got = psi.index_select(0, torch.from_numpy(rows).to("cuda")).cpu().to(torch.complex128).numpy()
    # float32 rounding plus the method's truncation error, t1 C h^4 lam^5 with
    # |lam| <= n/2 after the shift (about 4e-6 of the largest amplitude)
    assert np.max(np.abs(got - exact)) / np.max(np.abs(exact)) < 2e-5
    assert abs(st["norm2_final"] - 1.0) < 1e-5
    del psi
    ham.free()
    torch.cuda.empty_cache()


def test_sk_diagonal_full_size_exact_phases(eng):
    """Diagonal-only H(t) = s(t) H_SK: psi_T(z) = exp(-i E(z) int s dt) psi_0(z)."""
    engine, ctx, torch = eng
    n, T, t1, K = N_FULL, 30.0, 3.0, 60
    J, h = I.sk_couplings(n, np.random.default_rng(I.seed_for(2)))
    inst = I.sk_terms(n, J, h).instance([I.SCHED_S], I.sin2_path(T))
    ham = engine.Hamiltonian(ctx, inst)
    N = 1 << n
    psi = torch.full((N,), 1.0 / math.sqrt(N), dtype=torch.complex64, device="cuda")
    engine.evolve(ctx, ham, psi, 0.0, t1, method="pc4", n_steps=K, shift="center")
    # int_0^t1 sin^2(pi t / 2T) dt = t1/2 - (T/(2 pi)) sin(pi t1 / T)
    S = t1 / 2 - T / (2 * math.pi) * math.sin(math.pi * t1 / T)
    rows = _rows(np.random.default_rng(6), n)
    E = sqh.diagonal_rows(I.sk_terms(n, J, h).instance([I.SCHED_CONST], I.sin2_path(T)), 0.0, rows)
    exact = np.exp(-1j * E * S) / math.sqrt(N)
    got = psi.index_select(0, torch.from_numpy(rows).to("cuda")).cpu().to(torch.complex128).numpy()
    assert np.max(np.abs(got - exact)) * math.sqrt(N) < 2e-5
    del psi
    ham.free()
    torch.cuda.empty_cache()


def _colex_rank(z):
    """Rank of a weight-w basis state among those of its weight in increasing
    order: sum over its set bits p_0 < p_1 < ... of C(p_k, k + 1)."""
    r, k, p = 0, 0, 0
    while z:
        if z & 1:
            r += math.comb(p, k + 1)
            k += 1
        z >>= 1
        p += 1
    return r


def test_sector_apply_sampled_rows_full_size(eng):
    """The Hamming-weight sector of the sector benchmark (n = 30, w = 15,
    C(30, 15) = 155 117 520 states, complex64) on the clause-by-clause XY
    path: sampled rows of H psi against the oracle's row-wise product of the
    expanded state (amplitudes outside the sector are zero)."""
    engine, ctx, torch = eng
    n, w = N_FULL, 15
    inst = I.workload_ec3_paths(n=n, m=24, T=20.0, kind="cbc", seed=I.seed_for(5))
    ham = engine.Hamiltonian(ctx, inst)
    sec = engine.Sector(ctx, ham, w)
    assert sec.dim == math.comb(n, w)
    g = torch.Generator(device="cuda").manual_seed(7)
    psi = torch.randn(sec.dim, dtype=torch.complex64, device="cuda", generator=g)
    out = engine.apply(ctx, sec, 9.5, psi)
    rng = np.random.default_rng(8)
    rows = []
    while len(rows) < 300:                     # random weight-15 states
        rows.append(int(sum(1 << int(q) for q in rng.choice(n, w, replace=False))))
    rows += [(1 << w) - 1, ((1 << w) - 1) << (n - w)]   # the first and the last state
    rows = np.unique(np.array(rows, dtype=np.int64))

    def values_at(idx):
        idx = np.asarray(idx, dtype=np.int64)
        keep = np.array([bin(int(z)).count("1") == w for z in idx])
        vals = np.zeros(idx.shape, dtype=np.complex128)
        if keep.any():
            ranks = torch.tensor([_colex_rank(int(z)) for z in idx[keep]], dtype=torch.int64, device="cuda")
            vals[keep] = psi.index_select(0, ranks).cpu().to(torch.complex128).numpy()
        return vals

    want = sqh.apply_h_rows(inst, 9.5, values_at, rows)
    ranks = torch.tensor([_colex_rank(int(z)) for z in rows], dtype=torch.int64, device="cuda")
    got = out.index_select(0, ranks).cpu().to(torch.complex128).numpy()
    assert np.max(np.abs(got - want)) / np.abs(want).max() < 5e-6
    del out, psi
    sec.free()
    ham.free()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("w", [3, 31, 17])
def test_sector_apply_sampled_rows_max_qubits(eng, w):
    """The largest sectors the library takes: n = 34 (six 6-bit chunks of the
    rank table, states in 64-bit words) on the clause-by-clause XY path with 27 clauses,
    at weights 3 and 31 (the diagonal over the one bits and over the zero
    bits) and 17 (C(34, 17) = 2 333 606 220 states, ranks above 2^31,
    complex64): sampled rows of H psi against the oracle's row-wise product."""
    engine, ctx, torch = eng
    n = 34
    inst = I.workload_ec3_paths(n=n, m=27, T=20.0, kind="cbc", seed=I.seed_for(5))
    ham = engine.Hamiltonian(ctx, inst)
    sec = engine.Sector(ctx, ham, w)
    assert sec.dim == math.comb(n, w)
    g = torch.Generator(device="cuda").manual_seed(11)
    psi = torch.randn(sec.dim, dtype=torch.complex64, device="cuda", generator=g)
    out = engine.apply(ctx, sec, 13.0, psi)
    rng = np.random.default_rng(12)
    rows = []
    while len(rows) < 200:
        rows.append(int(sum(1 << int(q) for q in rng.choice(n, w, replace=False))))
    rows += [(1 << w) - 1, ((1 << w) - 1) << (n - w)]   # the first and the last state
    rows = np.unique(np.array(rows, dtype=np.int64))

    def values_at(idx):
        idx = np.asarray(idx, dtype=np.int64)
        keep = np.array([bin(int(z)).count("1") == w for z in idx])
        vals = np.zeros(idx.shape, dtype=np.complex128)
        if keep.any():
            ranks = torch.tensor([_colex_rank(int(z)) for z in idx[keep]], dtype=torch.int64, device="cuda")
            vals[keep] = psi.index_select(0, ranks).cpu().to(torch.complex128).numpy()
        return vals

    want = sqh.apply_h_rows(inst, 13.0, values_at, rows)
    ranks = torch.tensor([_colex_rank(int(z)) for z in rows], dtype=torch.int64, device="cuda")
    got = out.index_select(0, ranks).cpu().to(torch.complex128).numpy()
    assert np.max(np.abs(got - want)) / np.abs(want).max() < 5e-6
    del out, psi
    sec.free()
    ham.free()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("w", [16, 29])
def test_sector_apply_sampled_rows_word_limit(eng, w):
    """n = 32, the largest size whose states fit the kernel's 32-bit words
    (bit 31 set in half of the states, the last 6-bit chunk two bits wide):
    weight 16 (C(32, 16) = 601 080 390 states) and 29 (the diagonal over the
    zero bits), complex64, sampled rows of H psi against the oracle's
    row-wise product."""
    engine, ctx, torch = eng
    n = 32
    inst = I.workload_ec3_paths(n=n, m=26, T=20.0, kind="cbc", seed=I.seed_for(5))
    ham = engine.Hamiltonian(ctx, inst)
    sec = engine.Sector(ctx, ham, w)
    assert sec.dim == math.comb(n, w)
    g = torch.Generator(device="cuda").manual_seed(13)
    psi = torch.randn(sec.dim, dtype=torch.complex64, device="cuda", generator=g)
    out = engine.apply(ctx, sec, 11.0, psi)
    rng = np.random.default_rng(14)
    rows = []
    while len(rows) < 200:
        rows.append(int(sum(1 << int(q) for q in rng.choice(n, w, replace=False))))
    rows += [(1 << w) - 1, ((1 << w) - 1) << (n - w)]   # the first and the last state
    rows = np.unique(np.array(rows, dtype=np.int64))

    def values_at(idx):
        idx = np.asarray(idx, dtype=np.int64)
        keep = np.array([bin(int(z)).count("1") == w for z in idx])
        vals = np.zeros(idx.shape, dtype=np.complex128)
        if keep.any():
            ranks = torch.tensor([_colex_rank(int(z)) for z in idx[keep]], dtype=torch.int64, device="cuda")
            vals[keep] = psi.index_select(0, ranks).cpu().to(torch.complex128).numpy()
        return vals

    want = sqh.apply_h_rows(inst, 11.0, values_at, rows)
    ranks = torch.tensor([_colex_rank(int(z)) for z in rows], dtype=torch.int64, device="cuda")
    got = out.index_select(0, ranks).cpu().to(torch.complex128).numpy()
    assert np.max(np.abs(got - want)) / np.abs(want).max() < 5e-6
    del out, psi
    sec.free()
    ham.free()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [32, 33])
def test_apply_sampled_rows_past_32bit_indices(eng, n):
    """H psi of the SK workload with amplitude indices past 2^31 (n = 32) and
    past 2^32 (n = 33, 64 GiB per complex64 vector): sampled rows, the first
    and the last amplitude among them, against the oracle's row-wise product."""
    engine, ctx, torch = eng
    inst = I.workload_sk_sin2(n=n, T=30.0, seed=I.seed_for(2))
    ham = engine.Hamiltonian(ctx, inst)
    g = torch.Generator(device="cuda").manual_seed(5)
    psi = torch.randn(1 << n, dtype=torch.complex64, device="cuda", generator=g)
    out = engine.apply(ctx, ham, 17.0, psi)
    rows = _rows(np.random.default_rng(6), n)

    def values_at(idx):
        t = torch.from_numpy(np.ascontiguousarray(idx)).to("cuda")
        return psi.index_select(0, t).cpu().to(torch.complex128).numpy()

    want = sqh.apply_h_rows(inst, 17.0, values_at, rows)
    got = out.index_select(0, torch.from_numpy(rows).to("cuda")).cpu().to(torch.complex128).numpy()
    assert np.max(np.abs(got - want)) / np.abs(want).max() < 5e-6
    del out, psi
    ham.free()
    torch.cuda.empty_cache()
