"""GPU: the lowest eigenvalues of H(t) (aqc_lowest_eigs, thick-restart
Lanczos) against the oracle's dense and ARPACK spectra, in the full space
(one and several tiles) and in a Hamming-weight sector, with closed-form
levels of the transverse field; gap curves along the paths of Sec. IV.A."""
import numpy as np
import pytest

from oracle import spectrum, subspace
from paper_1311_3938_amd import instances as I
from tests._gpu import to_dev

pytestmark = pytest.mark.gpu

TOL_E = {"c128": 1e-9, "c64": 1e-6}     # on |dE| / max(1, |E|)
LZ_TOL = {"c128": 1e-10, "c64": 1e-5}


@pytest.fixture(scope="module")
def eng():
    from paper_1311_3938_amd import engine
    ctx = engine.Context(0)
    yield engine, ctx
    ctx.close()


def _dt(name):
    import torch
    return torch.complex128 if name == "c128" else torch.complex64


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind", ["linear", "cbc"])
def test_lowest_two_full_space_small(eng, kind, dt):
    engine, ctx = eng
    inst = I.workload_ec3_paths(n=10, m=8, T=1.0, kind=kind, seed=I.seed_for(5, 4))
    ham = engine.Hamiltonian(ctx, inst)
    import torch
    for s in (0.1, 0.5, 0.85):
        g = torch.empty(1 << 10, dtype=_dt(dt), device="cuda")
        ev, res, nmv = engine.lowest_eigs(ctx, ham, s, k=2, dtype=_dt(dt), tol=LZ_TOL[dt], ground=g)
        ref = spectrum.lowest(inst, s, 2)
        print(f"lanczos {kind} {dt} s={s}: rel err {np.max(np.abs(ev - ref) / np.maximum(1.0, np.abs(ref))):.2e}",
              flush=True)
        assert np.all(np.abs(ev - ref) <= TOL_E[dt] * np.maximum(1.0, np.abs(ref))), (s, ev, ref)
        assert nmv > 0
        # the returned vector is a normalised eigenvector of the oracle's H(s)
        gh = g.cpu().to(torch.complex128).numpy()
        from oracle import sqh
        assert abs(np.linalg.norm(gh) - 1.0) < 10 * TOL_E[dt]
        assert np.linalg.norm(sqh.apply_h(inst, s, gh) - ref[0] * gh) < 1e3 * TOL_E[dt] * max(1, abs(ref[0]))
    ham.free()


def test_lowest_three_several_tiles_arpack(eng):
    """16 qubits: transverse field plus random ZZ/Z (several tiles and
    register passes) against ARPACK."""
    engine, ctx = eng
    n = 16
    rng = np.random.default_rng(12)
    J, h = I.sk_couplings(n, rng)
    inst = I.interpolated(n, I.transverse_terms(n), I.sk_terms(n, J, h), I.linear_path(1.0))
    ham = engine.Hamiltonian(ctx, inst)
    ev, res, nmv = engine.lowest_eigs(ctx, ham, 0.6, k=3, tol=1e-10)
    ref = spectrum.lowest(inst, 0.6, 3)
    assert np.allclose(ev, ref, atol=1e-9, rtol=0), (ev, ref)
    ham.free()


def test_transverse_field_closed_form(eng):
    """sum_i (1 - sigma^x_i)/2 at 20 qubits: levels 0 and 1 (the second has
    multiplicity 20 and is reported once)."""
    engine, ctx = eng
    n = 20
    inst = I.transverse_terms(n).instance([I.SCHED_CONST], I.linear_path(1.0))
    ham = engine.Hamiltonian(ctx, inst)
    ev, res, nmv = engine.lowest_eigs(ctx, ham, 0.0, k=2, tol=1e-11)
    assert np.allclose(ev, [0.0, 1.0], atol=1e-10)
    ham.free()


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_lowest_two_in_a_sector(eng, dt):
    """A hard instance (connected clause graph, unique solution) in the
    sector of its solution's weight, where the two lowest levels are apart.
    (Random clause sets may leave bits unused; those split a sector into
    copies with equal levels, which one Krylov sequence reports once.)"""
    engine, ctx = eng
    n = 16
    inst = I.workload_usa(n, 0, "xy")
    w = inst.meta["weight"]
    ham = engine.Hamiltonian(ctx, inst)
    sec = engine.Sector(ctx, ham, w)
    for s in (0.3, 0.7):
        ev, res, nmv = engine.lowest_eigs(ctx, sec, s, k=2, dtype=_dt(dt), tol=LZ_TOL[dt])
        ref = spectrum.lowest(inst, s, 2, weight=w)
        assert ref[1] - ref[0] > 1e-3
        print(f"lanczos sector {dt} s={s}: rel err {np.max(np.abs(ev - ref) / np.maximum(1.0, np.abs(ref))):.2e}",
              flush=True)
        assert np.all(np.abs(ev - ref) <= TOL_E[dt] * np.maximum(1.0, np.abs(ref))), (s, ev, ref)
    # the Dicke state as the start vector gives the same levels
    ev2, _, _ = engine.lowest_eigs(ctx, sec, 0.7, k=2, dtype=_dt(dt), tol=LZ_TOL[dt],
                                   start=sec.dicke(_dt(dt)))
    assert np.all(np.abs(ev2 - ref) <= TOL_E[dt] * np.maximum(1.0, np.abs(ref)))
    sec.free()
    ham.free()


def test_xyz_sector_ground_energy_zero(eng):
    engine, ctx = eng
    # a connected clause graph: the Dicke state is the only ground state of
    # H^xyz (s = 0) in each sector
    n, w = 14, 5
    inst = I.workload_usa(n, 1, "xyz")
    ham = engine.Hamiltonian(ctx, inst)
    sec = engine.Sector(ctx, ham, w)
    ev, _, _ = engine.lowest_eigs(ctx, sec, 0.0, k=2, tol=1e-11)
    assert abs(ev[0]) < 1e-10
    assert ev[1] == pytest.approx(spectrum.lowest(inst, 0.0, 2, weight=w)[1], abs=1e-9)
    sec.free()
    ham.free()


def test_not_converged_is_reported(eng):
    engine, ctx = eng
    from paper_1311_3938_amd import _lib as L
    inst = I.workload_ec3_paths(n=12, m=9, T=1.0, kind="linear", seed=I.seed_for(5, 6))
    ham = engine.Hamiltonian(ctx, inst)
    with pytest.raises(L.AqcError) as ei:
        engine.lowest_eigs(ctx, ham, 0.5, k=2, max_basis=6, max_matvecs=6, tol=1e-14)
    assert ei.value.status == L.AQC_EUNSTABLE
    with pytest.raises(ValueError):
        engine.lowest_eigs(ctx, ham, 0.5, k=2, max_basis=60)
    ham.free()


@pytest.mark.parametrize("n,m,seed", [(3, 8, 40), (4, 16, 42), (4, 12, 42)])
def test_krylov_space_as_large_as_the_state(eng, n, m, seed):
    """A basis as large as the state (n = 3 with 8 vectors, n = 4 with 16) or
    nearly so (n = 4, 12 of 16): the Krylov space can exhaust the whole space;
    the two lowest levels of a random Hamiltonian (seeds whose levels are all
    at least 0.05 apart: a Krylov space holds one vector of a degenerate
    level) still match the oracle's dense spectrum."""
    engine, ctx = eng
    inst = I.random_terms(n, 10, np.random.default_rng(seed)).instance([I.SCHED_CONST], I.linear_path(1.0))
    ham = engine.Hamiltonian(ctx, inst)
    ev, res, nmv = engine.lowest_eigs(ctx, ham, 0.0, k=2, max_basis=m, tol=1e-10)
    ref = spectrum.lowest_dense(inst, 0.0, 2)
    assert np.all(np.abs(ev - ref) <= 1e-9 * np.maximum(1.0, np.abs(ref))), (ev, ref)
    ham.free()
