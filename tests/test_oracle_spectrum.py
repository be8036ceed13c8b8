"""Pins of the spectrum oracle (Sec. IV.B): closed-form spectra of the
transverse field, of H^xy in the one-excitation sector (3m minus the clause
graph's adjacency spectrum) and of H^xyz (ground energy 0 in every sector);
ARPACK agrees with dense diagonalisation."""
import numpy as np
import pytest

from oracle import spectrum
from paper_1311_3938_amd import instances as I
from tests._dense import dense_h


def test_transverse_field_levels():
    """sum_i (1 - sigma^x_i)/2 has the eigenvalues 0, 1, ..., n with
    multiplicities C(n, k): the lowest two are 0 and 1."""
    n = 9
    inst = I.transverse_terms(n).instance([I.SCHED_CONST], I.linear_path(1.0))
    assert np.allclose(spectrum.lowest(inst, 0.0, 3), [0.0, 1.0, 1.0], atol=1e-10)
    assert spectrum.gap(inst, 0.0) == pytest.approx(1.0, abs=1e-10)


def test_xy_one_excitation_sector_spectrum():
    n = 10
    clauses = I.ec3_random_clauses(n, 8, np.random.default_rng(4))
    inst = I.xy_initial_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    A = np.zeros((n, n))
    for (i, j), c in I.clause_pair_counts(clauses).items():
        A[i - 1, j - 1] = A[j - 1, i - 1] = c
    want = np.sort(3 * len(clauses) - np.linalg.eigvalsh(A))[:2]
    assert np.allclose(spectrum.lowest(inst, 0.0, 2, weight=1), want, atol=1e-10)


def test_xyz_ground_energy_zero_in_every_sector():
    n = 8
    clauses = I.ec3_random_clauses(n, 6, np.random.default_rng(6))
    inst = I.xyz_initial_terms(n, clauses).instance([I.SCHED_CONST], I.linear_path(1.0))
    for w in (1, 3, 4):
        assert spectrum.lowest(inst, 0.0, 1, weight=w)[0] == pytest.approx(0.0, abs=1e-10)


@pytest.mark.parametrize("kind", ["linear", "cbc"])
def test_arpack_matches_dense(kind):
    """Inside the path (s < 1, hops present); at s = 1 the EC3 levels are
    degenerate and the dense route is the reference."""
    inst = I.workload_ec3_paths(n=8, m=6, T=1.0, kind=kind, seed=3)
    for s in (0.0, 0.4, 0.77, 1.0):
        d = np.linalg.eigvalsh(dense_h(inst, s))[:2]
        assert np.allclose(spectrum.lowest_dense(inst, s, 2), d, atol=1e-12)
        assert np.allclose(spectrum.lowest(inst, s, 2), d, atol=1e-12)
        if s < 1.0:
            assert np.allclose(spectrum.lowest(inst, s, 2, dense_max=0), d, atol=1e-9)
    # the sector block: eigenvalues of the weight-3 rows and columns
    b = [z for z in range(256) if bin(z).count("1") == 3]
    Hb = dense_h(inst, 0.4)[np.ix_(b, b)]
    assert np.allclose(spectrum.lowest(inst, 0.4, 2, weight=3, dense_max=0), np.linalg.eigvalsh(Hb)[:2],
                       atol=1e-9)
