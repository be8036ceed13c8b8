"""The C-ABI library loads on the host and exports exactly what include/aqc.h
declares; struct layouts agree between C and the ctypes binding (no GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aqc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aqc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1311_3938_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for nm in names:
        assert hasattr(lib, nm), nm
    from paper_1311_3938_amd import _lib
    assert set(_lib.SIGNATURES) == set(names)


def test_struct_layouts_match_c(tmp_path):
    from paper_1311_3938_amd import _lib
    prog = tmp_path / "sz.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "aqc.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(aqc_sched),"
        " sizeof(aqc_path), sizeof(aqc_evolve_opts), sizeof(aqc_evolve_stats), sizeof(aqc_ham_info_t),"
        " offsetof(aqc_evolve_opts, replay), offsetof(aqc_evolve_stats, t_reached),"
        " offsetof(aqc_evolve_opts, carry), sizeof(aqc_pc4_carry), offsetof(aqc_pc4_carry, phase_re));"
        " return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(_lib.Sched), C.sizeof(_lib.Path), C.sizeof(_lib.EvolveOpts),
            C.sizeof(_lib.EvolveStats), C.sizeof(_lib.HamInfo), _lib.EvolveOpts.replay.offset,
            _lib.EvolveStats.t_reached.offset, _lib.EvolveOpts.carry.offset, C.sizeof(_lib.Pc4Carry),
            _lib.Pc4Carry.phase_re.offset]
    assert got == want


def test_argument_errors_without_a_device(lib):
    """Validation happens before any device call: NULL handles and bad sizes
    are rejected with a status and a message."""
    from paper_1311_3938_amd import _lib
    assert lib.aqc_build_hamiltonian(None, 3, 0, None, None, None, None, 1, None, None,
                                     None) == _lib.AQC_EINVAL
    out = C.c_void_p()
    assert lib.aqc_build_hamiltonian(None, 3, 0, None, None, None, None, 1, None, None,
                                     C.byref(out)) == _lib.AQC_EINVAL
    assert b"ctx" in lib.aqc_last_error()
    assert lib.aqc_apply(None, None, 0.0, None, None, 0, None, 0) == _lib.AQC_EINVAL
    assert lib.aqc_evolve_workspace_bytes(None, 0, None) == 0
    d = C.c_double()
    assert lib.aqc_norm2(None, None, 0, 3, C.byref(d)) == _lib.AQC_EINVAL
    assert lib.aqc_norm2_len(None, None, 0, 10, C.byref(d)) == _lib.AQC_EINVAL
    assert lib.aqc_sector_create(None, None, 2, C.byref(out)) == _lib.AQC_EINVAL
    assert lib.aqc_ham_dim(None) == 0 and lib.aqc_ham_sector_weight(None) == -1
    assert lib.aqc_sector_dicke(None, None, None, 0) == _lib.AQC_EINVAL
    assert lib.aqc_version().startswith(b"aqc")


def test_host_hermitian_solver_matches_numpy(lib):
    """The host solver of the projected Lanczos problem (no device needed):
    random Hermitian matrices, a diagonal one with repeated entries and a
    2 x 2 with a complex coupling."""
    import numpy as np
    from paper_1311_3938_amd import engine
    rng = np.random.default_rng(0)
    for n in (1, 2, 5, 17, 48):
        a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        a = a + a.conj().T
        w, z = engine.hermitian_eigh(a)
        assert np.allclose(w, np.linalg.eigvalsh(a), atol=1e-11 * max(1, np.abs(w).max()))
        assert np.allclose(z.conj().T @ z, np.eye(n), atol=1e-12)
        assert np.allclose(a @ z, z * w, atol=1e-10 * max(1, np.abs(w).max()))
    d = np.diag([3.0, 1.0, 1.0, -2.0]).astype(complex)
    assert np.allclose(engine.hermitian_eigh(d)[0], [-2, 1, 1, 3])
    w, _ = engine.hermitian_eigh(np.array([[1.0, 2j], [-2j, 1.0]]))
    assert np.allclose(w, [-1.0, 3.0])
