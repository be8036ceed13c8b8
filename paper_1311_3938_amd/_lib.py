"""ctypes binding of libaqc.so (the C ABI declared in include/aqc.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built."""
import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaqc.so")

AQC_OK, AQC_EINVAL, AQC_ENOMEM, AQC_EDEVICE, AQC_EUNSTABLE, AQC_ENOTSUP, AQC_EBUSY = 0, -1, -2, -3, -4, -5, -6
C64, C128 = 0, 1
SCHED_CONST, SCHED_POLY_S, SCHED_TRIG_T, SCHED_PWL_S = 0, 1, 2, 3
PATH_LINEAR, PATH_SIN2 = 0, 1
METHOD_PC4, METHOD_RK4 = 0, 1
SHIFT_VALUE, SHIFT_CENTER = 0, 1
TARGET_STATE, TARGET_BASIS_LIST = 0, 1
PROF_HIGH_PASS, PROF_LAST_PASS = 0, 1

STATUS_NAMES = {0: "AQC_OK", -1: "AQC_EINVAL", -2: "AQC_ENOMEM", -3: "AQC_EDEVICE",
                -4: "AQC_EUNSTABLE", -5: "AQC_ENOTSUP", -6: "AQC_EBUSY"}


class Sched(C.Structure):
    _fields_ = [("kind", C.c_int32), ("degree", C.c_int32), ("hi_closed", C.c_int32),
                ("reserved", C.c_int32), ("coef", C.c_double * 8), ("s_lo", C.c_double),
                ("s_hi", C.c_double), ("amp", C.c_double), ("omega", C.c_double),
                ("phase", C.c_double)]


class Path(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("T", C.c_double)]


class HamInfo(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_terms", C.c_int32), ("n_diag_terms", C.c_int32),
                ("n_groups", C.c_int32), ("n_passes", C.c_int32 * 2), ("tile_bits", C.c_int32 * 2),
                ("spec_lo", C.c_double), ("spec_hi", C.c_double)]


class Pc4Carry(C.Structure):
    _fields_ = [("valid", C.c_int32), ("sub", C.c_int32), ("ypc", C.c_int32), ("dtype", C.c_int32),
                ("k", C.c_int64), ("t_start", C.c_double), ("h", C.c_double), ("shift", C.c_double),
                ("t_ref", C.c_double), ("ham", C.c_void_p), ("psi", C.c_void_p),
                ("workspace", C.c_void_p), ("phase_re", C.c_double), ("phase_im", C.c_double)]


class EvolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("n_steps", C.c_int32), ("shift_mode", C.c_int32),
                ("check_every", C.c_int32), ("shift", C.c_double), ("norm_tol", C.c_double),
                ("stab_limit", C.c_double), ("atol", C.c_double), ("h0", C.c_double),
                ("hmin", C.c_double), ("hmax", C.c_double), ("window", C.c_int32),
                ("n_replay", C.c_int32), ("replay", C.POINTER(C.c_double)),
                ("record", C.POINTER(C.c_double)), ("record_cap", C.c_int32),
                ("compensated", C.c_int32), ("carry", C.POINTER(Pc4Carry))]


class EvolveStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rejected", C.c_int64), ("matvecs", C.c_int64),
                ("n_segments", C.c_int32), ("status_step", C.c_int32), ("t_reached", C.c_double),
                ("h_last", C.c_double), ("shift_used", C.c_double), ("rho", C.c_double),
                ("norm2_initial", C.c_double), ("norm2_final", C.c_double),
                ("max_err", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AqcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

P = C.c_void_p
D = C.c_double
I32 = C.c_int32
I64 = C.c_int64
SZ = C.c_size_t

SIGNATURES = {
    "aqc_create": (I32, [C.c_int, P, C.POINTER(P)]),
    "aqc_destroy": (I32, [P]),
    "aqc_trim": (I32, [I32]),
    "aqc_set_stream": (I32, [P, P]),
    "aqc_last_error": (C.c_char_p, []),
    "aqc_version": (C.c_char_p, []),
    "aqc_build_hamiltonian": (I32, [P, C.c_int, I64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                    C.POINTER(D), C.POINTER(I32), C.c_int, C.POINTER(Sched),
                                    C.POINTER(Path), C.POINTER(P)]),
    "aqc_ham_free": (I32, [P]),
    "aqc_ham_info": (I32, [P, C.POINTER(HamInfo)]),
    "aqc_ham_set_tiling": (I32, [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "aqc_spectral_bounds": (I32, [P, P, D, D, C.POINTER(D), C.POINTER(D)]),
    "aqc_apply_workspace_bytes": (SZ, [P, C.c_int]),
    "aqc_apply": (I32, [P, P, D, P, P, C.c_int, P, SZ]),
    "aqc_evolve_workspace_bytes": (SZ, [P, C.c_int, C.POINTER(EvolveOpts)]),
    "aqc_evolve": (I32, [P, P, P, C.c_int, D, D, C.POINTER(EvolveOpts), P, SZ,
                         C.POINTER(EvolveStats)]),
    "aqc_norm2": (I32, [P, P, C.c_int, C.c_int, C.POINTER(D)]),
    "aqc_overlap": (I32, [P, P, P, C.c_int, C.c_int, C.POINTER(D), C.POINTER(D)]),
    "aqc_fidelity": (I32, [P, P, C.c_int, C.c_int, C.c_int, P, I64, C.POINTER(D)]),
    "aqc_ground_mass": (I32, [P, P, D, P, C.c_int, D, C.POINTER(D), C.POINTER(D)]),
    "aqc_energy": (I32, [P, P, D, P, C.c_int, P, SZ, C.POINTER(D)]),
    "aqc_energy_noalloc": (I32, [P, P, D, P, C.c_int, C.POINTER(D)]),
    "aqc_batch_create": (I32, [P, C.c_int, C.c_int, C.POINTER(P)]),
    "aqc_batch_destroy": (I32, [P]),
    "aqc_batch_set_graph": (I32, [P, C.c_int]),
    "aqc_batch_set_resident": (I32, [P, C.c_int]),
    "aqc_batch_workspace_bytes": (SZ, [P, C.c_int]),
    "aqc_batch_admit": (I32, [P, P, P, P, SZ, D, D, I64, D, C.POINTER(C.c_int)]),
    "aqc_batch_step": (I32, [P, C.c_int, C.POINTER(C.c_int)]),
    "aqc_batch_poll": (I32, [P, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)]),
    "aqc_batch_retire": (I32, [P, C.c_int, C.POINTER(EvolveStats)]),
    "aqc_batch_info": (I32, [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(I64)]),
    "aqc_norm2_len": (I32, [P, P, C.c_int, I64, C.POINTER(D)]),
    "aqc_overlap_len": (I32, [P, P, P, C.c_int, I64, C.POINTER(D), C.POINTER(D)]),
    "aqc_sector_create": (I32, [P, P, C.c_int, C.POINTER(P)]),
    "aqc_ham_dim": (I64, [P]),
    "aqc_ham_sector_weight": (C.c_int, [P]),
    "aqc_sector_expand": (I32, [P, P, P, P, C.c_int]),
    "aqc_sector_dicke": (I32, [P, P, P, C.c_int]),
    "aqc_lowest_eigs": (I32, [P, P, D, C.c_int, C.c_int, C.c_int, C.c_int, D, P, P, SZ,
                              C.POINTER(D), C.POINTER(D), C.POINTER(C.c_int), P]),
    "aqc_lowest_eigs_workspace_bytes": (SZ, [P, C.c_int, C.c_int]),
    "aqc_hermitian_eigh": (I32, [C.c_int, C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
    "aqc_profile_enable": (I32, [P, C.c_int]),
    "aqc_profile_reset": (I32, [P]),
    "aqc_profile_read": (I32, [P, C.c_int, C.POINTER(D), C.POINTER(I64), C.POINTER(D)]),
}


def lib():
    """The loaded library; raises if libaqc.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1311_3938_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != AQC_OK:
        raise AqcError(status, lib().aqc_last_error().decode(errors="replace"))
    return status


def make_sched(spec):
    s = Sched()
    k = spec["kind"]
    if k == "const":
        s.kind = SCHED_CONST
    elif k == "poly_s":
        s.kind = SCHED_POLY_S
        coef = list(spec["coef"])
        if not 1 <= len(coef) <= 8:
            raise ValueError("poly_s needs 1..8 coefficients")
        s.degree = len(coef) - 1
        for i, c in enumerate(coef):
            s.coef[i] = c
        s.s_lo = spec.get("s_lo", -math.inf)
        s.s_hi = spec.get("s_hi", math.inf)
        s.hi_closed = 1 if spec.get("hi_closed", False) else 0
    elif k == "pwl_s":
        s.kind = SCHED_PWL_S
        knots = [(float(a), float(v)) for a, v in spec["knots"]]
        if not 1 <= len(knots) <= 4:
            raise ValueError("pwl_s needs 1..4 knots")
        s.degree = len(knots) - 1
        for i, (a, v) in enumerate(knots):
            s.coef[2 * i], s.coef[2 * i + 1] = a, v
    elif k == "trig_t":
        s.kind = SCHED_TRIG_T
        s.amp, s.omega, s.phase = spec["amp"], spec["omega"], spec.get("phase", 0.0)
    else:
        raise ValueError(k)
    return s


def make_path(spec):
    p = Path()
    p.kind = {"linear": PATH_LINEAR, "sin2": PATH_SIN2}[spec["kind"]]
    p.T = spec["T"]
    return p
